#!/usr/bin/env python3
"""Apply throughput of the multidimensional butterfly factorization on one GPU.

One step = one mbf_apply of the whole factorization (leaf projection, every
stage block product, middle scaling, leaf reconstruction) to one batch of
nrhs right-hand sides that are already resident in HBM.  Prints one JSON
line (see the repository contract): RHS/s, the roofline of the dominant
kernel (the stage block product) measured with HIP events over the timed
steps, the relative error against an FP64 reference, and the CPU oracle's
direct summation timed on a bounded sample of rows.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--config NAME] [--prec c64|bf16x3]
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MBF apply RHS/s and % roofline at N=512²; rel err vs FP64; p50/p99 latency"

# Workloads: (kernel, grid side n, tolerance, leaf side, right-hand sides)
CONFIGS = {
    "dft512": dict(kernel="dft", n=512, tol=1e-6, leaf=4, nrhs=256, split="none"),
    "dft256": dict(kernel="dft", n=256, tol=1e-6, leaf=4, nrhs=256, split="none"),
    "dft128": dict(kernel="dft", n=128, tol=1e-6, leaf=4, nrhs=256, split="none"),
    "dft64": dict(kernel="dft", n=64, tol=1e-8, leaf=8, nrhs=1, split="none"),
}
DEFAULT_CONFIG = os.environ.get("MBF_BENCH_CONFIG", "dft128")

PEAK = {  # MI355X published dense peaks
    "c64": ("mfma", 157.3, "TFLOP/s"),     # FP32
    "bf16x3": ("mfma", 2500.0, "TFLOP/s"),  # BF16 matrix cores
    "c128": ("mfma", 78.6, "TFLOP/s"),     # FP64
    "hbm": 8000.0,                          # GB/s
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default=DEFAULT_CONFIG, choices=sorted(CONFIGS))
    ap.add_argument("--prec", default="c64", choices=["c64", "bf16x3", "c128"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-check", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: multi-GPU runs are not part of this build "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import mbf_workloads as W
    import paper_1509_07925_amd as mbf

    cfg = CONFIGS[args.config]
    n, nrhs = cfg["n"], cfg["nrhs"]
    N = n * n
    dev = torch.device("cuda:0")
    if cfg["kernel"] == "dft":
        x, xi = W.grid_x_integer(n), W.grid_omega(n)
    else:
        x, xi = W.grid_x_unit(n), W.grid_omega(n)
    precs = [args.prec] + ([] if args.no_fp64_check or args.prec == "c128" else ["c128"])
    log("[bench] building %s (n=%d tol=%g leaf=%d) precs=%s" % (args.config, n, cfg["tol"], cfg["leaf"], precs))
    t0 = time.time()
    F = mbf.Factor.build(x, xi, n, kernel=cfg["kernel"], tol=cfg["tol"], leaf_side=cfg["leaf"],
                         split=cfg["split"], precs=precs, max_rank=4096)
    build_s = time.time() - t0
    inf = F.info()
    log("[bench] build %.1fs nnz=%.3e depth=%d ranks=%s device GB=%.2f" % (
        build_s, inf.nnz, inf.depth, list(inf.max_rank[:inf.depth + 1]), inf.device_bytes / 1e9))

    g_host = W.rhs(N, nrhs, seed=0)
    vdt = torch.complex128 if args.prec == "c128" else torch.complex64
    g = torch.from_numpy(np.ascontiguousarray(g_host.T)).to(dev, vdt).t()
    u = torch.empty((nrhs, N), dtype=vdt, device=dev).t()
    ws = torch.empty(F.workspace_size(args.prec, nrhs), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        F.apply(g, out=u, prec=args.prec, workspace=ws)
    torch.cuda.synchronize()
    nl = 4 + 2 * inf.depth if inf.depth else 256
    F.profile_begin(args.steps * nl + 16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        F.apply(g, out=u, prec=args.prec, workspace=ws, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    recs = F.profile_end()
    total_s = t1 - t0
    ms_per_step = 1e3 * total_s / args.steps
    value = nrhs * args.steps / total_s

    stage = [r for r in recs if r["kind"] == 1]
    st_ms = sum(r["ms"] for r in stage)
    st_flops = sum(r["flops"] for r in stage)
    st_bytes = sum(r["bytes"] for r in stage)
    n_launch = len(stage)
    bound, peak, unit = PEAK[args.prec]
    exec_mult = 3.0 if args.prec == "bf16x3" else 1.0  # hi*hi + hi*lo + lo*hi
    achieved = exec_mult * st_flops / (st_ms * 1e-3) / 1e12 if st_ms > 0 else 0.0
    roofline = {"bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
                "frac": round(achieved / peak, 4), "traffic": None,
                "kernel": "stage block product", "launches": n_launch,
                "avg_launch_ms": round(st_ms / max(n_launch, 1), 4),
                "alg_flops_per_step": st_flops / args.steps,
                "alg_bytes_per_step": st_bytes / args.steps,
                "hbm_gbps_alg": round(st_bytes / (st_ms * 1e-3) / 1e9, 1) if st_ms > 0 else 0.0,
                "kernel_share_of_step": round(st_ms / (sum(r["ms"] for r in recs) or 1.0), 4)}

    out = {"metric": METRIC, "value": round(value, 2), "unit": "RHS/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None,
           "dtype": {"c64": "f32", "bf16x3": "bf16x3-f32acc", "c128": "f64"}[args.prec],
           "data": "synthetic",
           "config": {"workload": "dft2d_n%d_tol%g_leaf%dx%d_rhs%d" % (n, cfg["tol"], cfg["leaf"], cfg["leaf"], nrhs),
                      "kernel": cfg["kernel"], "n": n, "N": N, "nrhs": nrhs, "tol": cfg["tol"],
                      "depth": inf.depth, "ranks": list(inf.max_rank[:inf.depth + 1]), "nnz": inf.nnz,
                      "factor_gb": round(inf.device_bytes / 1e9, 3), "build_s": round(build_s, 1),
                      "prec": args.prec},
           "roofline": roofline}

    # Arithmetic error: same factors, FP64 instantiation on the GPU.
    u_np = None
    if "c128" in precs and args.prec != "c128":
        g64 = torch.from_numpy(np.ascontiguousarray(g_host.T)).to(dev, torch.complex128).t()
        u64 = F.apply(g64, prec="c128")
        torch.cuda.synchronize()
        d = (u.to(torch.complex128) - u64).abs().pow(2).sum().sqrt() / u64.abs().pow(2).sum().sqrt()
        out["rel_err_vs_fp64_apply"] = float(d)
        del g64, u64
    u_np = u.t().contiguous().cpu().numpy().astype(np.complex128).T

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, x, xi, g_host, u_np, out)
    print(json.dumps(out), flush=True)


def cpu_baseline(cfg, x, xi, g, u_gpu, out):
    """Oracle leg: direct FP64 summation (eq. (kernel)) on sampled rows."""
    import numpy as np
    import threadpoolctl

    import mbf_workloads as W
    from oracle import direct, kernels

    n, nrhs = cfg["n"], g.shape[1]
    N = n * n
    K = kernels.dft(n) if cfg["kernel"] == "dft" else kernels.fio_radon(n)
    # bounded sample: about 10-30 s of host work at n = 512
    nrows = max(64, min(N, int(4096 * (256.0 / n) ** 2)))
    rows = W.sample_rows(N, nrows, seed=1)
    info = threadpoolctl.threadpool_info()
    cores = max([i.get("num_threads", 1) for i in info] + [1])
    t0 = time.perf_counter()
    ref = direct.direct_rows(K, x, xi, g, rows, block=256)
    dt = time.perf_counter() - t0
    rhs_per_s = nrhs / (dt * N / nrows)
    out["rel_err_vs_direct_sampled_rows"] = direct.rel_err(u_gpu[rows], ref)
    return {"value": round(rhs_per_s, 6), "unit": "RHS/s", "cores": int(cores), "kind": "oracle",
            "sample": "direct FP64 sum of eq. (kernel) on %d of %d rows x %d RHS in %.2f s, "
                      "scaled to the full N" % (nrows, N, nrhs, dt)}


if __name__ == "__main__":
    main()
