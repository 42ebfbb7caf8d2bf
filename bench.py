#!/usr/bin/env python3
"""Apply throughput of the multidimensional butterfly factorization on one GPU.

One step = one mbf_apply of the whole factorization (leaf projection, every
stage block product, middle scaling, leaf reconstruction) to one batch of
nrhs right-hand sides that are already resident in HBM.  Prints one JSON
line: RHS/s of the plain FP32 apply, the roofline of the dominant kernel
(the stage block product) measured with HIP events over the timed steps,
the relative errors against the FP64 apply of the same factors and against
the direct sum on sampled rows, the split-BF16 apply on the same factors,
a short served request mix (p50 / p99 latency), and the CPU oracle's direct
summation timed on a bounded sample of rows.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--config NAME]
                       [--save PATH | --load PATH] [--no-cpu-baseline] ...
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
    # FIO of Example 1 with the polar split (Section 3.2), 64 RHS
    "fio128polar": dict(kernel="fio", n=128, tol=1e-6, leaf=4, nrhs=64, split="polar"),
    # FIO with the multiscale split (Section 4.2), 16 RHS, apply and adjoint; the
    # 1024^2 case keeps only the FP32 factors resident
    "fio256ms": dict(kernel="fio", n=256, tol=1e-4, leaf=4, nrhs=16, split="multiscale", adjoint=True),
    "fio1024ms": dict(kernel="fio", n=1024, tol=1e-4, leaf=4, nrhs=16, split="multiscale", adjoint=True,
                      fp32_only=True),
}
DEFAULT_CONFIG = os.environ.get("MBF_BENCH_CONFIG", "dft512")

PEAK = {  # MI355X published dense peaks (TFLOP/s)
    "c64": ("mfma", 157.3),     # FP32 matrix
    "bf16x3": ("mfma", 2500.0),  # BF16 matrix
    "c128": ("mfma", 78.6),     # FP64
}


def workload_name(cfg):
    if cfg["kernel"] == "dft" and cfg["split"] == "none":
        return "dft2d_n%d_tol%g_leaf%dx%d_rhs%d" % (cfg["n"], cfg["tol"], cfg["leaf"], cfg["leaf"], cfg["nrhs"])
    return "%s2d_n%d_%s_tol%g_leaf%dx%d_rhs%d" % (cfg["kernel"], cfg["n"], cfg["split"], cfg["tol"], cfg["leaf"],
                                                 cfg["leaf"], cfg["nrhs"])


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def timed_apply(F, g, u, ws, prec, steps, warmup, adjoint=False):
    """Warmup, then `steps` timed applies (or adjoint applies) bracketed by
    device synchronisation."""
    import torch
    fn = F.apply_adjoint if adjoint else F.apply
    for _ in range(warmup):
        fn(g, out=u, prec=prec, workspace=ws)
    torch.cuda.synchronize()
    inf = F.info()
    F.profile_begin(steps * (4 + 2 * max(inf.depth, 8)) + 64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn(g, out=u, prec=prec, workspace=ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return t1 - t0, F.profile_end()


def roofline(recs, steps, prec):
    stage = [r for r in recs if r["kind"] == 1]
    st_ms = sum(r["ms"] for r in stage)
    st_flops = sum(r["flops"] for r in stage)
    st_bytes = sum(r["bytes"] for r in stage)
    bound, peak = PEAK[prec]
    mult = 3.0 if prec == "bf16x3" else 1.0  # hi*hi + hi*lo + lo*hi executed
    achieved = mult * st_flops / (st_ms * 1e-3) / 1e12 if st_ms > 0 else 0.0
    return {"bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4), "traffic": None,
            "kernel": "stage block product", "launches": len(stage),
            "avg_launch_ms": round(st_ms / max(len(stage), 1), 4),
            "alg_flops_per_launch_avg": st_flops / max(len(stage), 1),
            "alg_flops_per_step": st_flops / steps, "executed_flops_factor": mult,
            "alg_bytes_per_step": st_bytes / steps,
            "alg_hbm_gbps": round(st_bytes / (st_ms * 1e-3) / 1e9, 1) if st_ms > 0 else 0.0,
            "kernel_share_of_step": round(st_ms / (sum(r["ms"] for r in recs) or 1.0), 4)}


def breakdown(recs, steps):
    """Milliseconds per step by launch kind (HIP events)."""
    names = {0: "leaf_project", 1: "stages", 2: "leaf_reconstruct", 3: "center"}
    out = {}
    for r in recs:
        k = names.get(r["kind"], str(r["kind"]))
        out[k] = out.get(k, 0.0) + r["ms"] / steps
    return {k: round(v, 4) for k, v in out.items()}


def hbm_roofline(recs):
    """Stage launches measured against HBM bandwidth (few right-hand sides)."""
    stage = [r for r in recs if r["kind"] == 1]
    st_ms = sum(r["ms"] for r in stage)
    st_bytes = sum(r["bytes"] for r in stage)
    achieved = st_bytes / (st_ms * 1e-3) / 1e9 if st_ms > 0 else 0.0
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": 8000.0, "unit": "GB/s",
            "frac": round(achieved / 8000.0, 4), "traffic": None, "kernel": "stage block product (16 x 16 tile, few RHS)",
            "launches": len(stage), "avg_launch_ms": round(st_ms / max(len(stage), 1), 4),
            "alg_bytes_per_launch_avg": st_bytes / max(len(stage), 1),
            "kernel_share_of_step": round(st_ms / (sum(r["ms"] for r in recs) or 1.0), 4)}


def measured_traffic(workload, prec):
    """HBM bytes per stage launch from the committed rocprofv3 counter runs
    (profiles/hbm_traffic_*.json), or None when those counters were taken
    on another workload / precision or before the stage kernel last changed."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_1509_07925_amd", "csrc", "stage_mfma.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    for path in glob.glob(os.path.join(ROOT, "profiles", "hbm_traffic_*.json")):
        rec = json.load(open(path))
        if rec.get("workload") == workload and rec.get("prec") == prec and rec.get("kernel_source_sha256_16") == sha:
            return rec["traffic_bytes_per_launch"]
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default=DEFAULT_CONFIG, choices=sorted(CONFIGS))
    ap.add_argument("--save", default=None, help="save the built factors to this file")
    ap.add_argument("--save-precs", default="c64,bf16x3", help="precisions written by --save")
    ap.add_argument("--load", default=None, help="load factors saved with --save instead of building")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-check", action="store_true")
    ap.add_argument("--no-split", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run one 1 GiB device-to-device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": a.numel() * 4}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU; multi-GPU runs are not implemented "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    # Long builds report progress on stderr (at most every 10 s).
    os.environ.setdefault("MBF_VERBOSE", "1")
    import numpy as np
    import torch

    import mbf_workloads as W
    import paper_1509_07925_amd as mbf

    cfg = CONFIGS[args.config]
    n, nrhs = cfg["n"], cfg["nrhs"]
    N = n * n
    dev = torch.device("cuda:0")
    x, xi = (W.grid_x_integer(n), W.grid_omega(n)) if cfg["kernel"] == "dft" else (W.grid_x_unit(n), W.grid_omega(n))
    if cfg.get("fp32_only"):
        args.no_split = args.no_fp64_check = True
    precs = ["c64"] + ([] if args.no_split else ["bf16x3"])
    t0 = time.time()
    if args.load:
        log("loading", args.load)
        F = mbf.Factor.load(args.load, precs=precs)
        built = False
    else:
        all_precs = precs + ([] if args.no_fp64_check else ["c128"])
        log("building %s (n=%d tol=%g leaf=%d) precs=%s" % (args.config, n, cfg["tol"], cfg["leaf"], all_precs))
        F = mbf.Factor.build(x, xi, n, kernel=cfg["kernel"], tol=cfg["tol"], leaf_side=cfg["leaf"],
                             split=cfg["split"], precs=all_precs, max_rank=4096)
        built = True
    setup_s = time.time() - t0
    inf = F.info()
    log("setup %.1fs nnz=%.3e depth=%d ranks=%s device GB=%.2f" % (
        setup_s, inf.nnz, inf.depth, list(inf.max_rank[:inf.depth + 1]), inf.device_bytes / 1e9))
    if args.save and built:
        t1 = time.time()
        F.save(args.save, precs=[p for p in args.save_precs.split(",") if p])
        log("saved %s in %.1fs" % (args.save, time.time() - t1))

    g_host = W.rhs(N, nrhs, seed=0)
    g = torch.from_numpy(np.ascontiguousarray(g_host.T)).to(dev, torch.complex64).t()
    u = torch.empty((nrhs, N), dtype=torch.complex64, device=dev).t()
    ws = torch.empty(max(F.workspace_size("c64", nrhs), F.workspace_size("bf16x3", nrhs) if "bf16x3" in precs else 0),
                     dtype=torch.uint8, device=dev)

    t1 = time.time()
    tuned = F.autotune("c64", nrhs, workspace=ws)
    if "bf16x3" in precs:
        tuned += F.autotune("bf16x3", nrhs, workspace=ws)
    log("autotuned %d stage shapes in %.1fs" % (tuned, time.time() - t1))
    total_s, recs = timed_apply(F, g, u, ws, "c64", args.steps, args.warmup)
    ms_per_step = 1e3 * total_s / args.steps
    value = nrhs * args.steps / total_s
    log("FP32: %.1f RHS/s (%.3f ms/step)" % (value, ms_per_step))

    out = {"metric": METRIC, "value": round(value, 2), "unit": "RHS/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": workload_name(cfg),
                      "kernel": cfg["kernel"], "split": cfg["split"], "n": n, "N": N, "nrhs": nrhs, "tol": cfg["tol"],
                      "depth": inf.depth, "ranks": list(inf.max_rank[:inf.depth + 1]), "nnz": inf.nnz,
                      "factor_gb_on_device": round(inf.device_bytes / 1e9, 3),
                      "setup_s": round(setup_s, 1), "setup": "load" if args.load else "mbf_build (host FP64)"},
           "roofline": roofline(recs, args.steps, "c64") if nrhs > 32 else hbm_roofline(recs)}
    out["roofline"]["traffic"] = measured_traffic(out["config"]["workload"], "c64")
    out["ms_per_step_by_kind"] = breakdown(recs, args.steps)

    u32 = u.clone()
    if cfg.get("adjoint"):
        h = torch.empty((nrhs, N), dtype=torch.complex64, device=dev).t()
        h.copy_(g)
        v = torch.empty((nrhs, N), dtype=torch.complex64, device=dev).t()
        a_total, a_recs = timed_apply(F, h, v, ws, "c64", args.steps, args.warmup, adjoint=True)
        out["adjoint"] = {"value": round(nrhs * args.steps / a_total, 2), "unit": "RHS/s",
                          "ms_per_step": round(1e3 * a_total / args.steps, 4),
                          "roofline": roofline(a_recs, args.steps, "c64") if nrhs > 32 else hbm_roofline(a_recs),
                          "ms_per_step_by_kind": breakdown(a_recs, args.steps)}
        log("FP32 adjoint: %.1f RHS/s" % out["adjoint"]["value"])
        del h, v
    # few right-hand sides: the 16 x 16 matrix-core stage kernel, bound by reading the blocks from HBM
    nn = 16
    if nrhs > nn:
        g_n, u_n = g[:, :nn], torch.empty((nn, N), dtype=torch.complex64, device=dev).t()
        n_total, n_recs = timed_apply(F, g_n, u_n, ws, "c64", args.steps, args.warmup)
        out["narrow_rhs16"] = {"value": round(nn * args.steps / n_total, 2), "unit": "RHS/s",
                               "ms_per_step": round(1e3 * n_total / args.steps, 4), "nrhs": nn,
                               "roofline": hbm_roofline(n_recs)}
        log("FP32 at %d RHS: %.1f RHS/s" % (nn, out["narrow_rhs16"]["value"]))

    # host-resident inputs and outputs: pinned buffers, copies on the same stream (context, not `value`)
    g_h = torch.empty((nrhs, N), dtype=torch.complex64, pin_memory=True)
    u_h = torch.empty((nrhs, N), dtype=torch.complex64, pin_memory=True)
    g_h.copy_(g.t())
    g_d = torch.empty((nrhs, N), dtype=torch.complex64, device=dev)
    u_d = torch.empty((nrhs, N), dtype=torch.complex64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pcie_steps = max(2, args.steps // 2)
    for _ in range(pcie_steps):
        g_d.copy_(g_h, non_blocking=True)
        F.apply(g_d.t(), out=u_d.t(), prec="c64", workspace=ws)
        u_h.copy_(u_d, non_blocking=True)
    torch.cuda.synchronize()
    t_p = time.perf_counter() - t0
    out["pcie_inclusive"] = {"value": round(nrhs * pcie_steps / t_p, 2), "unit": "RHS/s",
                             "ms_per_step": round(1e3 * t_p / pcie_steps, 4),
                             "note": "g copied host->device and u device->host (pinned) around each apply"}
    log("FP32 with host transfers: %.1f RHS/s" % out["pcie_inclusive"]["value"])
    del g_h, u_h, g_d, u_d

    if not args.no_split:
        u16 = torch.empty_like(u)
        s_total, s_recs = timed_apply(F, g, u16, ws, "bf16x3", args.steps, args.warmup)
        sval = nrhs * args.steps / s_total
        d = (u16.to(torch.complex128) - u32.to(torch.complex128)).abs().pow(2).sum().sqrt() / \
            u32.to(torch.complex128).abs().pow(2).sum().sqrt()
        out["split_bf16x3"] = {"value": round(sval, 2), "unit": "RHS/s", "ms_per_step": round(1e3 * s_total / args.steps, 4),
                               "dtype": "bf16 hi/lo x3, f32 accumulate", "roofline": roofline(s_recs, args.steps, "bf16x3"),
                               "rel_diff_vs_fp32_apply": float(d)}
        log("BF16x3: %.1f RHS/s" % sval)
        del u16

    if built and not args.no_fp64_check:
        g64 = torch.from_numpy(np.ascontiguousarray(g_host.T)).to(dev, torch.complex128).t()
        u64 = F.apply(g64, prec="c128")
        torch.cuda.synchronize()
        nrm = u64.abs().pow(2).sum().sqrt()
        out["rel_err_vs_fp64_apply"] = float((u32.to(torch.complex128) - u64).abs().pow(2).sum().sqrt() / nrm)
        if "narrow_rhs16" in out:
            u64n = u64[:, :nn]
            out["narrow_rhs16"]["rel_err_vs_fp64_apply"] = float(
                (u_n.to(torch.complex128) - u64n).abs().pow(2).sum().sqrt() / u64n.abs().pow(2).sum().sqrt())
        if "split_bf16x3" in out:
            u16 = F.apply(g, prec="bf16x3")
            torch.cuda.synchronize()
            out["split_bf16x3"]["rel_err_vs_fp64_apply"] = float(
                (u16.to(torch.complex128) - u64).abs().pow(2).sum().sqrt() / nrm)
            del u16
        del g64, u64
        torch.cuda.empty_cache()

    if not args.no_serve:
        out["serving"] = serve_mix(F, N, dev)
        out["serving_multi"] = serve_multi(args.config, F, N, dev)
        log("served: p50 %.1f ms p99 %.1f ms; %d factorizations: p50 %.1f ms p99 %.1f ms" % (
            out["serving"]["p50_ms"], out["serving"]["p99_ms"], out["serving_multi"]["factorizations"],
            out["serving_multi"]["p50_ms"], out["serving_multi"]["p99_ms"]))

    u_np = u32.t().contiguous().cpu().numpy().astype(np.complex128).T
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, x, xi, g_host, u_np, out)
    print(json.dumps(out), flush=True)


def serve_mix(F, N, dev, nreq=400, seed=0):
    """Poisson stream of requests with 1..32 RHS on the resident factorization:
    continuous batching through mbf_server; offered load ~80% of the measured
    batched throughput."""
    import numpy as np
    import torch

    import mbf_workloads as W
    import paper_1509_07925_amd as mbf

    rng = np.random.default_rng(seed)
    sizes = rng.integers(1, 33, size=nreq)
    pool = torch.randn((64, N), dtype=torch.complex64, device=dev)  # request inputs drawn from here
    outs = [torch.empty((int(k), N), dtype=torch.complex64, device=dev).t() for k in sizes]
    ins = [pool[: int(k)].t() for k in sizes]
    # offered load from a solo 32-RHS apply
    t0 = time.perf_counter()
    for _ in range(3):
        F.apply(ins[0] if sizes[0] == 32 else pool[:32].t())
    torch.cuda.synchronize()
    per_rhs = (time.perf_counter() - t0) / (3 * 32)
    rate = 0.8 / (per_rhs * float(np.mean(sizes)))
    arrivals = W.poisson_arrivals(nreq, rate, seed=seed)
    srv = mbf.Server(mem_budget=24 << 30, nslots=4, max_batch_rhs=256)
    t_start = time.perf_counter()
    for i in range(nreq):
        while time.perf_counter() - t_start < arrivals[i]:
            pass
        srv.submit(F, ins[i], outs[i])
    srv.drain()
    st = srv.stats()
    srv.close()
    return {"requests": int(st["requests"]), "rhs": int(st["rhs"]), "batches": int(st["batches"]),
            "p50_ms": round(st["p50_us"] / 1e3, 3), "p99_ms": round(st["p99_us"] / 1e3, 3),
            "rhs_per_s": round(st["rhs"] / st["wall_s"], 1) if st["wall_s"] > 0 else None,
            "offered_rhs_per_s": round(rate * float(np.mean(sizes)), 1),
            "max_concurrent_batches": int(st["max_concurrent_batches"])}


# Extra resident factorizations for the multi-factor serving leg: DFT and FIO
# (polar and multiscale) at uneven sizes, beside the benchmark's own factor.
SERVE_EXTRA = [
    ("dft64", dict(kernel="dft", n=64, tol=1e-6, leaf=4, split="none")),
    ("dft128", dict(kernel="dft", n=128, tol=1e-6, leaf=4, split="none")),
    ("fio64polar", dict(kernel="fio", n=64, tol=1e-6, leaf=4, split="polar")),
    ("fio128polar", dict(kernel="fio", n=128, tol=1e-6, leaf=4, split="polar")),
    ("fio64ms", dict(kernel="fio", n=64, tol=1e-4, leaf=4, split="multiscale")),
    ("fio128ms", dict(kernel="fio", n=128, tol=1e-4, leaf=4, split="multiscale")),
]


def serve_multi(main_name, F_main, N_main, dev, nreq=700, seed=1):
    """Poisson stream over several resident factorizations of uneven N: each
    request picks a factorization uniformly and has 1..32 RHS; continuous
    batching per factorization through one mbf_server (4 slots), offered at
    ~80% of the throughput estimated from solo 32-RHS applies."""
    import numpy as np
    import torch

    import mbf_workloads as W
    import paper_1509_07925_amd as mbf

    t0 = time.time()
    facs = [(main_name, F_main, N_main)]
    for name, c in SERVE_EXTRA:
        if name == main_name:
            continue
        n = c["n"]
        x, xi = (W.grid_x_integer(n), W.grid_omega(n)) if c["kernel"] == "dft" else (W.grid_x_unit(n), W.grid_omega(n))
        facs.append((name, mbf.Factor.build(x, xi, n, kernel=c["kernel"], tol=c["tol"], leaf_side=c["leaf"],
                                            split=c["split"], precs=["c64"], max_rank=4096), n * n))
    log("multi-factor serving: %d factorizations resident (extra builds %.1fs)" % (len(facs), time.time() - t0))
    rng = np.random.default_rng(seed)
    which = rng.integers(0, len(facs), size=nreq)
    sizes = rng.integers(1, 33, size=nreq)
    pools = [torch.randn((32, N), dtype=torch.complex64, device=dev) for _, _, N in facs]
    per_rhs = []
    for (name, F, N), pool in zip(facs, pools):
        F.apply(pool.t())
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(3):
            F.apply(pool.t())
        torch.cuda.synchronize()
        per_rhs.append((time.perf_counter() - t1) / (3 * 32))
    mean_service = float(np.mean([per_rhs[w] * k for w, k in zip(which, sizes)]))
    rate = 0.8 / mean_service
    arrivals = W.poisson_arrivals(nreq, rate, seed=seed)
    ins = [pools[w][: int(k)].t() for w, k in zip(which, sizes)]
    outs = [torch.empty((int(k), facs[w][2]), dtype=torch.complex64, device=dev).t() for w, k in zip(which, sizes)]
    srv = mbf.Server(mem_budget=24 << 30, nslots=4, max_batch_rhs=256)
    ids = []
    t_start = time.perf_counter()
    for i in range(nreq):
        while time.perf_counter() - t_start < arrivals[i]:
            pass
        ids.append(srv.submit(facs[which[i]][1], ins[i], outs[i]))
    srv.drain()
    lat_ms = np.array([srv.poll(r)[1] / 1e3 for r in ids])
    st = srv.stats()
    srv.close()
    per = {}
    for j, (name, _, N) in enumerate(facs):
        sel = lat_ms[which == j]
        if sel.size:
            per[name] = {"N": int(N), "requests": int(sel.size), "p50_ms": round(float(np.percentile(sel, 50)), 3),
                         "p99_ms": round(float(np.percentile(sel, 99)), 3)}
    return {"factorizations": len(facs), "requests": int(st["requests"]), "rhs": int(st["rhs"]),
            "batches": int(st["batches"]), "p50_ms": round(st["p50_us"] / 1e3, 3), "p99_ms": round(st["p99_us"] / 1e3, 3),
            "rhs_per_s": round(st["rhs"] / st["wall_s"], 1) if st["wall_s"] > 0 else None,
            "offered_rhs_per_s": round(rate * float(np.mean(sizes)), 1),
            "max_concurrent_batches": int(st["max_concurrent_batches"]), "per_factorization": per}


def cpu_baseline(cfg, x, xi, g, u_gpu, out):
    """Oracle leg: direct FP64 summation (eq. (kernel)) on sampled rows."""
    import threadpoolctl

    import mbf_workloads as W
    from oracle import direct, kernels

    n, nrhs = cfg["n"], g.shape[1]
    N = n * n
    K = kernels.dft(n) if cfg["kernel"] == "dft" else kernels.fio_radon(n)
    # bounded sample: about 10 s of host work at n = 512
    nrows = max(64, min(N, int(4096 * (256.0 / n) ** 2)))
    rows = W.sample_rows(N, nrows, seed=1)
    info = threadpoolctl.threadpool_info()
    cores = max([i.get("num_threads", 1) for i in info] + [1])
    t0 = time.perf_counter()
    ref = direct.direct_rows(K, x, xi, g, rows, block=256)
    dt = time.perf_counter() - t0
    out["rel_err_vs_direct_sampled_rows"] = direct.rel_err(u_gpu[rows], ref)
    return {"value": round(nrhs / (dt * N / nrows), 6), "unit": "RHS/s", "cores": int(cores), "kind": "oracle",
            "sample": "direct FP64 sum of eq. (kernel) on %d of %d rows x %d RHS in %.2f s, "
                      "scaled to the full N" % (nrows, N, nrhs, dt)}


if __name__ == "__main__":
    main()
