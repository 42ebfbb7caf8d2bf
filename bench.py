#!/usr/bin/env python3
"""Apply throughput of the multidimensional butterfly factorization on one GPU.

One step = one mbf_apply of the whole factorization (leaf projection, every
stage block product, middle scaling, leaf reconstruction) to one batch of
nrhs right-hand sides that are already resident in HBM.  Prints one JSON
line: RHS/s of the plain FP32 apply, the roofline of the dominant kernel
(the stage block product) measured with HIP events over the timed steps,
the relative errors against the FP64 apply of the same factors and against
the direct sum on sampled rows, and the CPU oracle (direct FP64 sum and the
FFT closed form) timed on the host.  Optional legs (split BF16, 16 RHS,
PCIe-inclusive rate, served request mix) follow while the run stays inside
its time budget (--deadline seconds from the start); the line lists the
legs it skipped.  The factors are built on the GPU (FP64 device builder).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--config NAME]
                       [--save PATH | --load PATH] [--deadline S] ...
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
    device synchronisation; then the same number of applies again with the
    library's per-launch HIP events on, for the breakdown by kernel (the
    events cost time of their own, so they are kept out of the timed steps)."""
    import torch
    fn = F.apply_adjoint if adjoint else F.apply
    for _ in range(warmup):
        fn(g, out=u, prec=prec, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn(g, out=u, prec=prec, workspace=ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    inf = F.info()
    F.profile_begin(steps * (4 + 2 * max(inf.depth, 8)) + 64)
    for _ in range(steps):
        fn(g, out=u, prec=prec, workspace=ws)
    torch.cuda.synchronize()
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
    (profiles/hbm_traffic_*.json) with the file they come from, or (None,
    None) when those counters were taken on another workload / precision or
    before the stage kernel source last changed (its hash is recorded with
    the counters)."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_1509_07925_amd", "csrc", "stage_mfma.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "hbm_traffic_*.json"))):
        rec = json.load(open(path))
        if rec.get("workload") == workload and rec.get("prec") == prec and rec.get("kernel_source_sha256_16") == sha:
            return rec["traffic_bytes_per_launch"], {"file": os.path.relpath(path, ROOT), "stage_mfma_sha256_16": sha,
                                                     "command": rec.get("command")}
    return None, None


class Budget:
    """Time left before --deadline (seconds since the start of the run)."""

    def __init__(self, deadline):
        self.t0 = time.time()
        self.deadline = deadline
        self.skipped = []

    def left(self):
        return self.deadline - (time.time() - self.t0)

    def allow(self, name, need_s):
        if self.left() >= need_s:
            return True
        self.skipped.append(name)
        log("skipping %s (%.0f s left, about %.0f s needed)" % (name, self.left(), need_s))
        return False


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
    ap.add_argument("--deadline", type=float, default=float(os.environ.get("MBF_BENCH_DEADLINE", "420")),
                    help="seconds from the start after which optional legs are skipped")
    ap.add_argument("--builder", default="device", choices=["device", "host"])
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run one 1 GiB device-to-device copy (HBM counter calibration)")
    args = ap.parse_args()
    budget = Budget(args.deadline)
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

    # Long builds report progress on stderr.
    os.environ.setdefault("MBF_VERBOSE", "1")
    import signal

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
    out = {"metric": METRIC, "value": None, "unit": "RHS/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic"}

    # A SIGTERM (e.g. an outer time limit) prints what has been measured.
    def on_term(signum, frame):
        out["terminated"] = "SIGTERM before the run finished"
        out["skipped_legs"] = budget.skipped
        print(json.dumps(out), flush=True)
        os._exit(3)

    signal.signal(signal.SIGTERM, on_term)

    t0 = time.time()
    if args.load:
        log("loading", args.load)
        F = mbf.Factor.load(args.load, precs=precs)
        built = False
    else:
        all_precs = precs + ([] if args.no_fp64_check else ["c128"])
        log("building %s (n=%d tol=%g leaf=%d) precs=%s on the %s" % (args.config, n, cfg["tol"], cfg["leaf"],
                                                                       all_precs, args.builder))
        F = mbf.Factor.build(x, xi, n, kernel=cfg["kernel"], tol=cfg["tol"], leaf_side=cfg["leaf"],
                             split=cfg["split"], precs=all_precs, max_rank=4096, builder=args.builder)
        built = True
    torch.cuda.synchronize()
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
    log("autotuned %d FP32 stage shapes in %.1fs" % (tuned, time.time() - t1))
    total_s, recs = timed_apply(F, g, u, ws, "c64", args.steps, args.warmup)
    ms_per_step = 1e3 * total_s / args.steps
    value = nrhs * args.steps / total_s
    log("FP32: %.1f RHS/s (%.3f ms/step)" % (value, ms_per_step))
    out.update({"value": round(value, 2), "ms_per_step": round(ms_per_step, 4)})
    out["config"] = {"workload": workload_name(cfg),
                     "kernel": cfg["kernel"], "split": cfg["split"], "n": n, "N": N, "nrhs": nrhs, "tol": cfg["tol"],
                     "depth": inf.depth, "ranks": list(inf.max_rank[:inf.depth + 1]), "nnz": inf.nnz,
                     "factor_gb_on_device": round(inf.device_bytes / 1e9, 3),
                     "setup_s": round(setup_s, 1),
                     "setup": "load" if args.load else "mbf_build (%s FP64)" % args.builder}
    out["roofline"] = roofline(recs, args.steps, "c64") if nrhs > 32 else hbm_roofline(recs)
    traffic, src = measured_traffic(out["config"]["workload"], "c64")
    out["roofline"]["traffic"] = traffic
    out["roofline"]["traffic_source"] = src
    out["ms_per_step_by_kind"] = breakdown(recs, args.steps)
    u32 = u.clone()

    # error against the FP64 apply of the same factors (required)
    if built and not args.no_fp64_check:
        g64 = torch.from_numpy(np.ascontiguousarray(g_host.T)).to(dev, torch.complex128).t()
        u64 = F.apply(g64, prec="c128")
        torch.cuda.synchronize()
        nrm = u64.abs().pow(2).sum().sqrt()
        out["rel_err_vs_fp64_apply"] = float((u32.to(torch.complex128) - u64).abs().pow(2).sum().sqrt() / nrm)
        colerr = ((u32.to(torch.complex128) - u64).abs().pow(2).sum(0).sqrt() / u64.abs().pow(2).sum(0).sqrt())
        out["rel_err_vs_fp64_apply_worst_column"] = float(colerr.max())
        log("FP32 vs FP64 apply: %.2e (worst column %.2e)" % (out["rel_err_vs_fp64_apply"],
                                                              out["rel_err_vs_fp64_apply_worst_column"]))
        del g64
    else:
        u64 = None

    u_np = u32.t().contiguous().cpu().numpy().astype(np.complex128).T
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, x, xi, g_host, u_np, out)
        log("CPU baseline: %s" % out["cpu_baseline"]["sample"])

    # ------------------------------------------------------------ optional legs
    if cfg.get("adjoint") and budget.allow("adjoint", 30):
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

    if not args.no_split and budget.allow("split_bf16x3", 60):
        t1 = time.time()
        F.autotune("bf16x3", nrhs, workspace=ws)
        u16 = torch.empty_like(u)
        s_total, s_recs = timed_apply(F, g, u16, ws, "bf16x3", args.steps, args.warmup)
        sval = nrhs * args.steps / s_total
        d = (u16.to(torch.complex128) - u32.to(torch.complex128)).abs().pow(2).sum().sqrt() / \
            u32.to(torch.complex128).abs().pow(2).sum().sqrt()
        out["split_bf16x3"] = {"value": round(sval, 2), "unit": "RHS/s", "ms_per_step": round(1e3 * s_total / args.steps, 4),
                               "dtype": "bf16 hi/lo x3, f32 accumulate", "roofline": roofline(s_recs, args.steps, "bf16x3"),
                               "rel_diff_vs_fp32_apply": float(d), "autotune_s": round(time.time() - t1, 1)}
        if u64 is not None:
            out["split_bf16x3"]["rel_err_vs_fp64_apply"] = float(
                (u16.to(torch.complex128) - u64).abs().pow(2).sum().sqrt() / u64.abs().pow(2).sum().sqrt())
        log("BF16x3: %.1f RHS/s" % sval)
        del u16

    # few right-hand sides: the 16 x 16 matrix-core stage kernel, bound by reading the blocks from HBM
    nn = 16
    if nrhs > nn and budget.allow("narrow_rhs16", 30):
        g_n, u_n = g[:, :nn], torch.empty((nn, N), dtype=torch.complex64, device=dev).t()
        n_total, n_recs = timed_apply(F, g_n, u_n, ws, "c64", args.steps, args.warmup)
        out["narrow_rhs16"] = {"value": round(nn * args.steps / n_total, 2), "unit": "RHS/s",
                               "ms_per_step": round(1e3 * n_total / args.steps, 4), "nrhs": nn,
                               "roofline": hbm_roofline(n_recs)}
        if u64 is not None:
            u64n = u64[:, :nn]
            out["narrow_rhs16"]["rel_err_vs_fp64_apply"] = float(
                (u_n.to(torch.complex128) - u64n).abs().pow(2).sum().sqrt() / u64n.abs().pow(2).sum().sqrt())
        log("FP32 at %d RHS: %.1f RHS/s" % (nn, out["narrow_rhs16"]["value"]))
    del u64
    torch.cuda.empty_cache()

    # host-resident inputs and outputs: pinned buffers, copies on the same stream (context, not `value`)
    if budget.allow("pcie_inclusive", 30):
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

    if not args.no_serve and budget.allow("serving", 60):
        out["serving"] = serve_mix(F, N, dev, budget)
        log("served at %.0f%% of the measured capacity: p50 %.1f ms p99 %.1f ms" % (
            100 * out["serving"]["load"], out["serving"]["p50_ms"], out["serving"]["p99_ms"]))

    out["skipped_legs"] = budget.skipped
    out["wall_s"] = round(time.time() - budget.t0, 1)
    print(json.dumps(out), flush=True)


def _serve_run(srv_args, F, N, dev, ins, outs, arrivals):
    """Submit requests at the given arrival times; per-request latencies (ms)."""
    import numpy as np

    import paper_1509_07925_amd as mbf
    srv = mbf.Server(**srv_args)
    ids = []
    t_start = time.perf_counter()
    for i in range(len(ins)):
        while time.perf_counter() - t_start < arrivals[i]:
            pass
        ids.append(srv.submit(F, ins[i], outs[i], ready=False))
    srv.drain()
    wall = time.perf_counter() - t_start
    lat = np.array([srv.poll(r)[1] / 1e3 for r in ids])
    st = srv.stats()
    srv.close()
    return lat, wall, st


def serve_mix(F, N, dev, budget, nreq=1500, warm=200, load=0.8, seed=0):
    """Served Poisson stream on the resident factorization (continuous
    batching through mbf_server, 4 slots): 1..32 RHS per request, offered at
    `load` times the capacity measured on a saturated mixed stream of the
    same request sizes; p50 / p99 over the requests after a warm-up."""
    import numpy as np
    import torch

    import mbf_workloads as W

    rng = np.random.default_rng(seed)
    sizes = rng.integers(1, 33, size=nreq + warm)
    pool = torch.randn((64, N), dtype=torch.complex64, device=dev)  # request inputs drawn from here
    outs = [torch.empty((int(k), N), dtype=torch.complex64, device=dev).t() for k in sizes]
    ins = [pool[: int(k)].t() for k in sizes]
    torch.cuda.synchronize()
    srv_args = dict(mem_budget=24 << 30, nslots=4, max_batch_rhs=256)
    # capacity: every calibration request queued at once
    ncal = min(300, nreq)
    _, wall, st = _serve_run(srv_args, F, N, dev, ins[:ncal], outs[:ncal], np.zeros(ncal))
    capacity = float(np.sum(sizes[:ncal])) / wall
    rate = load * capacity / float(np.mean(sizes))
    arrivals = W.poisson_arrivals(nreq + warm, rate, seed=seed)
    if arrivals[-1] > budget.left() - 20:
        keep = int(np.searchsorted(arrivals, max(budget.left() - 20, 1.0)))
        arrivals, ins, outs, sizes = arrivals[:keep], ins[:keep], outs[:keep], sizes[:keep]
        warm = min(warm, keep // 4)
    lat, wall, st = _serve_run(srv_args, F, N, dev, ins, outs, arrivals)
    lat = lat[warm:]
    return {"requests": int(lat.size), "warmup_requests": int(warm), "load": load,
            "capacity_rhs_per_s": round(capacity, 1), "offered_rhs_per_s": round(load * capacity, 1),
            "served_rhs_per_s": round(float(np.sum(sizes)) / wall, 1),
            "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "batches": int(st["batches"]), "max_concurrent_batches": int(st["max_concurrent_batches"])}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _host_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(cfg, x, xi, g, u_gpu, out, reps=5):
    """Oracle leg: the direct FP64 sum of eq. (kernel) on sampled rows (the
    paper's error estimator and speed-up denominator), with all host cores
    and with one, median of `reps` runs each, scaled to RHS/s over all rows;
    for the DFT also the oracle's FFT closed form (numpy, one core) and the
    same transform with scipy.fft on all cores."""
    import numpy as np
    import threadpoolctl

    import mbf_workloads as W
    from oracle import direct, kernels

    n, nrhs = cfg["n"], g.shape[1]
    N = n * n
    cores = _host_cores()
    K = kernels.dft(n) if cfg["kernel"] == "dft" else kernels.fio_radon(n)
    rows = W.sample_rows(N, 256, seed=1)
    out["rel_err_vs_direct_sampled_rows"] = direct.rel_err(u_gpu[rows], direct.direct_rows(K, x, xi, g, rows, block=256))

    def med(fn):
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    # bounded sample: about 2 s per run at n = 512 on 16 cores
    nrows = max(16, min(N, int(256 * (512.0 / n) ** 2)))
    rows_all = W.sample_rows(N, nrows, seed=2)
    with threadpoolctl.threadpool_limits(cores):
        t_all = med(lambda: direct.direct_rows(K, x, xi, g, rows_all, block=256))
    rows_one = rows_all[: max(4, nrows // 16)]
    with threadpoolctl.threadpool_limits(1):
        t_one = med(lambda: direct.direct_rows(K, x, xi, g, rows_one, block=256))
    res = {"value": round(nrhs / (t_all * N / nrows), 6), "unit": "RHS/s", "cores": int(cores), "kind": "oracle",
           "sample": "direct FP64 sum of eq. (kernel) on %d of %d rows x %d RHS, median of %d runs %.2f s on %d "
                     "threads, scaled to all rows" % (nrows, N, nrhs, reps, t_all, cores),
           "cpu_model": _cpu_model(),
           "direct_one_core": {"value": round(nrhs / (t_one * N / rows_one.size), 6), "unit": "RHS/s", "cores": 1,
                               "sample": "%d rows, median of %d runs %.2f s" % (rows_one.size, reps, t_one)}}
    if cfg["kernel"] == "dft" and cfg["split"] == "none":
        import scipy.fft
        nf = min(nrhs, 64)
        gs = g[:, :nf]
        with threadpoolctl.threadpool_limits(1):
            t_fft1 = med(lambda: direct.dft_fft(n, gs))
        G = np.ascontiguousarray(gs.T.reshape(nf, n, n))
        t_fftc = med(lambda: scipy.fft.fft2(scipy.fft.ifftshift(G, axes=(1, 2)), axes=(1, 2), workers=cores))
        res["fft_one_core"] = {"value": round(nf / t_fft1, 2), "unit": "RHS/s", "cores": 1,
                               "sample": "oracle closed form (numpy fft2) on %d RHS, median of %d runs" % (nf, reps)}
        res["fft_all_cores"] = {"value": round(nf / t_fftc, 2), "unit": "RHS/s", "cores": int(cores),
                                "sample": "scipy.fft.fft2 with workers=%d on %d RHS, median of %d runs" % (
                                    cores, nf, reps)}
    return res


if __name__ == "__main__":
    main()
