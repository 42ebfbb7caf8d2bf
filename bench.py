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
                      fp32_only=True, deadline=1140),
    # served request mix over eight factorizations (see SERVE8)
    "serve8": dict(serve8=True, deadline=1100),
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
    # the parts of a multiscale apply one after the other here, so that each
    # launch's events time that kernel alone (side by side, launches overlap)
    prev = os.environ.get("MBF_PART_STREAMS")
    os.environ["MBF_PART_STREAMS"] = "0"
    try:
        F.profile_begin(steps * (4 + 2 * max(inf.depth, 8)) * max(inf.nparts, 1) + 64)
        for _ in range(steps):
            fn(g, out=u, prec=prec, workspace=ws)
        torch.cuda.synchronize()
        recs = F.profile_end()
    finally:
        if prev is None:
            del os.environ["MBF_PART_STREAMS"]
        else:
            os.environ["MBF_PART_STREAMS"] = prev
    return t1 - t0, recs


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


def hbm_roofline(recs, steps=None, ms_per_step=None, side_by_side=False):
    """Stage launches measured against HBM bandwidth (few right-hand sides),
    each launch timed alone (the profiled pass runs a multiscale apply's
    parts one after the other).  With the parts side by side in the timed
    steps, `whole_apply_gbps` adds the whole apply's algorithmic bytes (every
    launch) over the timed wall time per apply."""
    stage = [r for r in recs if r["kind"] == 1]
    st_ms = sum(r["ms"] for r in stage)
    st_bytes = sum(r["bytes"] for r in stage)
    per_launch = st_bytes / (st_ms * 1e-3) / 1e9 if st_ms > 0 else 0.0
    out = {"bound": "hbm", "achieved": round(per_launch, 1), "peak": 8000.0, "unit": "GB/s",
           "frac": round(per_launch / 8000.0, 4), "traffic": None,
           "kernel": "stage block product (16 x 16 tile, few RHS)",
           "launches": len(stage), "avg_launch_ms": round(st_ms / max(len(stage), 1), 4),
           "alg_bytes_per_launch_avg": st_bytes / max(len(stage), 1),
           "kernel_share_of_step": round(st_ms / (sum(r["ms"] for r in recs) or 1.0), 4)}
    if side_by_side and steps and ms_per_step:
        all_bytes = sum(r["bytes"] for r in recs) / steps
        out.update({"alg_bytes_per_step": all_bytes,
                    "whole_apply_gbps": round(all_bytes / (ms_per_step * 1e-3) / 1e9, 1),
                    "note": "timed steps: corona parts and center on side streams; per-launch events: "
                            "the parts one after the other"})
    return out


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
    ap.add_argument("--deadline", type=float, default=None,
                    help="seconds from the start after which optional legs are skipped (default: the "
                         "config's, else MBF_BENCH_DEADLINE, else 420)")
    ap.add_argument("--builder", default="device", choices=["device", "host"])
    ap.add_argument("--serve-requests", type=int, default=10000, help="serve8: measured requests per load")
    ap.add_argument("--serve-warmup", type=int, default=500, help="serve8: warm-up requests per load")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run one 1 GiB device-to-device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.deadline is None:
        args.deadline = float(CONFIGS[args.config].get("deadline", os.environ.get("MBF_BENCH_DEADLINE", "420")))
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
    if cfg.get("serve8"):
        serve8_main(args, budget)
        return
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
    side = inf.nparts > 1 and os.environ.get("MBF_PART_STREAMS", "1") != "0"
    out["roofline"] = roofline(recs, args.steps, "c64") if nrhs > 32 else hbm_roofline(recs, args.steps,
                                                                                       ms_per_step, side)
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
    adj = None
    if cfg.get("adjoint"):
        # adjoint of another random input h, and the identity <h, K g> = <K^* h, g>
        h_host = W.rhs(N, nrhs, seed=2)
        h = torch.from_numpy(np.ascontiguousarray(h_host.T)).to(dev, torch.complex64).t()
        v = F.apply_adjoint(h)
        torch.cuda.synchronize()
        v_np = v.t().contiguous().cpu().numpy().astype(np.complex128).T
        lhs, rhs = np.vdot(h_host, u_np), np.vdot(v_np, g_host)
        out["adjoint_identity_rel"] = float(abs(lhs - rhs) / abs(lhs))
        log("adjoint identity: %.2e" % out["adjoint_identity_rel"])
        adj = (h_host, v_np)
        del h, v
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, x, xi, g_host, u_np, out, adj=adj)
        log("CPU baseline: %s" % out["cpu_baseline"]["sample"])

    # ------------------------------------------------------------ optional legs
    if cfg.get("adjoint") and budget.allow("adjoint", 30):
        h = torch.empty((nrhs, N), dtype=torch.complex64, device=dev).t()
        h.copy_(g)
        v = torch.empty((nrhs, N), dtype=torch.complex64, device=dev).t()
        a_total, a_recs = timed_apply(F, h, v, ws, "c64", args.steps, args.warmup, adjoint=True)
        out["adjoint"] = {"value": round(nrhs * args.steps / a_total, 2), "unit": "RHS/s",
                          "ms_per_step": round(1e3 * a_total / args.steps, 4),
                          "roofline": roofline(a_recs, args.steps, "c64") if nrhs > 32 else hbm_roofline(
                              a_recs, args.steps, 1e3 * a_total / args.steps, side),
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
        out["serving"] = serve_loads([(out["config"]["workload"], F, N)], dev, budget)

    out["skipped_legs"] = budget.skipped
    out["wall_s"] = round(time.time() - budget.t0, 1)
    print(json.dumps(out), flush=True)


class _Stream:
    """A seeded request stream over resident factorizations: request i goes
    to factorization fac[i] (uniform) with size[i] in 1..32 RHS; inputs are
    column slices of one random block per factorization, outputs a ring of
    64 blocks per factorization (the bench never reads them)."""

    def __init__(self, facs, dev, count, seed):
        import numpy as np
        import torch
        rng = np.random.default_rng(seed)
        self.fac = rng.integers(0, len(facs), size=count)
        self.size = rng.integers(1, 33, size=count)
        self.facs = facs
        self.src = [torch.randn((32, N), dtype=torch.complex64, device=dev) for _, _, N in facs]
        self.ring = [[torch.empty((32, N), dtype=torch.complex64, device=dev) for _ in range(64)]
                     for _, _, N in facs]
        torch.cuda.synchronize()

    def request(self, i):
        k, m = int(self.fac[i]), int(self.size[i])
        return self.facs[k][1], self.src[k][:m].t(), self.ring[k][i % 64][:m].t()


def _serve_run(srv, stream, lo, hi, arrivals):
    """Submit requests lo..hi-1 at the given arrival times (seconds from the
    start); per-request latencies (ms) and the wall time to the last completion."""
    import numpy as np
    ids = []
    t_start = time.perf_counter()
    for i in range(lo, hi):
        while time.perf_counter() - t_start < arrivals[i - lo]:
            pass
        F, g, u = stream.request(i)
        ids.append(srv.submit(F, g, u, ready=False))
    srv.drain()
    wall = time.perf_counter() - t_start
    lat = np.array([srv.poll(r)[1] / 1e3 for r in ids])
    return lat, wall


def serve_loads(facs, dev, budget, loads=(0.5, 0.8, 0.95), nreq=1500, warm=200, ncal=600, graphs=True,
                seed=0, mem_budget=48 << 30):
    """Served Poisson streams over the resident factorizations (continuous
    batching through one mbf_server, 4 slots, up to 256 RHS per batch,
    graph-captured applies when `graphs`): 1..32 RHS per request on a
    uniformly drawn factorization.  The capacity is measured on a saturated
    stream (ncal requests queued at once); each load then offers
    warm + nreq Poisson arrivals at load x capacity, and p50 / p99 are taken
    over the nreq requests after the warm-up."""
    import numpy as np

    import mbf_workloads as W
    import paper_1509_07925_amd as mbf
    total = ncal + len(loads) * (warm + nreq)
    stream = _Stream(facs, dev, total, seed)
    srv = mbf.Server(mem_budget=mem_budget, nslots=4, max_batch_rhs=256, graphs=graphs)
    res = {"graphs": bool(graphs), "slots": 4, "max_batch_rhs": 256, "mem_budget_gb": round(mem_budget / 2 ** 30, 1),
           "factorizations": [name for name, _, _ in facs], "request_rhs": "uniform 1..32",
           "factorization_choice": "uniform", "loads": []}
    # capacity: the calibration requests queued at once (twice: the first pass
    # also captures the graphs)
    for rep in range(2):
        _, wall = _serve_run(srv, stream, 0, ncal, np.zeros(ncal))
    capacity = float(np.sum(stream.size[:ncal])) / wall
    res["capacity_rhs_per_s"] = round(capacity, 1)
    lo = ncal
    for li, load in enumerate(loads):
        rate = load * capacity / float(np.mean(stream.size))
        arrivals = W.poisson_arrivals(warm + nreq, rate, seed=seed + 1 + li)
        hi = lo + warm + nreq
        if arrivals[-1] > budget.left() - 20:
            budget.skipped.append("serving load %.2f (%.0f s of arrivals, %.0f s left)" % (
                load, arrivals[-1], budget.left()))
            lo = hi
            continue
        lat, wall = _serve_run(srv, stream, lo, hi, arrivals)
        sizes = stream.size[lo:hi]
        lat_m = lat[warm:]
        res["loads"].append({"load": load, "requests": int(lat_m.size), "warmup_requests": int(warm),
                             "offered_rhs_per_s": round(load * capacity, 1),
                             "served_rhs_per_s": round(float(np.sum(sizes)) / wall, 1),
                             "p50_ms": round(float(np.percentile(lat_m, 50)), 3),
                             "p99_ms": round(float(np.percentile(lat_m, 99)), 3),
                             "mean_ms": round(float(np.mean(lat_m)), 3)})
        log("served %s at %.2f of capacity (%.0f RHS/s): p50 %.2f ms p99 %.2f ms" % (
            "graphs" if graphs else "direct", load, capacity, res["loads"][-1]["p50_ms"],
            res["loads"][-1]["p99_ms"]))
        lo = hi
    st = srv.stats()
    srv.close()
    res.update({"batches": int(st["batches"]), "max_concurrent_batches": int(st["max_concurrent_batches"]),
                "graphs_captured": int(st["graphs_captured"]), "graph_batches": int(st["graph_batches"])})
    return res


# The served mix over eight resident factorizations: the 2D DFT and the FIO
# of Example 1 at n = 64, 128, 256, 512 (FP32 factors only).
SERVE8 = [dict(kernel=k, n=n, tol=1e-6 if k == "dft" else 1e-4, leaf=4, split="none" if k == "dft" else "multiscale")
          for k in ("dft", "fio") for n in (64, 128, 256, 512)]


def serve8_main(args, budget):
    """--config serve8: build the eight factorizations, then serve the same
    seeded stream with per-kernel launches and with graph launches at loads
    0.5, 0.8 and 0.95 of each mode's measured capacity (10000 requests after
    500 warm-up requests per load)."""
    import torch

    import mbf_workloads as W
    import paper_1509_07925_amd as mbf
    dev = torch.device("cuda:0")
    out = {"metric": "served RHS/s and p50/p99 latency over a Poisson request mix", "value": None,
           "unit": "RHS/s", "n_gpus": 1, "steps": None, "warmup": None, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic"}
    facs = []
    t0 = time.time()
    for c in SERVE8:
        n = c["n"]
        x, xi = (W.grid_x_integer(n), W.grid_omega(n)) if c["kernel"] == "dft" else (W.grid_x_unit(n), W.grid_omega(n))
        t1 = time.time()
        F = mbf.Factor.build(x, xi, n, kernel=c["kernel"], tol=c["tol"], leaf_side=c["leaf"], split=c["split"],
                             precs=["c64"], max_rank=4096, builder="device")
        ws = torch.empty(F.workspace_size("c64", 256), dtype=torch.uint8, device=dev)
        for w in (32, 64, 256):
            F.autotune("c64", w, workspace=ws)
        del ws
        name = workload_name(dict(c, nrhs=0)).replace("_rhs0", "")
        log("built %s in %.1f s" % (name, time.time() - t1))
        facs.append((name, F, n * n))
    torch.cuda.empty_cache()
    out["config"] = {"workload": "serve_mix8_dft_fio_n64-512", "factorizations": [f[0] for f in facs],
                     "setup_s": round(time.time() - t0, 1)}
    modes = {}
    for graphs in (False, True):
        modes["graphs" if graphs else "direct"] = serve_loads(facs, dev, budget, nreq=args.serve_requests,
                                                              warm=args.serve_warmup, ncal=2000, graphs=graphs)
    out["serving"] = modes
    g = modes["graphs"]["loads"]
    if g:
        out["value"] = g[-1]["served_rhs_per_s"]
        out["p50_ms"], out["p99_ms"] = g[-1]["p50_ms"], g[-1]["p99_ms"]
        out["value_at_load"] = g[-1]["load"]
    out["skipped_legs"] = budget.skipped
    out["wall_s"] = round(time.time() - budget.t0, 1)
    print(json.dumps(out), flush=True)


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


def cpu_baseline(cfg, x, xi, g, u_gpu, out, reps=5, adj=None):
    """Oracle leg: the direct FP64 sum of eq. (kernel) on sampled rows (the
    paper's error estimator and speed-up denominator), with all host cores
    and with one, median of `reps` runs each, scaled to RHS/s over all rows;
    for the DFT also the oracle's FFT closed form (numpy, one core) and the
    same transform with scipy.fft on all cores.  With adj = (h, v) (v the
    library's adjoint of h) also the adjoint's error on 256 sampled Omega
    points, against the conjugate-transposed kernel columns summed directly."""
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
    if adj is not None:
        h, v_gpu = adj
        cols = W.sample_rows(N, 256, seed=3)
        v_direct = K(x, xi[cols]).conj().T @ h
        out["rel_err_adjoint_vs_direct_sampled_cols"] = direct.rel_err(v_gpu[cols], v_direct)

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
