"""Serving loop on the GPU: continuous batching, memory admission, p50/p99.

Every result computed inside a mixed, co-batched stream of requests must
match the same request applied alone and agree with the oracle's FP64 apply
of the same factors, column by column (FP32 bar 1e-6, tests/bars.py).
"""

import time

import numpy as np
import pytest

import mbf_workloads as W
from oracle import butterfly, direct, kernels
from tests.bars import assert_columns_close
from tests.factor_io import to_import

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _factors():
    import paper_1509_07925_amd as mbf
    out = []
    for n, leaf, kern in ((16, 2, "dft"), (32, 4, "fio")):
        if kern == "dft":
            x, xi = W.grid_x_integer(n), W.grid_omega(n)
            bf = butterfly.build_plain(kernels.dft(n), x, xi, ((0, 0), n), ((-n / 2, -n / 2), n),
                                       int(np.log2(n // leaf)), 1e-6, 10 ** 6, method="exact")
        else:
            x, xi = W.grid_x_unit(n), W.grid_omega(n)
            bf = butterfly.build_polar(kernels.fio_radon(n), x, xi, n, ((0, 0), 1.0), 3, 1e-6, 10 ** 6,
                                       method="exact")
        out.append((mbf.Factor.import_factors(precs=["c64"], **to_import(bf)), bf, n * n))
    return out


def _col(a, dev):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a).T)).to(dev, torch.complex64).t()


def _np(t):
    return t.t().contiguous().cpu().numpy().astype(np.complex128).T


def _hold_stream(dev):
    """Queue tens of milliseconds of work on the current stream: requests
    submitted next (each waits for an event recorded after it) pile up in
    the server's queue while the first ones hold the slots, so the later
    ones share batches whatever the host's timing."""
    busy = torch.randn((4096, 4096), device=dev)
    for _ in range(6):
        busy = busy @ busy
        busy = busy / busy.abs().max()
    return busy


@pytest.mark.parametrize("graphs", [False, True])
def test_mixed_stream_equals_solo_and_oracle(graphs):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1509_07925_amd as mbf
    dev = torch.device("cuda:0")
    facs = _factors()
    rng = np.random.default_rng(0)
    srv = mbf.Server(mem_budget=256 << 20, nslots=4, max_batch_rhs=128, graphs=graphs)
    pending = []
    for i in range(60):
        k = int(rng.integers(len(facs)))
        N = facs[k][2]
        nr = int(rng.integers(1, 33))
        g = W.rhs(N, nr, seed=100 + i)
        pending.append((k, g, _col(g, dev), torch.empty((nr, N), dtype=torch.complex64, device=dev).t()))
    reqs = []
    for i, (k, g, gt, ut) in enumerate(pending):
        if i % 20 == 0:
            _hold_stream(dev)  # three waves of arrivals while earlier batches wait or run
        reqs.append((srv.submit(facs[k][0], gt, ut), k, g, gt, ut))
    srv.drain()
    st = srv.stats()
    assert st["requests"] == 60
    assert st["batches"] < 60  # requests were co-batched
    assert st["p99_us"] >= st["p50_us"] > 0
    if graphs:  # every batch replayed a graph; at most one capture per (slot, factor, width)
        assert st["graph_batches"] == st["batches"]
        assert 1 <= st["graphs_captured"] <= min(st["batches"], 4 * len(facs) * 4)
    else:
        assert st["graph_batches"] == 0 and st["graphs_captured"] == 0
    for rid, k, g, gt, ut in reqs:
        done, lat = srv.poll(rid)
        assert done and lat > 0
        F, bf, N = facs[k]
        mixed = _np(ut)
        solo = _np(F.apply(gt))
        assert_columns_close(mixed, solo, 1e-6, "request %d: mix vs alone" % rid)
        assert_columns_close(mixed, bf.apply(g), 1e-6, "request %d: mix vs oracle" % rid)
    srv.close()


def test_memory_admission_serializes_batches():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1509_07925_amd as mbf
    dev = torch.device("cuda:0")
    F, bf, N = _factors()[0]
    one = 2 * N * 32 * 8 + F.workspace_size("c64", 32) + 4096
    srv = mbf.Server(mem_budget=one, nslots=4, max_batch_rhs=32)
    outs = []
    for i in range(12):
        g = W.rhs(N, 32, seed=i)
        ut = torch.empty((32, N), dtype=torch.complex64, device=dev).t()
        gt = _col(g, dev)
        torch.cuda.synchronize()
        outs.append((srv.submit(F, gt, ut), g, gt, ut))
    srv.drain()
    st = srv.stats()
    assert st["requests"] == 12 and st["max_concurrent_batches"] == 1
    for rid, g, gt, ut in outs:
        assert_columns_close(_np(ut), bf.apply(g), 1e-6, "request %d" % rid)
    # a request that can never fit the budget fails cleanly
    g = W.rhs(N, 64, seed=99)
    gt = _col(g, dev)
    ut = torch.empty((64, N), dtype=torch.complex64, device=dev).t()
    small = mbf.Server(mem_budget=1 << 16, nslots=1, max_batch_rhs=64)
    rid = small.submit(F, gt, ut)
    with pytest.raises(mbf.MBFError):
        for _ in range(2000):
            done, _ = small.poll(rid)
            if done:
                break
            time.sleep(0.001)
    small.close()
    srv.close()


def test_batch_above_budget_waits_instead_of_failing():
    """Queued requests that together exceed the memory pool are split over
    several batches: each request that fits alone completes (none fails with
    MBF_ERR_OOM), with the right result.  A request id that was already
    reported is refused."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1509_07925_amd as mbf
    dev = torch.device("cuda:0")
    F, bf, N = _factors()[0]
    one = 2 * N * 32 * 8 + F.workspace_size("c64", 32) + 4096
    srv = mbf.Server(mem_budget=one, nslots=2, max_batch_rhs=256)
    reqs = []
    gs = [W.rhs(N, 32, seed=200 + i) for i in range(8)]
    gts = [_col(g, dev) for g in gs]
    torch.cuda.synchronize()
    for g, gt in zip(gs, gts):
        ut = torch.empty((32, N), dtype=torch.complex64, device=dev).t()
        reqs.append((srv.submit(F, gt, ut), g, ut))
    srv.drain()
    st = srv.stats()
    assert st["requests"] == 8 and st["batches"] >= 8
    for rid, g, ut in reqs:
        done, lat = srv.poll(rid)
        assert done and lat > 0
        assert_columns_close(_np(ut), bf.apply(g), 1e-6, "request %d" % rid)
    with pytest.raises(mbf.MBFError) as e:
        srv.poll(reqs[0][0])
    assert e.value.status == -1
    srv.close()


def test_request_waits_for_its_input_event():
    """submit records an event on the caller's stream: g written by work
    still running there is read only after that work (the server's streams
    do not follow the caller's)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1509_07925_amd as mbf
    dev = torch.device("cuda:0")
    F, bf, N = _factors()[0]
    g = W.rhs(N, 8, seed=300)
    src = _col(g, dev)
    srv = mbf.Server(mem_budget=64 << 20, nslots=2, max_batch_rhs=64)
    busy = torch.randn((4096, 4096), device=dev)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        gt = torch.zeros_like(src)
        for _ in range(8):  # keep the stream busy before g is written
            busy = busy @ busy
            busy = busy / busy.abs().max()
        gt.copy_(src)
        ut = torch.empty((8, N), dtype=torch.complex64, device=dev).t()
        rid = srv.submit(F, gt, ut)
    srv.drain()
    done, _ = srv.poll(rid)
    assert done
    assert_columns_close(_np(ut), bf.apply(g), 1e-6, "request after a slow producer")
    srv.close()


def test_graph_regions_are_given_back_between_factorizations():
    """Graph mode with a pool that holds one slot region at a time:
    alternating factorizations make a slot give back its region and take a
    larger one (dropping its graphs), and every result stays right."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1509_07925_amd as mbf
    dev = torch.device("cuda:0")
    facs = _factors()
    big = max(2 * N * 16 * 8 + F.workspace_size("c64", 16) for F, _, N in facs)
    srv = mbf.Server(mem_budget=big + 8192, nslots=2, max_batch_rhs=16, graphs=True)
    for rnd in range(3):
        for k in (0, 1, 0):
            F, bf, N = facs[k]
            g = W.rhs(N, 5, seed=400 + 10 * rnd + k)
            gt = _col(g, dev)
            ut = torch.empty((5, N), dtype=torch.complex64, device=dev).t()
            torch.cuda.synchronize()
            rid = srv.submit(F, gt, ut)
            srv.drain()
            done, _ = srv.poll(rid)
            assert done
            assert_columns_close(_np(ut), bf.apply(g), 1e-6, "round %d factor %d" % (rnd, k))
    st = srv.stats()
    assert st["graph_batches"] == 9 and st["graphs_captured"] >= 3
    srv.close()


@pytest.mark.parametrize("graphs", [True, False])
def test_device_built_mix_at_n64_and_n128(graphs):
    """Served mix over device-built factorizations of the 2D DFT and the
    multiscale FIO at n = 64 and 128, with graph launches (multiscale parts
    one after the other inside the graphs) and with per-kernel launches
    (multiscale parts on side streams of each slot): every request's result
    equals the same request applied alone (per column), and on 64 sampled
    rows matches the direct sum within the factorization's bar."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1509_07925_amd as mbf
    dev = torch.device("cuda:0")
    facs = []
    for kern, n, tol, split in (("dft", 64, 1e-6, "none"), ("fio", 64, 1e-4, "multiscale"),
                                ("dft", 128, 1e-6, "none"), ("fio", 128, 1e-4, "multiscale")):
        x, xi = (W.grid_x_integer(n), W.grid_omega(n)) if kern == "dft" else (W.grid_x_unit(n), W.grid_omega(n))
        F = mbf.Factor.build(x, xi, n, kernel=kern, tol=tol, leaf_side=4, split=split, precs=["c64"],
                             builder="device")
        K = kernels.dft(n) if kern == "dft" else kernels.fio_radon(n)
        facs.append((F, K, x, xi, n * n, tol))
    rng = np.random.default_rng(5)
    srv = mbf.Server(mem_budget=1 << 30, nslots=4, max_batch_rhs=128, graphs=graphs)
    pending = []
    for i in range(48):
        k = int(rng.integers(len(facs)))
        N = facs[k][4]
        nr = int(rng.integers(1, 33))
        g = W.rhs(N, nr, seed=500 + i)
        pending.append((k, g, _col(g, dev), torch.empty((nr, N), dtype=torch.complex64, device=dev).t()))
    reqs = []
    for i, (k, g, gt, ut) in enumerate(pending):
        if i % 16 == 0:
            _hold_stream(dev)  # three waves of arrivals while earlier batches wait or run
        reqs.append((srv.submit(facs[k][0], gt, ut), k, g, gt, ut))
    srv.drain()
    st = srv.stats()
    assert st["requests"] == 48 and st["batches"] < 48
    assert st["graph_batches"] == (st["batches"] if graphs else 0)
    for rid, k, g, gt, ut in reqs:
        F, K, x, xi, N, tol = facs[k]
        mixed = _np(ut)
        assert_columns_close(mixed, _np(F.apply(gt)), 1e-6, "request %d: mix vs alone" % rid)
        rows = W.sample_rows(N, 64, seed=rid)
        ref = direct.direct_rows(K, x, xi, g, rows, block=64)
        err = np.linalg.norm(mixed[rows] - ref) / np.linalg.norm(ref)
        assert err < 50 * tol, "request %d: %.2e against the direct sum" % (rid, err)
    srv.close()
