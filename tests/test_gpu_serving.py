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


def test_mixed_stream_equals_solo_and_oracle():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1509_07925_amd as mbf
    dev = torch.device("cuda:0")
    facs = _factors()
    rng = np.random.default_rng(0)
    srv = mbf.Server(mem_budget=256 << 20, nslots=4, max_batch_rhs=128)
    reqs = []
    for i in range(60):
        k = int(rng.integers(len(facs)))
        F, bf, N = facs[k]
        nr = int(rng.integers(1, 33))
        g = W.rhs(N, nr, seed=100 + i)
        gt = _col(g, dev)
        ut = torch.empty((nr, N), dtype=torch.complex64, device=dev).t()
        torch.cuda.synchronize()
        rid = srv.submit(F, gt, ut)
        reqs.append((rid, k, g, gt, ut))
        if i % 7 == 0:
            time.sleep(0.002)  # arrivals while earlier batches run
    srv.drain()
    st = srv.stats()
    assert st["requests"] == 60
    assert st["batches"] < 60  # requests were co-batched
    assert st["p99_us"] >= st["p50_us"] > 0
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
