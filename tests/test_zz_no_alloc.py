"""mbf_apply_scratch, the apply that allocates nothing, against mbf_apply
through the C ABI: the same kernels on the same factors give the same
result, on two calls in a row (the second smaller, so the scratch holds the
first call's data when the second starts), and a request larger than the
scratch is refused."""

import ctypes

import numpy as np
import pytest

import mbf_workloads as W
from oracle import butterfly, kernels
from tests.bars import assert_columns_close
from tests.factor_io import to_import

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BAR = {"c128": 1e-12, "c64": 1e-6}


def _mbf():
    import paper_1509_07925_amd as mbf
    return mbf


def _factor(precs):
    mbf = _mbf()
    n = 32
    x, xi = W.grid_x_integer(n), W.grid_omega(n)
    bf = butterfly.build_plain(kernels.dft(n), x, xi, ((0, 0), n), ((-n / 2, -n / 2), n), 4, 1e-6, 10 ** 6,
                               method="exact")
    return mbf.Factor.import_factors(precs=precs, **to_import(bf)), bf, n * n


def _abi_apply(F, prec, g, scratch):
    mbf = _mbf()
    lib = mbf.lib()
    nin, nrhs = g.shape
    nout = F.info().nx
    u = torch.full((nrhs, nout), float("nan"), dtype=g.dtype, device=g.device).t()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    gp, up = ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(u.data_ptr())
    if scratch:
        st = lib.mbf_apply_scratch(F._h, mbf.PREC[prec], nrhs, gp, nin, up, nout, stream)
    else:
        ws = torch.empty(max(F.workspace_size(prec, nrhs), 1), dtype=torch.uint8, device=g.device)
        st = lib.mbf_apply(F._h, mbf.PREC[prec], nrhs, gp, nin, up, nout, ctypes.c_void_p(ws.data_ptr()),
                           ws.numel(), stream)
    assert st == 0, lib.mbf_last_error().decode()
    torch.cuda.synchronize()
    return u.t().contiguous().cpu().numpy().astype(np.complex128).T


def _gpu(a, prec):
    dt = torch.complex128 if prec == "c128" else torch.complex64
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a).T)).to("cuda:0", dt).t()


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_scratch_apply_equals_apply_on_two_calls(prec):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    F, bf, N = _factor([prec])
    assert _mbf().lib().mbf_scratch_bytes() == 128 << 20
    for nrhs, seed in ((48, 1), (5, 2)):  # the second call is smaller
        g = W.rhs(N, nrhs, seed=seed)
        gt = _gpu(g, prec)
        got = _abi_apply(F, prec, gt, scratch=True)
        ref = _abi_apply(F, prec, gt, scratch=False)
        assert np.isfinite(got).all()
        np.testing.assert_array_equal(got, ref)  # same kernels, same data
        assert_columns_close(got, ref, BAR[prec], "scratch apply vs apply (%d RHS)" % nrhs)
        assert_columns_close(got, bf.apply(g), BAR[prec], "scratch apply vs oracle (%d RHS)" % nrhs)


def test_scratch_apply_refuses_more_than_the_scratch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    mbf = _mbf()
    lib = mbf.lib()
    F, bf, N = _factor(["c64"])
    per = F.workspace_size("c64", 64) / 64.0
    nrhs = int(lib.mbf_scratch_bytes() / per) + 64
    assert F.workspace_size("c64", nrhs) > lib.mbf_scratch_bytes()
    g = torch.zeros((nrhs, N), dtype=torch.complex64, device="cuda:0").t()
    u = torch.zeros((nrhs, N), dtype=torch.complex64, device="cuda:0").t()
    st = lib.mbf_apply_scratch(F._h, mbf.PREC["c64"], nrhs, ctypes.c_void_p(g.data_ptr()), N,
                               ctypes.c_void_p(u.data_ptr()), N, None)
    assert st == -1
    assert "scratch" in lib.mbf_last_error().decode()
    # the scratch still serves a fitting request afterwards
    g2 = W.rhs(N, 3, seed=9)
    got = _abi_apply(F, "c64", _gpu(g2, "c64"), scratch=True)
    assert_columns_close(got, bf.apply(g2), 1e-6, "after a refused request")
