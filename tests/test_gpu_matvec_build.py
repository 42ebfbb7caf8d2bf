"""Build case (i) in the library (mbf_build_matvec), applied on the GPU.

Case (i) of Section 2.3: K is known only through fast products with K and
K^*; every middle-level block is factored from products with zero-padded
Gaussian probes (SVD via random matrix-vector products, Section 2.1).

* the 2D DFT at n = 16 with full-rank middle blocks: the library's build
  from the dense black box and the oracle's build from the same probes are
  the same operator (exact recovery; FP64 apply to 1e-10 per column);
* Example 2 (Section 3.3, eq. (example2mfio), eq. (KFK)) at n = 32: the
  library's PBF-m of K~ = K F K from the oracle's dense black box and the
  oracle's PBF-m from the same probes both approximate the direct
  evaluation of K~, and agree with each other;
* Example 2 at n = 64 with the library's own apply and adjoint of the FIO
  (device-built PBF, FP64) and FFTs as the black box: the PBF-m of K~
  reproduces the direct evaluation K F K g (dense K and F in FP64) within
  the error the oracle's PBF-m reaches at the same rank (3.5e-2 at r = 20,
  2.7e-3 at r = 32 on the CPU), forward and adjoint, and its FP32 apply
  stays within the FP32 bar of its FP64 apply.
"""

import numpy as np
import pytest

import mbf_workloads as W
from oracle import butterfly, direct, kernels
from tests.bars import assert_columns_close

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _gauss(rng, m, q):
    return (rng.standard_normal((m, q)) + 1j * rng.standard_normal((m, q))) / np.sqrt(2.0)


def _np(t):
    return t.t().contiguous().cpu().numpy().astype(np.complex128).T


def _apply(F, g, prec, adjoint=False):
    dev = torch.device("cuda:0")
    dt = torch.complex128 if prec == "c128" else torch.complex64
    gt = torch.from_numpy(np.ascontiguousarray(np.asarray(g).T)).to(dev, dt).t()
    out = F.apply_adjoint(gt, prec=prec) if adjoint else F.apply(gt, prec=prec)
    torch.cuda.synchronize()
    return _np(out)


def test_matvec_build_of_the_dft_matches_the_oracle():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1509_07925_amd as mbf
    n = 16
    x, xi = W.grid_x_integer(n), W.grid_omega(n)
    D = kernels.dft(n)(x, xi)
    N, q = n * n, 16 + 10
    rng = np.random.default_rng(20)
    probes = (_gauss(rng, N, q), _gauss(rng, N, q))
    mv = lambda adj, B: D.conj().T @ B if adj else D @ B
    F = mbf.Factor.build_matvec(x, xi, n, mv, tol=1e-12, max_rank=16, oversample=10, leaf_side=1, split="none",
                                probes=probes, precs=["c128", "c64"])
    bf = butterfly.build_plain(None, x, xi, ((0, 0), n), ((-n / 2, -n / 2), n), 4, 1e-12, 16, method="matvec",
                               matvec=mv, probes=probes)
    g, h = W.rhs(N, 5, seed=21), W.rhs(N, 5, seed=22)
    assert_columns_close(_apply(F, g, "c128"), bf.apply(g), 1e-10, "case (i) DFT apply vs oracle")
    assert_columns_close(_apply(F, h, "c128", adjoint=True), bf.adjoint(h), 1e-10, "case (i) DFT adjoint vs oracle")
    assert_columns_close(_apply(F, g, "c64"), D @ g, 1e-6, "case (i) DFT FP32 apply vs dense")


def test_example2_pbf_m_n32_library_and_oracle():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1509_07925_amd as mbf
    n, rmax = 32, 32
    x, xi = W.grid_x_unit(n), W.grid_omega(n)
    op = direct.ComposedFIO(kernels.fio_radon(n), x, xi)
    N, q = n * n, rmax + 10
    rng = np.random.default_rng(23)
    probes = (_gauss(rng, N, q), _gauss(rng, N, q))
    F = mbf.Factor.build_matvec(x, xi, n, op.matvec, tol=1e-8, max_rank=rmax, oversample=10, leaf_side=1,
                                split="polar", probes=probes, precs=["c128"])
    bf = butterfly.build_polar(None, x, xi, n, ((0, 0), 1.0), 5, 1e-8, rmax, method="matvec", matvec=op.matvec,
                               probes=probes)
    g, h = W.rhs(N, 4, seed=24), W.rhs(N, 4, seed=25)
    u, ref, uo = _apply(F, g, "c128"), op.apply(g), bf.apply(g)
    e_lib, e_ora = direct.rel_err(u, ref), direct.rel_err(uo, ref)
    assert e_lib < 1e-3 and e_ora < 1e-3, (e_lib, e_ora)
    assert direct.rel_err(u, uo) < 1e-3
    assert direct.rel_err(_apply(F, h, "c128", adjoint=True), op.adjoint(h)) < 1e-3


class _GpuComposition:
    """Black box of K~ = K F K on the GPU: the library's FP64 apply and
    adjoint of the FIO factorization K, and F / F^* by 2D FFTs
    (F[eta, y] = exp(-2 pi i y . eta), y = (i1, i2) / n, eta integer)."""

    def __init__(self, K, x, xi, n):
        self.K, self.n = K, n
        dev = torch.device("cuda:0")
        ix = np.rint(np.asarray(x) * n).astype(np.int64) % n
        ie = np.rint(np.asarray(xi)).astype(np.int64) % n
        self.xi1, self.xi2 = (torch.from_numpy(ix[:, k]).to(dev) for k in (0, 1))
        self.e1, self.e2 = (torch.from_numpy(ie[:, k]).to(dev) for k in (0, 1))
        self.calls = 0

    def _F(self, v):  # v: x-grid values, N x c
        n, c = self.n, v.shape[1]
        V = torch.zeros((c, n, n), dtype=torch.complex128, device=v.device)
        V[:, self.xi1, self.xi2] = v.t()
        return torch.fft.fft2(V)[:, self.e1, self.e2].t()  # N x c, column-major

    def _Fadj(self, w):  # w: Omega values, N x c
        n, c = self.n, w.shape[1]
        Wg = torch.zeros((c, n, n), dtype=torch.complex128, device=w.device)
        Wg[:, self.e1, self.e2] = w.t()
        return (torch.fft.ifft2(Wg) * (n * n))[:, self.xi1, self.xi2].t()

    def matvec(self, adjoint, block):
        self.calls += 1
        b = torch.from_numpy(np.ascontiguousarray(block.T)).to("cuda:0", torch.complex128).t()
        if adjoint:
            y = self.K.apply_adjoint(b, prec="c128")
            y = self._Fadj(y)
            y = self.K.apply_adjoint(y, prec="c128")
        else:
            y = self.K.apply(b, prec="c128")
            y = self._F(y)
            y = self.K.apply(y, prec="c128")
        torch.cuda.synchronize()
        return _np(y)


@pytest.mark.parametrize("rmax,bar", [(20, 1e-1), (32, 1e-2)])
def test_example2_composition_n64_through_the_library(rmax, bar):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1509_07925_amd as mbf
    n = 64
    x, xi = W.grid_x_unit(n), W.grid_omega(n)
    K = mbf.Factor.build(x, xi, n, kernel="fio", tol=1e-7, leaf_side=4, split="polar", precs=["c128"],
                         builder="device")
    box = _GpuComposition(K, x, xi, n)
    Kt = mbf.Factor.build_matvec(x, xi, n, box.matvec, tol=1e-8, max_rank=rmax, oversample=10, leaf_side=1,
                                 split="polar", seed=7, precs=["c128", "c64"])
    assert box.calls >= 2
    op = direct.ComposedFIO(kernels.fio_radon(n), x, xi)
    N = n * n
    g, h = W.rhs(N, 3, seed=26), W.rhs(N, 3, seed=27)
    # the black box itself: the library's K F K against the direct evaluation
    assert direct.rel_err(box.matvec(False, g), op.apply(g)) < 1e-5
    u = _apply(Kt, g, "c128")
    err = direct.rel_err(u, op.apply(g))
    assert err < bar, "K F K, r = %d: %.3e" % (rmax, err)
    assert direct.rel_err(_apply(Kt, h, "c128", adjoint=True), op.adjoint(h)) < bar
    assert_columns_close(_apply(Kt, g, "c64"), u, 1e-5, "FP32 apply of the K F K factors vs FP64")
