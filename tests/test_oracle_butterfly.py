"""Pins of the oracle's butterfly factorizations (CPU only).

* full rank: the factorization reproduces the dense kernel matrix
  (brute force) -- any wrong index, permutation, transpose or dropped
  factor in the build or the apply breaks it;
* adjoint identity <K~ g, h> = <g, K~^* h> for the factorized operator;
* ranks of the 2D DFT blocks equal the count obtained from the Kronecker
  structure of the kernel (independent 1D SVDs);
* accuracy at a tolerance against FFT closed forms (DFT, and the FIO with
  c1 = c2 = 0 for the polar and multiscale splits) and direct sums;
* planted mistakes in the oracle make these pins fail.
"""

import numpy as np
import pytest

import mbf_workloads as W
from oracle import butterfly, direct, kernels, lowrank, trees


def _dft_bf(n, leaf, tol, method="exact", rmax=10 ** 6, seed=0):
    x, xi = W.grid_x_integer(n), W.grid_omega(n)
    L = int(np.log2(n // leaf))
    return butterfly.build_plain(kernels.dft(n), x, xi, ((0, 0), n), ((-n / 2, -n / 2), n), L,
                                 tol, rmax, method=method, seed=seed)


def _dense(K, x, xi):
    return K(x, xi)


@pytest.mark.parametrize("n,leaf", [(4, 1), (4, 2), (8, 1), (8, 2), (8, 4), (16, 2), (16, 4)])
def test_full_rank_dft_equals_dense(n, leaf):
    bf = _dft_bf(n, leaf, 1e-14)
    x, xi = W.grid_x_integer(n), W.grid_omega(n)
    Kd = kernels.dft(n)(x, xi)
    g = W.rhs(n * n, 3, seed=1)
    assert direct.rel_err(bf.apply(g), Kd @ g) < 1e-12
    h = W.rhs(n * n, 3, seed=2)
    assert direct.rel_err(bf.adjoint(h), Kd.conj().T @ h) < 1e-12


@pytest.mark.parametrize("n,depth", [(8, 3), (16, 3), (16, 4)])
def test_full_rank_fio_polar_equals_dense(n, depth):
    x, xi = W.grid_x_unit(n), W.grid_omega(n)
    K = kernels.fio_radon(n)
    bf = butterfly.build_polar(K, x, xi, n, ((0, 0), 1.0), depth, 1e-14, 10 ** 6, method="exact")
    Kd = K(x, xi)
    g = W.rhs(n * n, 2, seed=3)
    assert direct.rel_err(bf.apply(g), Kd @ g) < 1e-12
    assert direct.rel_err(bf.adjoint(g), Kd.conj().T @ g) < 1e-12


def test_full_rank_multiscale_equals_dense():
    n = 64
    x, xi = W.grid_x_unit(n), W.grid_omega(n)
    K = kernels.fio_radon(n)
    ms = butterfly.build_multiscale(K, x, xi, n, ((0, 0), 1.0), 1e-14, 10 ** 6,
                                    leaf_side=4, method="exact")
    assert [t for t, _, _ in ms.parts] == [0, 1]
    g = W.rhs(n * n, 1, seed=4)
    rows = W.sample_rows(n * n, 64, seed=0)
    ref = direct.direct_rows(K, x, xi, g, rows)
    assert direct.rel_err(ms.apply(g)[rows], ref) < 1e-11


@pytest.mark.parametrize("n,leaf,tol", [(16, 2, 1e-6), (32, 4, 1e-6), (32, 2, 1e-4)])
def test_adjoint_identity(n, leaf, tol):
    bf = _dft_bf(n, leaf, tol, method="sampling")
    g = W.rhs(n * n, 2, seed=5)
    h = W.rhs(n * n, 2, seed=6)
    lhs = np.vdot(h, bf.apply(g))
    rhs = np.vdot(bf.adjoint(h), g)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def _kron_rank(n, wa, wb, tol):
    """Rank of a 2D DFT block of side wa x wb from the 1D spectra."""
    x = np.arange(wa)
    xi = np.arange(wb)
    K1 = np.exp(-2j * np.pi * np.outer(x, xi) / n)
    s = np.linalg.svd(K1, compute_uv=False)
    prod = np.outer(s, s).ravel()
    return int(np.count_nonzero(prod > tol * prod.max()))


@pytest.mark.parametrize("n,leaf,tol", [(32, 2, 1e-6), (64, 8, 1e-8)])
def test_dft_middle_ranks_match_kronecker_spectra(n, leaf, tol):
    bf = _dft_bf(n, leaf, tol, method="exact")
    L, m = bf.L, bf.m
    want = _kron_rank(n, n >> m, n >> (L - m), tol)
    assert set(bf.rank[m].values()) == {want}
    if n == 64:
        # the 8x8-leaf profile of the n = 64 correctness configuration
        assert bf.max_rank() == [64, 248, 248, 64]


@pytest.mark.parametrize("n,leaf,tol", [(32, 2, 1e-6), (32, 2, 1e-4), (32, 4, 1e-3)])
def test_dft_accuracy_against_fft(n, leaf, tol):
    bf = _dft_bf(n, leaf, tol, method="sampling")
    g = W.rhs(n * n, 2, seed=8)
    err = direct.rel_err(bf.apply(g), direct.dft_fft(n, g))
    assert err < 10 * tol
    # truncation really happened: the error is not at rounding level
    assert err > 1e-3 * tol


def test_sampling_matches_exact_svd_on_dft_block():
    n = 64
    x, xi = W.grid_x_integer(n), W.grid_omega(n)
    K = kernels.dft(n)
    xt = trees.QuadTree(x, (0, 0), n, 4)
    ot = trees.QuadTree(xi, (-n / 2, -n / 2), n, 4)
    ia, ib = xt.points(2, 6), ot.points(2, 9)
    Z = K(x[ia], xi[ib])
    rng = np.random.default_rng(0)
    U0, s, V0 = lowrank.svd_sampling(lambda I, J: K(x[ia[I]], xi[ib[J]]), ia.size, ib.size,
                                     1e-6, 10 ** 6, rng)
    _, se, _ = lowrank.svd_trunc(Z, 1e-6, 10 ** 6)
    assert abs(s.size - se.size) <= 2
    k = min(s.size, se.size)
    np.testing.assert_allclose(s[:k], se[:k], rtol=0, atol=1e-5 * se[0])
    err = np.linalg.norm(Z - (U0 * s) @ V0.conj().T, 2) / se[0]
    assert err < 1e-5


def test_polar_split_reproduces_linear_phase_closed_form():
    n = 32
    x, xi = W.grid_x_unit(n), W.grid_omega(n)
    K = kernels.fio_radon(n, c_scale=0.0)
    bf = butterfly.build_polar(K, x, xi, n, ((0, 0), 1.0), 4, 1e-7, 10 ** 6, method="sampling")
    g = W.rhs(n * n, 2, seed=9)
    assert direct.rel_err(bf.apply(g), direct.linear_phase_ifft(n, g)) < 1e-5


def test_multiscale_split_reproduces_linear_phase_closed_form():
    n = 64
    x, xi = W.grid_x_unit(n), W.grid_omega(n)
    K = kernels.fio_radon(n, c_scale=0.0)
    ms = butterfly.build_multiscale(K, x, xi, n, ((0, 0), 1.0), 1e-7, 10 ** 6, leaf_side=4)
    g = W.rhs(n * n, 1, seed=10)
    assert direct.rel_err(ms.apply(g), direct.linear_phase_ifft(n, g)) < 1e-5
    h = W.rhs(n * n, 1, seed=11)
    assert abs(np.vdot(h, ms.apply(g)) - np.vdot(ms.adjoint(h), g)) < 1e-10 * abs(np.vdot(h, ms.apply(g)))


def test_example1_polar_and_multiscale_against_direct():
    n = 32
    x, xi = W.grid_x_unit(n), W.grid_omega(n)
    K = kernels.fio_radon(n)
    g = W.rhs(n * n, 1, seed=12)
    ref = direct.direct(K, x, xi, g)
    pb = butterfly.build_polar(K, x, xi, n, ((0, 0), 1.0), 4, 1e-6, 10 ** 6)
    assert direct.rel_err(pb.apply(g), ref) < 1e-4
    ms = butterfly.build_multiscale(K, x, xi, n, ((0, 0), 1.0), 1e-6, 10 ** 6, leaf_side=2)
    assert direct.rel_err(ms.apply(g), ref) < 1e-4


# --------------------------------------------------------- planted mistakes
def test_planted_mistake_wrong_middle_scaling_is_caught(monkeypatch):
    good = lowrank.form1
    monkeypatch.setattr(lowrank, "form1", lambda U0, s, V0: (good(U0, s, V0)[0], s,
                                                             good(U0, s, V0)[2]))
    bf = _dft_bf(8, 2, 1e-14)
    Kd = kernels.dft(8)(W.grid_x_integer(8), W.grid_omega(8))
    g = W.rhs(64, 1, seed=1)
    assert direct.rel_err(bf.apply(g), Kd @ g) > 1e-3


def test_planted_mistake_swapped_children_is_caught(monkeypatch):
    orig = trees.QuadTree.children

    def swapped(self, level, code):
        kids = orig(self, level, code)
        return kids[::-1] if level == 0 else kids

    monkeypatch.setattr(trees.QuadTree, "children", swapped)
    bf = _dft_bf(8, 2, 1e-14)
    monkeypatch.setattr(trees.QuadTree, "children", orig)
    Kd = kernels.dft(8)(W.grid_x_integer(8), W.grid_omega(8))
    g = W.rhs(64, 1, seed=1)
    assert direct.rel_err(bf.apply(g), Kd @ g) > 1e-3


def test_planted_mistake_unconjugated_adjoint_is_caught(monkeypatch):
    bf = _dft_bf(8, 2, 1e-14)
    for k in bf.UL:
        bf.UL[k] = bf.UL[k].conj()  # plant: apply uses U instead of conj(U) in the adjoint
    Kd = kernels.dft(8)(W.grid_x_integer(8), W.grid_omega(8))
    h = W.rhs(64, 1, seed=2)
    assert direct.rel_err(bf.adjoint(h), Kd.conj().T @ h) > 1e-3


def _bounding(p):
    lo = p.min(axis=0)
    return (lo[0], lo[1]), float((p.max(axis=0) - lo).max())


def test_general_point_sets_full_rank_equals_dense():
    """General point sets (Section 2.6): clustered X and non-grid Omega in a
    disk, trees over the bounding squares with empty nodes dropped, plain and
    polar Omega trees; at full rank the factorization reproduces the dense
    kernel (brute force) forward and adjoint."""
    x = W.clustered_points(400, seed=7)
    xi = W.disk_frequencies(300, 12.0, seed=8)
    K = kernels.fio_points()
    Kd = K(x, xi)
    g, h = W.rhs(300, 3, seed=9), W.rhs(400, 3, seed=10)
    r = np.hypot(xi[:, 0], xi[:, 1])
    polar = np.stack([r / r.max(), np.mod(np.arctan2(xi[:, 1], xi[:, 0]) / (2 * np.pi), 1.0)], axis=1)
    for pts, obox in ((xi, _bounding(xi)), (polar, ((0.0, 0.0), 1.0))):
        ent = lambda I, J: K(x[I], xi[J])
        bf = butterfly.Butterfly.build(ent, x, pts, _bounding(x), obox, 3, 1e-14, 10 ** 6, method="exact")
        assert len(bf.xt.nodes[3]) < 64 and len(bf.ot.nodes[3]) <= 64  # empty leaves dropped
        assert direct.rel_err(bf.apply(g), Kd @ g) < 1e-11
        assert direct.rel_err(bf.adjoint(h), Kd.conj().T @ h) < 1e-11


def test_point_set_kernel_agrees_with_grid_kernel_on_grids():
    n = 16
    x, xi = W.grid_x_unit(n), W.grid_omega(n)
    np.testing.assert_allclose(kernels.fio_points()(x, xi), kernels.fio_radon(n)(x, xi), atol=1e-11)
