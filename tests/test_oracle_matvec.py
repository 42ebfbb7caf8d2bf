"""Pins of the oracle's build case (i) and of Example 2 (CPU only).

Case (i) (Section 2.3): the middle-level blocks are known only through
products of K and K^* with zero-padded Gaussian probes, and each is
factored by the SVD via random matrix-vector products (Section 2.1, first
option).  Example 2 (Section 3.3, eq. (example2mfio), eq. (KFK)): the
composition K~ = K F K of the Example 1 FIO with the discrete Fourier
transform, evaluated directly.

* exact recovery: a block of rank below the probe count is reproduced to
  rounding, and its singular values are those of the dense SVD;
* a planted mistake (products with K^T in place of K^*) breaks that
  recovery;
* the case (i) build of the 2D DFT with full-rank blocks reproduces the
  dense kernel, and equals the entry-based build;
* K F K with c1 = c2 = 0 has the closed form N K (K F = N I on these grids),
  the FFT closed form of the linear-phase FIO;
* the adjoint of the composition satisfies <K~ g, h> = <g, K~^* h>;
* PBF-m and MBF-m of K F K at n = 32 approximate its direct evaluation, and
  a larger rank makes the approximation better.
"""

import numpy as np

import mbf_workloads as W
from oracle import butterfly, direct, kernels, lowrank


def _gauss(rng, m, q):
    return (rng.standard_normal((m, q)) + 1j * rng.standard_normal((m, q))) / np.sqrt(2.0)


def test_svd_matvec_recovers_a_low_rank_block():
    rng = np.random.default_rng(0)
    m, n, r = 40, 30, 6
    Z = _gauss(rng, m, r) @ _gauss(rng, r, n)
    C, R = _gauss(rng, n, 16), _gauss(rng, m, 16)
    U0, s, V0 = lowrank.svd_matvec(Z @ C, Z.conj().T @ R, C, R, 1e-12, 10)
    assert s.size == r
    assert np.linalg.norm(U0 @ np.diag(s) @ V0.conj().T - Z) < 1e-12 * np.linalg.norm(Z)
    np.testing.assert_allclose(s, np.linalg.svd(Z, compute_uv=False)[:r], rtol=1e-11)


def test_svd_matvec_planted_transpose_fails():
    rng = np.random.default_rng(1)
    m, n, r = 40, 30, 6
    Z = _gauss(rng, m, r) @ _gauss(rng, r, n)
    C, R = _gauss(rng, n, 16), _gauss(rng, m, 16)
    # Z^T R where Z^* R belongs: the row basis spans the conjugate space
    U0, s, V0 = lowrank.svd_matvec(Z @ C, Z.T @ R, C, R, 1e-12, 10)
    assert np.linalg.norm(U0 @ np.diag(s) @ V0.conj().T - Z) > 1e-3 * np.linalg.norm(Z)


def test_svd_matvec_of_zero_block_has_rank_zero():
    rng = np.random.default_rng(2)
    C, R = _gauss(rng, 9, 5), _gauss(rng, 7, 5)
    U0, s, V0 = lowrank.svd_matvec(np.zeros((7, 5)), np.zeros((9, 5)), C, R, 1e-8, 3)
    assert s.size == 0 and U0.shape == (7, 0) and V0.shape == (9, 0)


def test_case_i_build_of_the_dft_is_exact_and_matches_entry_build():
    n, leaf = 16, 1
    x, xi = W.grid_x_integer(n), W.grid_omega(n)
    D = kernels.dft(n)(x, xi)
    N, L = n * n, int(np.log2(n // leaf))
    rng = np.random.default_rng(3)
    q = 16 + 10
    probes = (_gauss(rng, N, q), _gauss(rng, N, q))
    mv = lambda adj, B: D.conj().T @ B if adj else D @ B
    bf = butterfly.build_plain(None, x, xi, ((0, 0), n), ((-n / 2, -n / 2), n), L, 1e-12, 16,
                               method="matvec", matvec=mv, probes=probes)
    ex = butterfly.build_plain(kernels.dft(n), x, xi, ((0, 0), n), ((-n / 2, -n / 2), n), L, 1e-12, 16,
                               method="exact")
    g = W.rhs(N, 3, seed=4)
    assert direct.rel_err(bf.apply(g), D @ g) < 1e-10
    assert direct.rel_err(bf.apply(g), ex.apply(g)) < 1e-10
    h = W.rhs(N, 3, seed=5)
    assert direct.rel_err(bf.adjoint(h), D.conj().T @ h) < 1e-10
    assert bf.max_rank() == ex.max_rank()


def test_composition_with_linear_phase_is_n_squared_times_k():
    n = 16
    x, xi = W.grid_x_unit(n), W.grid_omega(n)
    op = direct.ComposedFIO(kernels.fio_radon(n, c_scale=0.0), x, xi)
    g = W.rhs(n * n, 2, seed=6)
    ref = (n * n) * direct.linear_phase_ifft(n, g)
    assert direct.rel_err(op.apply(g), ref) < 1e-12


def test_composition_adjoint_identity():
    n = 16
    x, xi = W.grid_x_unit(n), W.grid_omega(n)
    op = direct.ComposedFIO(kernels.fio_radon(n), x, xi)
    g, h = W.rhs(n * n, 1, seed=7)[:, 0], W.rhs(n * n, 1, seed=8)[:, 0]
    lhs, rhs = np.vdot(h, op.apply(g)), np.vdot(op.adjoint(h), g)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def _kfk_build(n, rmax, split, seed=9):
    x, xi = W.grid_x_unit(n), W.grid_omega(n)
    op = direct.ComposedFIO(kernels.fio_radon(n), x, xi)
    N = n * n
    rng = np.random.default_rng(seed)
    q = rmax + 10
    probes = (_gauss(rng, N, q), _gauss(rng, N, q))
    if split == "polar":
        bf = butterfly.build_polar(None, x, xi, n, ((0, 0), 1.0), int(np.log2(n)), 1e-8, rmax,
                                   method="matvec", matvec=op.matvec, probes=probes)
    else:
        bf = butterfly.build_multiscale(None, x, xi, n, ((0, 0), 1.0), 1e-8, rmax, center_side=16,
                                        leaf_side=1, method="matvec", matvec=op.matvec, probes=probes)
    return op, bf


def test_pbf_m_of_the_composition_n32():
    errs = []
    for rmax in (16, 32):
        op, bf = _kfk_build(32, rmax, "polar")
        g, h = W.rhs(32 * 32, 2, seed=10), W.rhs(32 * 32, 2, seed=11)
        errs.append(direct.rel_err(bf.apply(g), op.apply(g)))
        assert direct.rel_err(bf.adjoint(h), op.adjoint(h)) < 10 * errs[-1] + 1e-12
    assert errs[0] < 1e-1 and errs[1] < 1e-3 and errs[1] < errs[0] / 10


def test_mbf_m_of_the_composition_n32():
    op, bf = _kfk_build(32, 32, "multiscale")
    g = W.rhs(32 * 32, 2, seed=12)
    assert direct.rel_err(bf.apply(g), op.apply(g)) < 2e-2
    # the dense center is K~ restricted to its columns, exactly
    E = np.zeros((32 * 32, bf.center_idx.size), complex)
    E[bf.center_idx, np.arange(bf.center_idx.size)] = 1.0
    assert np.abs(bf.KC - op.apply(E)).max() < 1e-9 * np.abs(bf.KC).max()
