"""Pins of the oracle's kernels and plain summation (CPU only)."""

import os

import numpy as np
import pytest

import mbf_workloads as W
from oracle import direct, kernels

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    return np.loadtxt(os.path.join(GOLD, name), comments="#")


def test_dft_kernel_matches_hand_values_n2():
    n = 2
    K = kernels.dft(n)(W.grid_x_integer(n), W.grid_omega(n))
    ref = _load("dft_n2.txt")
    np.testing.assert_allclose(K.real, ref, atol=1e-15)
    np.testing.assert_allclose(K.imag, 0.0, atol=1e-15)


def test_fio_phase_matches_hand_values():
    rows = _load("fio_phase.txt")
    Phi = kernels.fio_phase()
    for x1, x2, a, b, val in rows:
        got = Phi(np.array([[x1, x2]]), np.array([[a, b]]))[0, 0]
        assert abs(got - val) < 1e-14


def test_fio_kernel_is_exp_of_phase_and_homogeneous():
    n = 16
    x = W.grid_x_unit(n)
    xi = W.grid_omega(n)
    K = kernels.fio_radon(n)(x, xi)
    Phi = kernels.fio_phase()(x, xi)
    np.testing.assert_allclose(K, np.exp(2j * np.pi * Phi), atol=1e-12)
    # homogeneous of degree one in xi (Section 3.1): K(x, 2 xi) = K(x, xi)^2
    K2 = kernels.fio_radon(2 * n)(x, 2 * xi)
    np.testing.assert_allclose(K2, K * K, atol=1e-12)


@pytest.mark.parametrize("n", [4, 8, 16])
def test_direct_dft_equals_fft(n):
    g = W.rhs(n * n, 3, seed=n)
    x, xi = W.grid_x_integer(n), W.grid_omega(n)
    u = direct.direct(kernels.dft(n), x, xi, g)
    assert direct.rel_err(u, direct.dft_fft(n, g)) < 1e-14
    # Parseval: the DFT matrix is sqrt(N) times a unitary matrix.
    np.testing.assert_allclose(np.sum(np.abs(u) ** 2, 0), n * n * np.sum(np.abs(g) ** 2, 0),
                               rtol=1e-12)


@pytest.mark.parametrize("n", [4, 8])
def test_direct_dft_adjoint_closed_form(n):
    h = W.rhs(n * n, 2, seed=3)
    x, xi = W.grid_x_integer(n), W.grid_omega(n)
    K = kernels.dft(n)(x, xi)
    np.testing.assert_allclose(K.conj().T @ h, direct.dft_fft_adjoint(n, h), atol=1e-11)


def test_fio_with_zero_ellipses_is_inverse_fft():
    n = 16
    g = W.rhs(n * n, 2, seed=5)
    x, xi = W.grid_x_unit(n), W.grid_omega(n)
    u = direct.direct(kernels.fio_radon(n, c_scale=0.0), x, xi, g)
    assert direct.rel_err(u, direct.linear_phase_ifft(n, g)) < 1e-13


def test_direct_rows_is_subset_of_full():
    n = 8
    g = W.rhs(n * n, 2, seed=7)
    x, xi = W.grid_x_unit(n), W.grid_omega(n)
    K = kernels.fio_radon(n)
    rows = W.sample_rows(n * n, 10, seed=1)
    np.testing.assert_allclose(direct.direct_rows(K, x, xi, g, rows),
                               direct.direct(K, x, xi, g)[rows], atol=1e-12)
