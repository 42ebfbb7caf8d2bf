"""Kernel entries K(x, xi) in FP64 (test infrastructure; see package header).

Both kernels are of the form e^{2 pi i Phi(x, xi)}:

* 2D DFT on integer grids: Phi = -(x . xi) / n.  The integer product
  x . xi is reduced modulo n before scaling, which is exact in integer
  arithmetic and keeps the phase argument in [0, 2 pi).
* Example 1 of Section 3.3 (generalized Radon transform), eq. (example1phi):
  Phi(x, xi) = x . xi + sqrt(c1(x)^2 xi1^2 + c2(x)^2 xi2^2),
  c1 = (2 + sin(2 pi x1) sin(2 pi x2)) / 16,
  c2 = (2 + cos(2 pi x1) cos(2 pi x2)) / 16,
  with x in the unit grid (eq. (X)) and xi in the integer grid (eq. (Omega)).
  ``c_scale = 0`` gives Phi = x . xi (the closed-form check of the split
  operators).
"""

import numpy as np


def dft(n):
    """K(x, xi) = exp(-2 pi i x.xi / n); x, xi integer coordinates (any
    dimension: x.xi sums over every coordinate)."""

    def K(x, xi):
        x = np.asarray(x, dtype=np.float64)
        xi = np.asarray(xi, dtype=np.float64)
        xi_i = np.rint(xi).astype(np.int64)
        x_i = np.rint(x).astype(np.int64)
        k = np.zeros((x_i.shape[0], xi_i.shape[0]), dtype=np.int64)
        for j in range(x_i.shape[1]):
            k += np.outer(x_i[:, j], xi_i[:, j])
        k %= n
        return np.exp(-2j * np.pi * (k.astype(np.float64) / n))

    return K


def fio_phase(c_scale=1.0):
    """Phi(x, xi) of eq. (example1phi) in FP64 for arbitrary real xi."""

    def Phi(x, xi):
        x = np.asarray(x, dtype=np.float64)
        xi = np.asarray(xi, dtype=np.float64)
        c1 = c_scale * (2.0 + np.sin(2 * np.pi * x[:, 0]) * np.sin(2 * np.pi * x[:, 1])) / 16.0
        c2 = c_scale * (2.0 + np.cos(2 * np.pi * x[:, 0]) * np.cos(2 * np.pi * x[:, 1])) / 16.0
        lin = np.outer(x[:, 0], xi[:, 0]) + np.outer(x[:, 1], xi[:, 1])
        return lin + np.sqrt(np.outer(c1 * c1, xi[:, 0] ** 2) + np.outer(c2 * c2, xi[:, 1] ** 2))

    return Phi


def fio_radon(n, c_scale=1.0):
    """Example 1 FIO kernel exp(2 pi i Phi(x, xi)); x in [0,1)^2 grid, xi integer."""

    def K(x, xi):
        x = np.asarray(x, dtype=np.float64)
        xi = np.asarray(xi, dtype=np.float64)
        # x . xi = (n1 xi1 + n2 xi2) / n with integer n1, n2, xi: reduce mod n.
        n1 = np.rint(x * n).astype(np.int64)
        xi_i = np.rint(xi).astype(np.int64)
        k = (np.outer(n1[:, 0], xi_i[:, 0]) + np.outer(n1[:, 1], xi_i[:, 1])) % n
        lin = k.astype(np.float64) / n
        s1 = np.sin(2 * np.pi * x[:, 0])
        s2 = np.sin(2 * np.pi * x[:, 1])
        co1 = np.cos(2 * np.pi * x[:, 0])
        co2 = np.cos(2 * np.pi * x[:, 1])
        c1 = c_scale * (2.0 + s1 * s2) / 16.0
        c2 = c_scale * (2.0 + co1 * co2) / 16.0
        rad = np.sqrt(np.outer(c1 * c1, xi[:, 0] ** 2) + np.outer(c2 * c2, xi[:, 1] ** 2))
        return np.exp(2j * np.pi * (lin + rad))

    return K


def fio_points(c_scale=1.0):
    """Example 1 FIO kernel exp(2 pi i Phi(x, xi)) of eq. (example1phi) for
    arbitrary real points x and xi (general point sets): the phase is
    evaluated directly, without the grid's exact reduction of x . xi."""
    Phi = fio_phase(c_scale)

    def K(x, xi):
        ph = Phi(x, xi)
        return np.exp(2j * np.pi * (ph - np.floor(ph)))

    return K


def restrict(K, x, xi):
    """Entry function over index sets: f(I, J) = K(x[I], xi[J])."""

    def f(I, J):
        return K(x[np.asarray(I)], xi[np.asarray(J)])

    return f
