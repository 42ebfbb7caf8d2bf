"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module holds point sets and random right-hand sides only.  It contains
none of the butterfly method's arithmetic and no kernel evaluation: both the
CPU oracle and the GPU library receive exactly these arrays and compute
everything else on their own.

Point sets follow the uniform grids of the paper (Section 1.1, eq. (X) and
eq. (Omega)):

* X  = {(n1/n, n2/n) : 0 <= n1, n2 < n}      (FIO examples, Section 3.3)
* X' = {(n1, n2)     : 0 <= n1, n2 < n}      (2D DFT with K = exp(-2 pi i x.xi / n))
* Omega = {(n1, n2) : -n/2 <= n1, n2 < n/2}

User order of a grid is row-major with the first coordinate as the row:
index = i1 * n + i2, where i1, i2 are the 0-based grid indices.  RHS blocks
are column-major complex matrices of shape (N, nrhs) with iid standard
normal real and imaginary parts.
"""

import numpy as np


def grid_x_integer(n):
    """Integer X grid {0..n-1}^2 in user order, shape (n*n, 2), float64."""
    i1, i2 = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return np.stack([i1.ravel(), i2.ravel()], axis=1).astype(np.float64)


def grid_x_unit(n):
    """X grid {(n1/n, n2/n)} of [0,1)^2 in user order, shape (n*n, 2)."""
    return grid_x_integer(n) / float(n)


def grid_omega(n):
    """Frequency grid {-n/2..n/2-1}^2 in user order, shape (n*n, 2)."""
    return grid_x_integer(n) - float(n // 2)


def rhs(npts, nrhs, seed=0, dtype=np.complex128):
    """Seeded RHS block (npts x nrhs), column-major (Fortran order)."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal((nrhs, npts))
    im = rng.standard_normal((nrhs, npts))
    g = (re + 1j * im).T.astype(dtype)
    return np.asfortranarray(g)


def sample_rows(npts, k, seed=0):
    """k distinct indices of [0, npts) drawn without replacement (sorted)."""
    rng = np.random.default_rng(seed)
    k = min(k, npts)
    return np.sort(rng.choice(npts, size=k, replace=False))


def poisson_arrivals(nreq, rate_per_s, seed=0):
    """Arrival times (seconds) of a Poisson stream with the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=nreq))


def clustered_points(npts, seed=0, k=5, width=0.08):
    """Non-uniform points of [0,1)^2 (general point sets, Section 2.6): a
    mixture of k Gaussian clusters of the given width around uniformly drawn
    centres, folded into the unit square; shape (npts, 2)."""
    rng = np.random.default_rng(seed)
    centres = rng.random((k, 2))
    which = rng.integers(0, k, size=npts)
    p = centres[which] + width * rng.standard_normal((npts, 2))
    return np.mod(p, 1.0)


def disk_frequencies(npts, radius, seed=0):
    """Non-uniform frequencies in the disk |xi| < radius, denser towards the
    origin (radius drawn as radius * u^2 for uniform u, angle uniform);
    shape (npts, 2)."""
    rng = np.random.default_rng(seed)
    r = radius * rng.random(npts) ** 2
    t = 2.0 * np.pi * rng.random(npts)
    return np.stack([r * np.cos(t), r * np.sin(t)], axis=1)


def grid_integer_nd(n, d):
    """Integer grid {0..n-1}^d in user order (row-major, first coordinate the
    slowest), shape (n**d, d), float64."""
    axes = np.meshgrid(*([np.arange(n)] * d), indexing="ij")
    return np.stack([a.ravel() for a in axes], axis=1).astype(np.float64)


def grid_omega_nd(n, d):
    """Frequency grid {-n/2..n/2-1}^d in user order, shape (n**d, d)."""
    return grid_integer_nd(n, d) - float(n // 2)
