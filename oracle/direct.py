"""Plain definition u = K g by direct summation (test infrastructure).

Section 1.1, eq. (kernel): u(x) = sum_{xi in Omega} K(x, xi) g(xi), x in X.
The relative error estimator of Sections 3.3 / 4.3 compares on a set S of
sampled rows; ``direct_rows`` evaluates only those rows.
"""

import numpy as np


def direct(K, x, xi, g, block=2048):
    """u = K g in FP64 for all rows; g has shape (N_xi,) or (N_xi, nrhs)."""
    return direct_rows(K, x, xi, g, np.arange(x.shape[0]), block)


def direct_rows(K, x, xi, g, rows, block=2048):
    """u[rows] = K[rows, :] g in FP64, rows evaluated in blocks."""
    g = np.asarray(g, dtype=np.complex128)
    vec = g.ndim == 1
    if vec:
        g = g[:, None]
    rows = np.asarray(rows)
    out = np.zeros((rows.size, g.shape[1]), dtype=np.complex128)
    for s in range(0, rows.size, block):
        r = rows[s:s + block]
        out[s:s + r.size] = K(x[r], xi) @ g
    return out[:, 0] if vec else out


def dft_fft(n, g):
    """Closed form of the 2D DFT case: u = fft2(ifftshift(G)).

    x = (i1, i2) integer, xi = (j1 - n/2, j2 - n/2), user order row-major;
    K = exp(-2 pi i x.xi / n) is n-periodic in xi, so the sum is the
    standard forward 2D DFT of G after moving xi = 0 to index (0, 0).
    """
    g = np.asarray(g, dtype=np.complex128)
    vec = g.ndim == 1
    if vec:
        g = g[:, None]
    nr = g.shape[1]
    G = g.T.reshape(nr, n, n)
    U = np.fft.fft2(np.fft.ifftshift(G, axes=(1, 2)), axes=(1, 2))
    u = U.reshape(nr, n * n).T
    return u[:, 0] if vec else u


def dft_fftn(n, d, g):
    """Closed form of the d-dimensional DFT case (x in {0..n-1}^d, xi in
    {-n/2..n/2-1}^d, user order row-major): u = fftn(ifftshift(G))."""
    g = np.asarray(g, dtype=np.complex128)
    vec = g.ndim == 1
    if vec:
        g = g[:, None]
    nr = g.shape[1]
    G = g.T.reshape((nr,) + (n,) * d)
    axes = tuple(range(1, d + 1))
    U = np.fft.fftn(np.fft.ifftshift(G, axes=axes), axes=axes)
    u = U.reshape(nr, n ** d).T
    return u[:, 0] if vec else u


def dft_fft_adjoint(n, h):
    """Closed form of K^* h for the 2D DFT case: N * fftshift(ifft2(H))."""
    h = np.asarray(h, dtype=np.complex128)
    vec = h.ndim == 1
    if vec:
        h = h[:, None]
    nr = h.shape[1]
    H = h.T.reshape(nr, n, n)
    V = np.fft.fftshift(np.fft.ifft2(H, axes=(1, 2)), axes=(1, 2)) * (n * n)
    v = V.reshape(nr, n * n).T
    return v[:, 0] if vec else v


def linear_phase_ifft(n, g):
    """Closed form of sum_xi exp(+2 pi i x.xi) g(xi) with x = (n1/n, n2/n).

    This is the FIO of Example 1 with c1 = c2 = 0 (Phi = x . xi), which is
    N times the inverse 2D DFT of G after ifftshift.
    """
    g = np.asarray(g, dtype=np.complex128)
    vec = g.ndim == 1
    if vec:
        g = g[:, None]
    nr = g.shape[1]
    G = g.T.reshape(nr, n, n)
    U = np.fft.ifft2(np.fft.ifftshift(G, axes=(1, 2)), axes=(1, 2)) * (n * n)
    u = U.reshape(nr, n * n).T
    return u[:, 0] if vec else u


class ComposedFIO:
    """Example 2 of Section 3.3 (eq. (example2mfio), eq. (KFK)): the
    composition K~ = K F K of the Example 1 FIO K with the discrete Fourier
    transform F[eta, y] = exp(-2 pi i y . eta) (y in the unit grid X, eta in
    the integer grid Omega), evaluated directly: K and F are formed densely
    from their definitions in FP64 and applied one after the other.
    ``apply(g)`` = K F K g, ``adjoint(h)`` = K^* F^* K^* h."""

    def __init__(self, K, x, xi):
        x = np.asarray(x, dtype=np.float64)
        xi = np.asarray(xi, dtype=np.float64)
        self.K = K(x, xi)
        self.F = np.exp(-2j * np.pi * (np.outer(xi[:, 0], x[:, 0]) + np.outer(xi[:, 1], x[:, 1])))

    def apply(self, g):
        return self.K @ (self.F @ (self.K @ np.asarray(g, dtype=np.complex128)))

    def adjoint(self, h):
        Kh = self.K.conj().T
        return Kh @ (self.F.conj().T @ (Kh @ np.asarray(h, dtype=np.complex128)))

    def matvec(self, adjoint, block):
        """The black box of case (i): K~ block or K~^* block."""
        return self.adjoint(block) if adjoint else self.apply(block)


def rel_err(a, b):
    """sqrt(sum |a-b|^2 / sum |b|^2) (the estimator of Sections 3.3 / 4.3)."""
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.sqrt(np.sum(np.abs(b) ** 2))
    return float(np.sqrt(np.sum(np.abs(a - b) ** 2)) / den) if den > 0 else float(
        np.sqrt(np.sum(np.abs(a - b) ** 2)))
