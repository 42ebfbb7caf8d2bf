"""Low-rank approximations (Section 2.1) in FP64 (test infrastructure).

Truncation rule (the paper fixes a rank r; tolerance reading): keep the
singular values sigma_k > tol * sigma_1, at most ``rmax`` of them.

SVD via random matrix-vector products (Section 2.1, first option) works
from products with Gaussian matrices only; SVD via random sampling (second
option) from sampled entries.

Three forms of a truncated SVD Z ~ U0 S0 V0^* (eq. (lowrank1)-(lowrank3)):
  form 1: U = U0 S0, S = S0^{-1}, V^* = S0 V0^*
  form 2: U = U0 S0, V^* = V0^*
  form 3: U = U0,    V^* = S0 V0^*
"""

import numpy as np
import scipy.linalg as sla


def _rank(s, tol, rmax):
    if s.size == 0 or s[0] <= 0.0:
        return 0
    r = int(np.count_nonzero(s > tol * s[0]))
    return min(r, int(rmax))


def svd_trunc(Z, tol, rmax):
    """Truncated SVD: returns U0 (m x r), s (r,), V0 (n x r) with Z ~ U0 diag(s) V0^*."""
    Z = np.asarray(Z, dtype=np.complex128)
    if Z.shape[0] == 0 or Z.shape[1] == 0:
        return (np.zeros((Z.shape[0], 0), complex), np.zeros(0), np.zeros((Z.shape[1], 0), complex))
    U, s, Vh = np.linalg.svd(Z, full_matrices=False)
    r = _rank(s, tol, rmax)
    return U[:, :r], s[:r], Vh[:r].conj().T


def _pivot_rank(R, tol, rmax):
    d = np.abs(np.diag(R))
    if d.size == 0 or d[0] <= 0.0:
        return 0
    return min(int(np.count_nonzero(d > tol * d[0])), int(rmax))


def svd_sampling(entries, m, n, tol, rmax, rng, q=None, max_rounds=3, oversample=10):
    """Approximate truncated SVD via random sampling (Section 2.1, case ii).

    ``entries(I, J)`` returns the submatrix Z[I][:, J].  Steps, in the
    order of the paper:
      1. discover representative columns and rows progressively with
         pivoted QR on randomly selected rows / columns, each new set of
         representatives feeding the next selection, until both sets stop
         changing (at most ``max_rounds`` rounds);
      2. orthonormal bases Q_col of Z[:, reps_c] and Q_row of Z[reps_r, :]^*
         by pivoted QR;
      3. M = pinv(Q_col[I_row]) Z[I_row, I_col] pinv(Q_row[I_col]^*), with
         I_row / I_col the representatives plus fresh random indices;
      4. SVD of M:  Z ~ (Q_col U_M) S_M (Q_row V_M)^*, truncated.
    The sample size |I| = O(r) is not fixed by the paper: with ``q=None``
    it starts at 32 and doubles while the rank found reaches q - oversample.
    Returns (U0, s, V0) like ``svd_trunc``.
    """
    if m == 0 or n == 0:
        return (np.zeros((m, 0), complex), np.zeros(0), np.zeros((n, 0), complex))
    if q is None:
        q = 32
        while True:
            out = svd_sampling(entries, m, n, tol, rmax, rng, q, max_rounds, oversample)
            r = out[1].size
            if r + oversample <= q or q >= min(m, n) or r >= rmax:
                return out
            q *= 2
    qr_ = min(q, m)
    qc_ = min(q, n)
    reps_r = np.zeros(0, dtype=np.int64)
    reps_c = np.zeros(0, dtype=np.int64)
    qtol = tol * 1e-2
    for _ in range(max_rounds):
        Ir = np.union1d(reps_r, rng.choice(m, size=qr_, replace=False))
        Zr = entries(Ir, np.arange(n))
        _, R, piv = sla.qr(Zr, mode="economic", pivoting=True)
        new_c = np.sort(piv[:_pivot_rank(R, qtol, min(rmax + 10, n))])
        Ic = np.union1d(new_c, rng.choice(n, size=qc_, replace=False))
        Zc = entries(np.arange(m), Ic)
        _, R, piv = sla.qr(Zc.conj().T, mode="economic", pivoting=True)
        new_r = np.sort(piv[:_pivot_rank(R, qtol, min(rmax + 10, m))])
        stable = np.array_equal(new_c, reps_c) and np.array_equal(new_r, reps_r)
        reps_c, reps_r = new_c, new_r
        if stable:
            break
    if reps_c.size == 0 or reps_r.size == 0:
        return (np.zeros((m, 0), complex), np.zeros(0), np.zeros((n, 0), complex))
    Qc, R, _ = sla.qr(entries(np.arange(m), reps_c), mode="economic", pivoting=True)
    Qc = Qc[:, :max(_pivot_rank(R, qtol * 1e-2, reps_c.size), 1)]
    Qr, R, _ = sla.qr(entries(reps_r, np.arange(n)).conj().T, mode="economic", pivoting=True)
    Qr = Qr[:, :max(_pivot_rank(R, qtol * 1e-2, reps_r.size), 1)]
    Irow = np.union1d(reps_r, rng.choice(m, size=qr_, replace=False))
    Icol = np.union1d(reps_c, rng.choice(n, size=qc_, replace=False))
    Zs = entries(Irow, Icol)
    M = np.linalg.pinv(Qc[Irow]) @ Zs @ np.linalg.pinv(Qr[Icol].conj().T)
    Um, sm, Vmh = np.linalg.svd(M, full_matrices=False)
    r = _rank(sm, tol, rmax)
    return Qc @ Um[:, :r], sm[:r], Qr @ Vmh[:r].conj().T


def svd_matvec(ZC, ZsR, C, R, tol, rmax):
    """Approximate truncated SVD via random matrix-vector products
    (Section 2.1, first option; Section 2.3, case (i)).

    Inputs are the products with Gaussian matrices C (n x q) and R (m x q):
    ZC = Z C (m x q) and ZsR = Z^* R (n x q); Z itself is never formed.
    The probes carry q = r + k columns for the rank r = ``rmax`` and an
    oversampling k > 0.  Steps, in the paper's order:
      1. pivoted QR of ZC and of Z^*R: orthonormal Q_col (m x kc) and
         Q_row (n x kr), kc, kr <= r, spanning the column and row spaces
         (columns kept while the pivot magnitude exceeds tol * 1e-2 of the
         first, at most r of them: the k extra probe columns keep the
         solves of step 2 overdetermined);
      2. M = pinv(R^* Q_col) (R^* Z C) pinv(Q_row^* C), where R^* Z C is
         R^* (ZC);
      3. SVD of M:  Z ~ (Q_col U_M) S_M (Q_row V_M)^*, truncated by ``tol``
         and ``rmax`` like ``svd_trunc``.
    Returns (U0, s, V0) like ``svd_trunc``.
    """
    ZC = np.asarray(ZC, dtype=np.complex128)
    ZsR = np.asarray(ZsR, dtype=np.complex128)
    m, n = ZC.shape[0], ZsR.shape[0]
    if m == 0 or n == 0:
        return (np.zeros((m, 0), complex), np.zeros(0), np.zeros((n, 0), complex))
    qtol = tol * 1e-2
    r_max = min(int(rmax), ZC.shape[1])
    Qc, Rc, _ = sla.qr(ZC, mode="economic", pivoting=True)
    Qc = Qc[:, :max(_pivot_rank(Rc, qtol, min(m, r_max)), 1)]
    Qr, Rr, _ = sla.qr(ZsR, mode="economic", pivoting=True)
    Qr = Qr[:, :max(_pivot_rank(Rr, qtol, min(n, r_max)), 1)]
    RZC = R.conj().T @ ZC
    M = np.linalg.pinv(R.conj().T @ Qc) @ RZC @ np.linalg.pinv(Qr.conj().T @ C)
    Um, sm, Vmh = np.linalg.svd(M, full_matrices=False)
    r = _rank(sm, tol, rmax)
    return Qc @ Um[:, :r], sm[:r], Qr @ Vmh[:r].conj().T


def form1(U0, s, V0):
    """eq. (lowrank1): U = U0 S0, S = S0^{-1}, V = V0 S0 (so V^* = S0 V0^*)."""
    return U0 * s[None, :], 1.0 / s, V0 * s[None, :]


def form2(U0, s, V0):
    """eq. (lowrank2): U = U0 S0, V^* = V0^*."""
    return U0 * s[None, :], V0.conj().T
