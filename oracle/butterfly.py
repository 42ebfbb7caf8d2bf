"""Butterfly factorization build / apply / adjoint in FP64 (test infrastructure).

Follows Section 2 of the paper, in its order and notation:

* Middle level (Section 2.3): for every pair (A at level h of T_X,
  B at level L-h of T_Omega), K_{A,B} ~ U_{A,B} S_{A,B} V_{B,A}^* in
  form 1 (eq. (lowrank1), eq. (Kij)); h = floor(L/2) (even L in the paper;
  odd L read as floor).
* Recursive factorization of U (Section 2.4.1, eq. (blockF), eq. (RSh2)):
  split the rows of U^l_{A,B} by the four children of A, merge the blocks
  of the children of a level-(L-l-1) node B' side by side, truncate in
  form 2 (eq. (lowrank2)):
      [U_{A, child_0 B'}|_{A_t} ... U_{A, child_3 B'}|_{A_t}] ~ U^{l+1}_{A_t,B'} G^l_{A_t,B'}.
* Recursive factorization of V (Section 2.4.2): the mirror image with the
  roles of T_X and T_Omega exchanged, giving H^l.
* The assembled factorization eq. (gbf):
      K ~ U^L G^{L-1} ... G^h M^h (H^h)^* ... (H^{L-1})^* (V^L)^*
  is applied right to left (Section 2.5: cost = number of nonzeros).

Pair bookkeeping ("stage s"): pairs (A at X-level s, B at Omega-level L-s).
Stage 0 holds one vector per Omega leaf, stage L one per X leaf.

Middle level from entries (case (ii): exact SVD or random sampling) or,
when K is known only through fast products with K and K^*, from products
with zero-padded Gaussian probes (case (i), Section 2.3; PBF-m / MBF-m).

PBF (Section 3.2): the Omega tree is built over p = polar(xi); entries
stay K(x, xi).  MSBF (Section 4.2, eq. (msumd), eq. (f1)): a sum over
coronas of butterfly factorizations plus a dense center block.
"""

import numpy as np

from . import lowrank, trees


class Butterfly:
    """A built factorization; see module docstring for the factor names."""

    def __init__(self, xt, ot, nx, nxi):
        self.xt = xt
        self.ot = ot
        self.L = xt.depth
        self.m = self.L // 2
        self.nx = nx
        self.nxi = nxi
        self.V0 = {}      # Omega leaf b -> V^L_b (|b| x r), columns carry sigma
        self.H = []       # H[s][(b_child, a)]  (r_s(a, b_child) x sum_t r_{s+1}(child_t a, parent))
        self.S = {}       # (a, b) at stage m -> 1 / sigma
        self.G = []       # G[s][(a_child, b')] (r_{s+1} x sum_sigma r_s(parent, child_sigma b'))
        self.UL = {}      # X leaf a -> U^L_a (|a| x r)
        self.rank = []    # rank[s][(a, b)]

    # ------------------------------------------------------------------ build
    @classmethod
    def build(cls, entries, x, xi_tree_pts, xbox, obox, depth, tol, rmax,
              method="sampling", seed=0, nxi=None, matvec=None, probes=None):
        """Build from an entry function ``entries(I, J) = K(x[I], xi[J])``.

        x : X points used for the X tree; xi_tree_pts : Omega points in the
        coordinates the Omega tree partitions (xi itself, or polar(xi));
        xbox / obox : (lo, side) of the root squares; depth : L.

        method "exact" (dense SVD of each middle block), "sampling" (SVD via
        random sampling, case (ii)) or "matvec" (case (i), Section 2.3): the
        middle blocks are known only through ``matvec(adjoint, block)``,
        which returns K block (block: nxi x q) or K^* block (block: nx x q),
        applied to the zero-padded Gaussian probes C^P_B and R^P_A taken
        from ``probes = (C, R)`` (nxi x q and nx x q: C_B = C[B], R_A = R[A]).
        ``entries`` is not used then.
        """
        rng = np.random.default_rng(seed)
        xt = trees.QuadTree(x, xbox[0], xbox[1], depth)
        ot = trees.QuadTree(xi_tree_pts, obox[0], obox[1], depth)
        self = cls(xt, ot, x.shape[0], xi_tree_pts.shape[0])
        L, m = self.L, self.m
        self.rank = [dict() for _ in range(L + 1)]

        if method == "matvec":
            # K C^P_B holds K_{A,B} C_B for every A; K^* R^P_A holds
            # K_{A,B}^* R_A for every B (Section 2.3, case (i)).
            Cp, Rp = probes
            KC, KsR = {}, {}
            for b in ot.nodes[L - m]:
                ib = ot.points(L - m, int(b))
                pad = np.zeros((self.nxi, Cp.shape[1]), complex)
                pad[ib] = Cp[ib]
                KC[int(b)] = matvec(False, pad)
            for a in xt.nodes[m]:
                ia = xt.points(m, int(a))
                pad = np.zeros((self.nx, Rp.shape[1]), complex)
                pad[ia] = Rp[ia]
                KsR[int(a)] = matvec(True, pad)

        # Middle level factorization (Section 2.3), form 1.
        U, V = {}, {}
        for a in xt.nodes[m]:
            ia = xt.points(m, int(a))
            for b in ot.nodes[L - m]:
                ib = ot.points(L - m, int(b))
                a_, b_ = int(a), int(b)
                if method == "exact":
                    U0, s, V0 = lowrank.svd_trunc(entries(ia, ib), tol, rmax)
                elif method == "matvec":
                    U0, s, V0 = lowrank.svd_matvec(KC[b_][ia], KsR[a_][ib], Cp[ib], Rp[ia], tol, rmax)
                else:
                    U0, s, V0 = lowrank.svd_sampling(
                        lambda I, J: entries(ia[I], ib[J]), ia.size, ib.size, tol, rmax, rng)
                Uf, Sf, Vf = lowrank.form1(U0, s, V0)
                U[(a_, b_)] = Uf
                V[(b_, a_)] = Vf
                self.S[(a_, b_)] = Sf
                self.rank[m][(a_, b_)] = s.size

        # Recursive factorization of U (Section 2.4.1): stages m .. L-1.
        self.G = [None] * L
        for s in range(m, L):
            Unew, Gs = {}, {}
            for a in xt.nodes[s]:
                a = int(a)
                for ac in xt.children(s, a):
                    r0, r1 = xt.child_rows(s, a, ac)
                    for bp in ot.nodes[L - s - 1]:
                        bp = int(bp)
                        kids = ot.children(L - s - 1, bp)
                        Wm = np.hstack([U[(a, bk)][r0:r1] for bk in kids])
                        U0, sv, V0 = lowrank.svd_trunc(Wm, tol, rmax)
                        Uf, Gf = lowrank.form2(U0, sv, V0)
                        Unew[(ac, bp)] = Uf
                        Gs[(ac, bp)] = Gf
                        self.rank[s + 1][(ac, bp)] = sv.size
            U = Unew
            self.G[s] = Gs
        root_o = int(ot.nodes[0][0])
        self.UL = {int(a): U[(int(a), root_o)] for a in xt.nodes[L]}

        # Recursive factorization of V (Section 2.4.2): stages m .. 1.
        self.H = [None] * m
        for s in range(m, 0, -1):
            Vnew, Hs = {}, {}
            for b in ot.nodes[L - s]:
                b = int(b)
                for bc in ot.children(L - s, b):
                    r0, r1 = ot.child_rows(L - s, b, bc)
                    for ap in xt.nodes[s - 1]:
                        ap = int(ap)
                        kids = xt.children(s - 1, ap)
                        Wm = np.hstack([V[(b, ak)][r0:r1] for ak in kids])
                        U0, sv, V0 = lowrank.svd_trunc(Wm, tol, rmax)
                        Vf, Hf = lowrank.form2(U0, sv, V0)
                        Vnew[(bc, ap)] = Vf
                        Hs[(bc, ap)] = Hf
                        self.rank[s - 1][(ap, bc)] = sv.size
            V = Vnew
            self.H[s - 1] = Hs
        root_x = int(xt.nodes[0][0])
        self.V0 = {int(b): V[(int(b), root_x)] for b in ot.nodes[L]}
        return self

    # ------------------------------------------------------------------ apply
    def _cols(self, s, a, bp):
        """Column ranges of H[s][(bk, a)]: one run per X child of a (stage s+1 ranks)."""
        out, c = [], 0
        for ak in self.xt.children(s, a):
            r = self.rank[s + 1][(ak, bp)]
            out.append((ak, c, c + r))
            c += r
        return out

    def _gcols(self, s, a, bp):
        """Column ranges of G[s][(ac, bp)]: one run per Omega child of bp (stage s ranks)."""
        L = self.L
        out, c = [], 0
        for bk in self.ot.children(L - s - 1, bp):
            r = self.rank[s][(a, bk)]
            out.append((bk, c, c + r))
            c += r
        return out

    def apply(self, g):
        """u ~ K g through eq. (gbf), right to left."""
        g = np.asarray(g, dtype=np.complex128)
        vec = g.ndim == 1
        if vec:
            g = g[:, None]
        xt, ot, L, m = self.xt, self.ot, self.L, self.m
        root_x = int(xt.nodes[0][0])
        root_o = int(ot.nodes[0][0])
        # (V^L)^*: one vector per Omega leaf.
        y = {(root_x, b): self.V0[b].conj().T @ g[ot.points(L, b)] for b in self.V0}
        # (H^l)^* factors: stages 0 .. m-1.
        for s in range(m):
            ynew = {}
            for a in xt.nodes[s]:
                a = int(a)
                for bp in ot.nodes[L - s - 1]:
                    bp = int(bp)
                    cols = self._cols(s, a, bp)
                    for ak, c0, c1 in cols:
                        acc = np.zeros((c1 - c0, g.shape[1]), complex)
                        for bk in ot.children(L - s - 1, bp):
                            acc += self.H[s][(bk, a)][:, c0:c1].conj().T @ y[(a, bk)]
                        ynew[(ak, bp)] = acc
            y = ynew
        # M^h: the (j,i) -> (i,j) block transpose is the pair relabeling; scale by S.
        z = {k: self.S[k][:, None] * v for k, v in y.items()}
        # G^l factors: stages m .. L-1.
        for s in range(m, L):
            znew = {}
            for a in xt.nodes[s]:
                a = int(a)
                for bp in ot.nodes[L - s - 1]:
                    bp = int(bp)
                    for ac in xt.children(s, a):
                        Gm = self.G[s][(ac, bp)]
                        acc = np.zeros((Gm.shape[0], g.shape[1]), complex)
                        for bk, c0, c1 in self._gcols(s, a, bp):
                            acc += Gm[:, c0:c1] @ z[(a, bk)]
                        znew[(ac, bp)] = acc
            z = znew
        u = np.zeros((self.nx, g.shape[1]), complex)
        for a, Um in self.UL.items():
            u[xt.points(L, a)] = Um @ z[(a, root_o)]
        return u[:, 0] if vec else u

    def adjoint(self, h):
        """v ~ K^* h: the chain of eq. (gbf) reversed with conjugate transposes."""
        h = np.asarray(h, dtype=np.complex128)
        vec = h.ndim == 1
        if vec:
            h = h[:, None]
        xt, ot, L, m = self.xt, self.ot, self.L, self.m
        root_x = int(xt.nodes[0][0])
        root_o = int(ot.nodes[0][0])
        z = {(a, root_o): Um.conj().T @ h[xt.points(L, a)] for a, Um in self.UL.items()}
        for s in range(L - 1, m - 1, -1):
            znew = {}
            for a in xt.nodes[s]:
                a = int(a)
                for bp in ot.nodes[L - s - 1]:
                    bp = int(bp)
                    gc = self._gcols(s, a, bp)
                    for bk, c0, c1 in gc:
                        acc = np.zeros((c1 - c0, h.shape[1]), complex)
                        for ac in xt.children(s, a):
                            acc += self.G[s][(ac, bp)][:, c0:c1].conj().T @ z[(ac, bp)]
                        znew[(a, bk)] = acc
            z = znew
        y = {k: self.S[k][:, None] * v for k, v in z.items()}
        for s in range(m - 1, -1, -1):
            ynew = {}
            for a in xt.nodes[s]:
                a = int(a)
                for bp in ot.nodes[L - s - 1]:
                    bp = int(bp)
                    cols = self._cols(s, a, bp)
                    for bk in ot.children(L - s - 1, bp):
                        Hm = self.H[s][(bk, a)]
                        acc = np.zeros((Hm.shape[0], h.shape[1]), complex)
                        for ak, c0, c1 in cols:
                            acc += Hm[:, c0:c1] @ y[(ak, bp)]
                        ynew[(a, bk)] = acc
            y = ynew
        v = np.zeros((self.nxi, h.shape[1]), complex)
        for b, Vm in self.V0.items():
            v[ot.points(L, b)] = Vm @ y[(root_x, b)]
        return v[:, 0] if vec else v

    # ------------------------------------------------------------ accounting
    def nnz(self):
        """Nonzeros of all factors (Section 2.5: the apply cost per vector)."""
        t = sum(v.size for v in self.V0.values()) + sum(u.size for u in self.UL.values())
        t += sum(sum(x.size for x in Hs.values()) for Hs in self.H)
        t += sum(sum(x.size for x in Gs.values()) for Gs in self.G[self.m:])
        t += sum(x.size for x in self.S.values())
        return t

    def max_rank(self):
        return [max(d.values()) if d else 0 for d in self.rank]


class Multiscale:
    """MSBF (Section 4.2): K ~ K_C R_C + sum_t BF_t R_t (eq. (f1))."""

    def __init__(self, parts, center_idx, KC, nx, nxi):
        self.parts = parts          # list of (t, idx_t, Butterfly)
        self.center_idx = center_idx
        self.KC = KC                # dense N_x x |Omega_C|
        self.nx = nx
        self.nxi = nxi

    def apply(self, g):
        g = np.asarray(g, dtype=np.complex128)
        u = self.KC @ g[self.center_idx]
        for _, idx, bf in self.parts:
            u = u + bf.apply(g[idx])
        return u

    def adjoint(self, h):
        h = np.asarray(h, dtype=np.complex128)
        shape = (self.nxi,) + h.shape[1:]
        v = np.zeros(shape, complex)
        v[self.center_idx] = self.KC.conj().T @ h
        for _, idx, bf in self.parts:
            v[idx] = bf.adjoint(h)
        return v

    def nnz(self):
        return self.KC.size + sum(bf.nnz() for _, _, bf in self.parts)


def corona_depth(n, t, leaf_side=1):
    """L_t = 2 floor((L - t) / 2) (Section 4.2) with L = log2(n / leaf_side)."""
    L = int(round(np.log2(n / leaf_side)))
    return max(2 * ((L - t) // 2), 0)


def _restrict(matvec, idx, nxi):
    """The black box of K restricted to the Omega columns idx: K[:, idx] B
    is K applied to B padded with zeros, (K[:, idx])^* B the rows idx of K^* B."""
    def mv(adjoint, block):
        if adjoint:
            return matvec(True, block)[idx]
        full = np.zeros((nxi, block.shape[1]), complex)
        full[idx] = block
        return matvec(False, full)
    return mv


def build_multiscale(K, x, xi, n, xbox, tol, rmax, center_side=16, leaf_side=1,
                     method="sampling", seed=0, matvec=None, probes=None):
    """MSBF build: corona split, one butterfly per corona, dense center.

    method "matvec" (MBF-m): K is not used; each corona's butterfly is built
    from ``matvec`` restricted to its columns (probes restricted likewise)
    and the dense center K_C is K applied to the unit vectors of Omega_C."""
    cor, center = trees.coronas(xi, n, center_side)
    parts = []
    for t, a, idx in cor:
        Lt = corona_depth(n, t, leaf_side)
        xs = xi[idx]
        if method == "matvec":
            bf = Butterfly.build(None, x, xs, xbox, ((-a, -a), 2 * a), Lt, tol, rmax, method="matvec",
                                 nxi=idx.size, matvec=_restrict(matvec, idx, xi.shape[0]),
                                 probes=(probes[0][idx], probes[1]))
        else:
            ent = (lambda xs_: (lambda I, J: K(x[I], xs_[J])))(xs)
            bf = Butterfly.build(ent, x, xs, xbox, ((-a, -a), 2 * a), Lt, tol, rmax,
                                 method=method, seed=seed + 101 * t, nxi=idx.size)
        parts.append((t, idx, bf))
    if method == "matvec":
        E = np.zeros((xi.shape[0], center.size), complex)
        E[center, np.arange(center.size)] = 1.0
        KC = matvec(False, E)
    else:
        KC = K(x, xi[center])
    return Multiscale(parts, center, KC, x.shape[0], xi.shape[0])


def build_polar(K, x, xi, n, xbox, depth, tol, rmax, method="sampling", seed=0, matvec=None, probes=None):
    """PBF build (Section 3.2): Omega tree over p = polar(xi) in [0,1]^2
    (PBF-m with method "matvec": K is not used)."""
    p = trees.polar_map(xi, n)
    ent = None if K is None else (lambda I, J: K(x[I], xi[J]))
    return Butterfly.build(ent, x, p, xbox, ((0.0, 0.0), 1.0), depth, tol, rmax,
                           method=method, seed=seed, matvec=matvec, probes=probes)


def build_plain(K, x, xi, xbox, obox, depth, tol, rmax, method="sampling", seed=0, matvec=None, probes=None):
    """BF build on the original Omega (Section 2)."""
    ent = None if K is None else (lambda I, J: K(x[I], xi[J]))
    return Butterfly.build(ent, x, xi, xbox, obox, depth, tol, rmax, method=method, seed=seed,
                           matvec=matvec, probes=probes)
