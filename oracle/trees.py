"""Quadtrees, the polar map and the corona split (test infrastructure).

* Quadtree (Section 2.2, Fig. 1): a square box is split recursively into
  2 x 2 children; the nodes of a level are numbered along the Z-order
  (Morton) curve, and node i of level l has children 4i + t, t = 0..3.
  Reading of Fig. 1: the first coordinate x1 is the more significant bit,
  t = 2 * [x1 in upper half] + [x2 in upper half].  Boxes are half-open,
  the last cell of each axis closed.  Nodes holding no point are dropped
  (Section 2.6).
* Polar map (Section 3.1, eq. (polar)):
  xi = (sqrt(2)/2) n p1 (cos 2 pi p2, sin 2 pi p2), p in [0,1]^2.
  The inverse used here is p1 = |xi| / R, p2 = atan2(xi2, xi1) / (2 pi) mod 1
  with R = (sqrt(2)/2) n; p(0) = (0, 0); p1 clamped to [0, 1].
* Corona split (Section 4.1, eq. (domaindecomp)) under the half-open
  reading: Omega_t = [-a_t, a_t)^2 minus [-a_t/2, a_t/2)^2, a_t = n / 2^(t+1),
  for t = 0..T with a_T / 2 = center_side / 2; Omega_C = [-c/2, c/2)^2.
"""

import numpy as np


def morton_nd(cells, level):
    """Z-order index of d-dimensional cells (rows of ``cells``, shape (m, d))
    at the given level: bit b of coordinate k goes to bit b d + (d - 1 - k),
    so the first coordinate is the most significant (d = 2: ``morton``)."""
    cells = np.asarray(cells, dtype=np.int64)
    d = cells.shape[1]
    code = np.zeros(cells.shape[0], dtype=np.int64)
    for b in range(level):
        for k in range(d):
            code |= ((cells[:, k] >> b) & 1) << (b * d + d - 1 - k)
    return code


def morton(c1, c2, level):
    """Z-order index of cell (c1, c2) at the given level, c1 more significant."""
    c1 = np.asarray(c1, dtype=np.int64)
    c2 = np.asarray(c2, dtype=np.int64)
    code = np.zeros(np.broadcast(c1, c2).shape, dtype=np.int64)
    for b in range(level):
        code |= ((c1 >> b) & 1) << (2 * b + 1)
        code |= ((c2 >> b) & 1) << (2 * b)
    return code


class QuadTree:
    """Quadtree of a 2D point set inside the box [lo, lo + side)^2 (for points
    of d coordinates, the same 2^d-ary tree over [lo, lo + side)^d: an octree
    for d = 3, children numbered like ``morton_nd``).

    Attributes
    ----------
    depth : number of levels below the root (leaves at level ``depth``).
    order : point indices sorted by leaf Morton code, then by index; every
            node covers a contiguous run ``order[start:end]``.
    nodes[l] : sorted Morton codes of the nonempty nodes at level l.
    span[l] : dict code -> (start, end) into ``order``.
    """

    def __init__(self, pts, lo, side, depth):
        pts = np.asarray(pts, dtype=np.float64)
        self.depth = int(depth)
        self.npts = pts.shape[0]
        self.dim = pts.shape[1]
        lo = np.asarray(lo, dtype=np.float64)
        nl = 1 << self.depth
        t = (pts - lo[None, :]) / float(side)
        c = np.floor(t * nl).astype(np.int64)
        c = np.clip(c, 0, nl - 1)
        self.leaf_code = morton(c[:, 0], c[:, 1], self.depth) if self.dim == 2 else morton_nd(c, self.depth)
        self.order = np.lexsort((np.arange(self.npts), self.leaf_code))
        sorted_codes = self.leaf_code[self.order]
        self.nodes = []
        self.span = []
        for lev in range(self.depth + 1):
            codes = sorted_codes >> (self.dim * (self.depth - lev))
            uniq, first = np.unique(codes, return_index=True)
            ends = np.append(first[1:], self.npts)
            self.nodes.append(uniq)
            self.span.append({int(u): (int(s), int(e)) for u, s, e in zip(uniq, first, ends)})

    def points(self, level, code):
        s, e = self.span[level][code]
        return self.order[s:e]

    def children(self, level, code):
        """Nonempty children (codes at level+1) of node ``code`` in Z-order."""
        sp = self.span[level + 1]
        nc = 1 << self.dim
        return [nc * code + t for t in range(nc) if (nc * code + t) in sp]

    def child_rows(self, level, code, child):
        """Row range of ``child`` (level+1) inside the point list of ``code``."""
        s, _ = self.span[level][code]
        cs, ce = self.span[level + 1][child]
        return cs - s, ce - s


def polar_map(xi, n):
    """p(xi) of eq. (polar): (|xi| / R, angle / 2 pi mod 1), R = sqrt(2)/2 n."""
    xi = np.asarray(xi, dtype=np.float64)
    R = np.sqrt(2.0) / 2.0 * n
    p1 = np.hypot(xi[:, 0], xi[:, 1]) / R
    p2 = np.arctan2(xi[:, 1], xi[:, 0]) / (2.0 * np.pi)
    p2 = np.mod(p2, 1.0)
    zero = (xi[:, 0] == 0) & (xi[:, 1] == 0)
    p2[zero] = 0.0
    p1 = np.clip(p1, 0.0, 1.0)
    return np.stack([p1, p2], axis=1)


def polar_inverse(p, n):
    """xi(p) of eq. (polar)."""
    p = np.asarray(p, dtype=np.float64)
    R = np.sqrt(2.0) / 2.0 * n
    return np.stack([R * p[:, 0] * np.cos(2 * np.pi * p[:, 1]),
                     R * p[:, 0] * np.sin(2 * np.pi * p[:, 1])], axis=1)


def coronas(xi, n, center_side=16):
    """Corona split of an integer frequency grid.

    Returns (list of (t, a_t, index array of Omega_t), index array of Omega_C).
    Omega_t = {xi in [-a_t, a_t)^2} minus {xi in [-a_t/2, a_t/2)^2}.
    """
    xi = np.asarray(xi, dtype=np.float64)

    def inbox(a):
        return np.all((xi >= -a) & (xi < a), axis=1)

    out = []
    t = 0
    a = n / 2.0
    while a / 2.0 >= center_side / 2.0 and a > center_side / 2.0:
        idx = np.nonzero(inbox(a) & ~inbox(a / 2.0))[0]
        out.append((t, a, idx))
        t += 1
        a /= 2.0
    center = np.nonzero(inbox(a))[0]
    return out, center
