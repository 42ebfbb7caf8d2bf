"""Pins of the oracle's butterfly factorization in three dimensions (CPU).

The construction carries over to d > 2 with 2^d-ary trees (the paper's
closing remarks); here for the 3D DFT K(x, xi) = exp(-2 pi i x.xi / n) on
x in {0..n-1}^3, xi in {-n/2..n/2-1}^3:

* Z-order of octree cells (first coordinate most significant) against
  hand-computed codes; every node's points inside its box;
* the kernel against the closed form fftn (brute force on small n);
* at full rank the factorization reproduces the dense kernel, forward and
  adjoint (several depths, odd and even L);
* at a tolerance it matches the fftn closed form within a small multiple of
  it, and a planted mistake in the child order breaks the full-rank pin.
"""

import numpy as np
import pytest

import mbf_workloads as W
from oracle import butterfly, direct, kernels, trees


def test_octree_morton_codes_by_hand():
    cells = np.array([[0, 0, 0], [0, 0, 1], [0, 1, 0], [1, 0, 0], [1, 1, 1]])
    np.testing.assert_array_equal(trees.morton_nd(cells, 1), [0, 1, 2, 4, 7])
    # level 2: bit 1 of the first coordinate is bit 1*3 + 2 = 5
    cells2 = np.array([[2, 0, 0], [0, 2, 0], [0, 0, 2], [3, 3, 3], [1, 2, 3]])
    np.testing.assert_array_equal(trees.morton_nd(cells2, 2), [32, 16, 8, 63, 0b100 | 0b001 | 0b010000 | 0b001000])
    # d = 2 agrees with the quadtree's numbering
    c = np.array([[0, 1], [1, 0], [3, 2], [2, 3]])
    np.testing.assert_array_equal(trees.morton_nd(c, 2), trees.morton(c[:, 0], c[:, 1], 2))


def test_octree_nodes_hold_their_points():
    n, L = 8, 2
    x = W.grid_integer_nd(n, 3)
    t = trees.QuadTree(x, (0, 0, 0), n, L)
    assert t.dim == 3 and len(t.nodes[L]) == 64 and len(t.nodes[1]) == 8
    for lev in range(L + 1):
        w = n >> lev
        for code in t.nodes[lev]:
            pts = x[t.points(lev, int(code))]
            assert pts.shape[0] == w ** 3
            assert np.all(pts.max(axis=0) - pts.min(axis=0) == w - 1)  # one box of side w
        if lev < L:
            for code in t.nodes[lev]:
                assert t.children(lev, int(code)) == [8 * int(code) + k for k in range(8)]


@pytest.mark.parametrize("n", [4, 8])
def test_3d_dft_kernel_is_the_fftn_closed_form(n):
    x, xi = W.grid_integer_nd(n, 3), W.grid_omega_nd(n, 3)
    g = W.rhs(n ** 3, 2, seed=1)
    assert direct.rel_err(kernels.dft(n)(x, xi) @ g, direct.dft_fftn(n, 3, g)) < 1e-12


def _bf3(n, L, tol, rmax=10 ** 6):
    x, xi = W.grid_integer_nd(n, 3), W.grid_omega_nd(n, 3)
    return butterfly.build_plain(kernels.dft(n), x, xi, ((0, 0, 0), n), ((-n / 2,) * 3, n), L, tol, rmax,
                                 method="exact")


@pytest.mark.parametrize("n,L", [(4, 1), (4, 2), (8, 2), (8, 3)])
def test_full_rank_3d_factorization_equals_dense(n, L):
    bf = _bf3(n, L, 1e-14)
    x, xi = W.grid_integer_nd(n, 3), W.grid_omega_nd(n, 3)
    Kd = kernels.dft(n)(x, xi)
    g, h = W.rhs(n ** 3, 3, seed=2), W.rhs(n ** 3, 3, seed=3)
    assert direct.rel_err(bf.apply(g), Kd @ g) < 1e-12
    assert direct.rel_err(bf.adjoint(h), Kd.conj().T @ h) < 1e-12


def test_3d_factorization_at_a_tolerance_matches_fftn():
    n = 8
    bf = _bf3(n, 3, 1e-9)
    g = W.rhs(n ** 3, 4, seed=4)
    assert direct.rel_err(bf.apply(g), direct.dft_fftn(n, 3, g)) < 1e-7


def test_planted_child_order_breaks_the_3d_pin(monkeypatch):
    orig = trees.QuadTree.children

    def swapped(self, level, code):
        kids = orig(self, level, code)
        return kids[1:2] + kids[:1] + kids[2:] if self.dim == 3 and len(kids) > 1 else kids

    monkeypatch.setattr(trees.QuadTree, "children", swapped)
    bf = _bf3(4, 2, 1e-14)
    monkeypatch.setattr(trees.QuadTree, "children", orig)
    x, xi = W.grid_integer_nd(4, 3), W.grid_omega_nd(4, 3)
    g = W.rhs(64, 2, seed=5)
    assert direct.rel_err(bf.apply(g), kernels.dft(4)(x, xi) @ g) > 1e-3
