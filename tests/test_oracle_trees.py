"""Pins of the oracle's trees, polar map and corona split (CPU only)."""

import os

import numpy as np
import pytest

import mbf_workloads as W
from oracle import kernels, trees

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_zorder_matches_figure_1():
    with open(os.path.join(GOLD, "fig1_zorder.txt")) as f:
        rows = [[int(v) for v in ln.split()] for ln in f if ln.strip() and not ln.startswith("#")]
    lvl1, lvl2 = np.array(rows[:2]), np.array(rows[2:])
    c1, c2 = np.meshgrid(np.arange(2), np.arange(2), indexing="ij")
    np.testing.assert_array_equal(trees.morton(c1, c2, 1), lvl1)
    c1, c2 = np.meshgrid(np.arange(4), np.arange(4), indexing="ij")
    np.testing.assert_array_equal(trees.morton(c1, c2, 2), lvl2)


@pytest.mark.parametrize("n,depth", [(8, 3), (16, 2), (16, 4)])
def test_quadtree_children_partition_parent(n, depth):
    x = W.grid_x_integer(n)
    t = trees.QuadTree(x, (0, 0), n, depth)
    for lev in range(depth):
        assert len(t.nodes[lev]) == 4 ** lev
        for c in t.nodes[lev]:
            pts = set(t.points(lev, int(c)).tolist())
            kids = t.children(lev, int(c))
            assert kids == [4 * int(c) + k for k in range(4)]
            union = set()
            for k in kids:
                r0, r1 = t.child_rows(lev, int(c), k)
                sub = t.points(lev, int(c))[r0:r1]
                np.testing.assert_array_equal(np.sort(sub), np.sort(t.points(lev + 1, k)))
                union |= set(sub.tolist())
            assert union == pts
    # each leaf is a square of (n / 2^depth)^2 grid points
    side = n >> depth
    for c in t.nodes[depth]:
        p = x[t.points(depth, int(c))]
        assert p.shape[0] == side * side
        assert np.ptp(p[:, 0]) == side - 1 and np.ptp(p[:, 1]) == side - 1


def test_polar_map_inverts_and_preserves_kernel():
    n = 32
    xi = W.grid_omega(n)
    p = trees.polar_map(xi, n)
    assert np.all(p >= 0.0) and np.all(p <= 1.0)
    np.testing.assert_allclose(trees.polar_inverse(p, n), xi, atol=1e-10)
    # Psi(x, p) = Phi(x, xi(p)) / n = (sqrt 2 / 2) Phi(x, (cos, sin)) p1 (Section 3.1)
    x = W.grid_x_unit(8)
    Phi = kernels.fio_phase()
    d = np.stack([np.cos(2 * np.pi * p[:, 1]), np.sin(2 * np.pi * p[:, 1])], axis=1)
    psi = np.sqrt(2.0) / 2.0 * Phi(x, d) * p[None, :, 0]
    np.testing.assert_allclose(n * psi, Phi(x, xi), atol=1e-9)


@pytest.mark.parametrize("n", [64, 128, 256, 1024])
def test_corona_split_partitions_grid(n):
    xi = W.grid_omega(n)
    cor, center = trees.coronas(xi, n, center_side=16)
    allidx = np.concatenate([c[2] for c in cor] + [center])
    assert allidx.size == n * n
    assert np.unique(allidx).size == n * n
    assert center.size == 256
    assert len(cor) == int(np.log2(n)) - 5 + 1  # t = 0 .. log2 n - s with s = 5
    for t, a, idx in cor:
        assert a == n / 2 ** (t + 1)
        assert idx.size == (2 * a) ** 2 - a ** 2
        m = np.max(np.abs(xi[idx]), axis=1)
        assert np.all(m >= a / 2) and np.all(m <= a)
        # 1/4 of the level-2 nodes of the bounding-square tree are empty (Section 4.2)
        tr = trees.QuadTree(xi[idx], (-a, -a), 2 * a, 2)
        assert len(tr.nodes[2]) == 12
