"""Pins of the oracle's bookkeeping (CPU only).

* corona depth L_t of the multiscale split (Section 4.2, Factorization step)
  against values worked out by hand from the rule L_t = 2 floor((L - t) / 2)
  (tests/golden/corona_depth.txt), plus the properties the rule implies:
  every L_t is even, L - t - 1 <= L_t <= L - t, and a corona's Omega tree
  ends in leaves of one or 2 x 2 grid points when the full tree has
  one-point leaves;
* number of nonzeros of a factorization (Section 2.5: the apply cost)
  counted by hand on factorizations whose ranks are fixed by the kernel
  (DFT blocks with orthogonal columns), for a plain factorization and for a
  multiscale one (dense center + a depth-0 corona factorization);
* planted mistakes in the depth rule make the pins fail.
"""

import os

import numpy as np
import pytest

import mbf_workloads as W
from oracle import butterfly, direct, kernels, trees

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden_depths():
    rows = []
    for line in open(os.path.join(HERE, "golden", "corona_depth.txt")):
        if line.strip() and not line.startswith("#"):
            rows.append(tuple(int(v) for v in line.split()))
    return rows


def _check_depths(fn):
    for n, leaf, t, want in _golden_depths():
        assert fn(n, t, leaf) == want, (n, leaf, t)


def test_corona_depth_golden_values():
    rows = _golden_depths()
    assert len(rows) == 27
    _check_depths(butterfly.corona_depth)


@pytest.mark.parametrize("n", [32, 64, 128, 256, 512, 1024])
def test_corona_depth_properties(n):
    L = int(np.log2(n))
    for t in range(L + 1):
        Lt = butterfly.corona_depth(n, t, 1)
        assert Lt % 2 == 0
        assert L - t - 1 <= Lt <= L - t
        # corona t spans a square of side a_t = n / 2^t grid points; its
        # tree of depth L_t has leaves of side a_t / 2^L_t = 1 or 2 points
        side = (n >> t) >> Lt
        assert side in (1, 2)


def test_planted_depth_mistakes_are_caught(monkeypatch):
    # depth L - t without rounding down to an even number
    odd = lambda n, t, leaf=1: int(round(np.log2(n / leaf))) - t
    with pytest.raises(AssertionError):
        _check_depths(odd)
    # L taken from the grid side instead of the number of leaf cells
    from_n = lambda n, t, leaf=1: max(2 * ((int(round(np.log2(n))) - t) // 2), 0)
    with pytest.raises(AssertionError):
        _check_depths(from_n)
    # off by one corona
    shifted = lambda n, t, leaf=1: max(2 * ((int(round(np.log2(n / leaf))) - t - 1) // 2), 0)
    with pytest.raises(AssertionError):
        _check_depths(shifted)


def _dft_exact(n, leaf):
    x, xi = W.grid_x_integer(n), W.grid_omega(n)
    L = int(np.log2(n // leaf))
    return butterfly.build_plain(kernels.dft(n), x, xi, ((0, 0), n), ((-n / 2, -n / 2), n), L,
                                 1e-14, 10 ** 6, method="exact")


def test_nnz_hand_count_n2_one_point_leaves():
    """n = 2, L = 1, h = 0: four one-point leaves on each side.
    Middle pairs (X root, Omega leaf): 4 x 1 columns, rank 1 each.
      V^L: 4 leaves x (1 x 1)            =  4
      S:   4 pairs x 1                   =  4
      G^0: 4 X children x (1 x 4)        = 16
      U^L: 4 leaves x (1 x 1)            =  4
    total 28."""
    bf = _dft_exact(2, 1)
    assert bf.L == 1 and bf.m == 0
    assert bf.nnz() == 28


def test_nnz_hand_count_n4_leaf_side_2():
    """n = 4, L = 1, h = 0: four 2 x 2 leaves on each side.
    Middle pairs (X root, Omega leaf): 16 x 4 columns of the DFT, which are
    orthogonal, so rank 4 each.
      V^L: 4 leaves x (4 x 4)            =  64
      S:   4 pairs x 4                   =  16
      G^0: 4 X children x (4 x 16)       = 256   (4 rows of the unitary DFT: rank 4)
      U^L: 4 leaves x (4 x 4)            =  64
    total 400."""
    bf = _dft_exact(4, 2)
    assert bf.max_rank() == [4, 4]
    assert bf.nnz() == 400


def test_multiscale_nnz_hand_count_and_depth_zero_part():
    """DFT kernel, n = 32, center 16 x 16, leaf side 32 (so L = 0):
    one corona Omega_0 = [-16,16)^2 minus [-8,8)^2 (768 points), center 256
    points.  The depth-0 factorization of K(X, Omega_0) (1024 x 768,
    orthogonal columns, rank 768) holds V (768 x 768), S (768) and U
    (1024 x 768); the dense center K_C is 1024 x 256.
    total 589824 + 768 + 786432 + 262144 = 1639168."""
    n = 32
    x, xi = W.grid_x_integer(n), W.grid_omega(n)
    K = kernels.dft(n)
    ms = butterfly.build_multiscale(K, x, xi, n, ((0, 0), n), 1e-14, 10 ** 6, center_side=16,
                                    leaf_side=32, method="exact")
    assert [(t, idx.size) for t, idx, _ in ms.parts] == [(0, 768)]
    assert ms.center_idx.size == 256
    assert ms.parts[0][2].L == 0
    assert ms.nnz() == 1639168
    g = W.rhs(n * n, 2, seed=3)
    assert direct.rel_err(ms.apply(g), direct.dft_fft(n, g)) < 1e-12


def test_corona_split_sizes_hand_count():
    """n = 64, center 16: coronas t = 0 ([-32,32)^2 minus [-16,16)^2, 3072
    points) and t = 1 ([-16,16)^2 minus [-8,8)^2, 768 points), center 256."""
    cor, center = trees.coronas(W.grid_omega(64), 64, 16)
    assert [(t, a, idx.size) for t, a, idx in cor] == [(0, 32.0, 3072), (1, 16.0, 768)]
    assert center.size == 256
