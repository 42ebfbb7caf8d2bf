"""Parity bars of the GPU tests, checked column by column and entry by entry.

For every right-hand side (column) j of a result block:
  * relative l2 error  ||got_j - ref_j|| / ||ref_j||  <= bar, and
  * every entry        |got_ij - ref_ij| <= 4 bar * max_i |ref_ij|.
One bad column among many therefore fails the check, however small its
share of the whole block's norm.

Why 4 bar per entry: an output entry is a sum of up to 4096 products (the
longest reductions are stage blocks of 4 x 1024 inputs and 1024-point
leaves).  Rounded in FP32 (unit roundoff 6e-8), such a sum carries an error
of order sqrt(K) u, up to 4e-6 of its scale at K = 4096, so a single entry
can exceed the l2 bar by that factor while its column stays within it.  The
bound still flags any entry that is wrong beyond rounding.
"""

import numpy as np


def column_errors(got, ref):
    got = np.asarray(got, np.complex128)
    ref = np.asarray(ref, np.complex128)
    if got.ndim == 1:
        got, ref = got[:, None], ref[:, None]
    assert got.shape == ref.shape, (got.shape, ref.shape)
    diff = got - ref
    den = np.linalg.norm(ref, axis=0)
    col = np.linalg.norm(diff, axis=0) / np.where(den > 0, den, 1.0)
    amax = np.abs(ref).max(axis=0)
    ent = np.abs(diff).max(axis=0) / np.where(amax > 0, amax, 1.0)
    return col, ent


ENTRY_FACTOR = 4.0


def assert_columns_close(got, ref, bar, what=""):
    col, ent = column_errors(got, ref)
    j = int(np.argmax(col))
    assert col[j] <= bar, "%s: column %d relative l2 error %.3e > %.1e" % (what, j, col[j], bar)
    k = int(np.argmax(ent))
    eb = ENTRY_FACTOR * bar
    assert ent[k] <= eb, "%s: column %d worst entry error / column max %.3e > %.1e" % (what, k, ent[k], eb)
