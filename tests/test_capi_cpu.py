"""C-ABI checks that need no GPU: the library loads, exports every entry
point that include/mbf.h declares, rejects invalid arguments before any
device work, and its ready-made kernel callbacks agree with the oracle's
kernel definitions."""

import ctypes
import os
import re

import numpy as np
import pytest

import mbf_workloads as W
import paper_1509_07925_amd as mbf
from oracle import kernels

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mbf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(mbf_[a-z_0-9]+)\s*\(", src))
    return sorted(n for n in names if not n.endswith("_t"))


def test_library_exports_every_declared_symbol():
    lib = mbf.lib()
    names = _declared()
    assert "mbf_apply" in names and "mbf_build" in names and "mbf_apply_adjoint" in names
    for n in names:
        assert hasattr(lib, n), n


def test_invalid_arguments_are_rejected_without_gpu():
    lib = mbf.lib()
    inf = mbf.Info()
    assert lib.mbf_info(None, ctypes.byref(inf)) == -1
    assert lib.mbf_workspace_size(None, 1, 4, None) == -1
    assert lib.mbf_apply(None, 1, 1, None, 1, None, 1, None, 0, None) == -1
    # invalid options are refused before any device work
    n = 8
    x = np.ascontiguousarray(W.grid_x_integer(n))
    with pytest.raises(mbf.MBFError) as e:
        mbf.Factor.build(x, W.grid_omega(n), n, tol=2.0)
    assert e.value.status == -1
    with pytest.raises(mbf.MBFError):
        mbf.Factor.build(x, W.grid_omega(n), n, leaf_side=3)
    with pytest.raises(mbf.MBFError):
        mbf.Factor.build(x, W.grid_omega(n), n, precs=())
    assert "mask" in lib.mbf_last_error().decode()
    # malformed import descriptor
    d = mbf._ImportDesc()
    h = ctypes.c_void_p()
    assert lib.mbf_import(ctypes.byref(d), 2, None, ctypes.byref(h)) == -1


def _call_kernel(name, n, x, xi, rows, cols, c_scale=1.0):
    lib = mbf.lib()
    x = np.ascontiguousarray(x)
    xi = np.ascontiguousarray(xi)
    p = mbf._KParams(n, c_scale, x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                     xi.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    r = np.ascontiguousarray(rows, np.int64)
    c = np.ascontiguousarray(cols, np.int64)
    out = np.zeros(2 * r.size * c.size)
    fn = getattr(lib, name)
    fn.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                   ctypes.c_void_p]
    fn.restype = ctypes.c_int
    assert fn(ctypes.byref(p), r.size, r.ctypes.data, c.size, c.ctypes.data, out.ctypes.data) == 0
    return out.view(np.complex128).reshape(c.size, r.size).T


@pytest.mark.parametrize("n", [8, 64])
def test_builtin_kernels_match_oracle_definitions(n):
    rows = W.sample_rows(n * n, 40, seed=1)
    cols = W.sample_rows(n * n, 30, seed=2)
    x, xi = W.grid_x_integer(n), W.grid_omega(n)
    got = _call_kernel("mbf_kernel_dft", n, x, xi, rows, cols)
    np.testing.assert_allclose(got, kernels.dft(n)(x[rows], xi[cols]), atol=1e-13)
    xu = W.grid_x_unit(n)
    got = _call_kernel("mbf_kernel_fio", n, xu, xi, rows, cols)
    np.testing.assert_allclose(got, kernels.fio_radon(n)(xu[rows], xi[cols]), atol=1e-11)


def test_load_rejects_missing_and_corrupted_files(tmp_path):
    with pytest.raises(mbf.MBFError) as e:
        mbf.Factor.load(str(tmp_path / "missing.mbf"))
    assert e.value.status == -7
    bad = tmp_path / "bad.mbf"
    bad.write_bytes(b"not a factor file at all")
    with pytest.raises(mbf.MBFError) as e:
        mbf.Factor.load(str(bad))
    assert e.value.status == -7
    wrongver = tmp_path / "ver.mbf"
    wrongver.write_bytes(b"MBFFACT1" + (99).to_bytes(4, "little") + bytes(40))
    with pytest.raises(mbf.MBFError) as e:
        mbf.Factor.load(str(wrongver))
    assert "version" in str(e.value)


def test_failing_entry_callback_reports_callback_error_and_leaks_no_handle():
    """A Python entry callback that raises aborts the host build with
    MBF_ERR_CALLBACK; the output handle stays null."""
    lib = mbf.lib()
    n = 8
    x = np.ascontiguousarray(W.grid_x_integer(n))
    xi = np.ascontiguousarray(W.grid_omega(n))
    calls = []

    def bad(rows, cols):
        calls.append(rows.size)
        raise RuntimeError("entry evaluation failed")

    with pytest.raises(mbf.MBFError) as e:
        mbf.Factor.build(x, xi, n, kernel=bad, tol=1e-6, leaf_side=2, builder="host")
    assert e.value.status == -3
    assert calls, "the callback was never reached"
    # the same failure through the raw ABI: the handle is left null
    cb = mbf.ENTRY_CB(lambda user, m, rows, k, cols, out: 7)
    o = mbf._Opts(1e-6, 64, 0, 2, n, 0, 16, 10, 0, 2, 1, 0, 0)
    h = ctypes.c_void_p(12345)
    st = lib.mbf_build(2, x.shape[0], x.ctypes.data, xi.shape[0], xi.ctypes.data, cb, None, ctypes.byref(o), None,
                       ctypes.byref(h))
    assert st == -3
    assert not h.value
    assert "callback" in lib.mbf_last_error().decode()


def test_device_builder_refuses_what_it_cannot_evaluate():
    """The device builder evaluates the ready-made kernels only, at tol >= 1e-7;
    other requests fail with MBF_ERR_UNSUPPORTED before any device work."""
    n = 8
    x, xi = W.grid_x_integer(n), W.grid_omega(n)
    with pytest.raises(mbf.MBFError) as e:
        mbf.Factor.build(x, xi, n, kernel=lambda r, c: np.ones((r.size, c.size)), builder="device")
    assert e.value.status == -5
    with pytest.raises(mbf.MBFError) as e:
        mbf.Factor.build(x, xi, n, kernel="dft", tol=1e-9, builder="device")
    assert e.value.status == -5
    with pytest.raises(KeyError):
        mbf.Factor.build(x, xi, n, builder="somewhere")


# ---------------------------------------------------------------- factor files
# A factor file written by hand in the documented layout (csrc/io.cpp): one
# part of depth 0 over one X point and one Omega point, rank 1, complex64.
# Every corrupted variant must be refused with MBF_ERR_IO while parsing, i.e.
# before any device memory is touched.

def _hash(stream):
    h = 0x84222325cbf29ce4
    mask = (1 << 64) - 1
    pad = stream + bytes((-len(stream)) % 8)
    for i in range(0, len(pad), 8):
        w = int.from_bytes(pad[i:i + 8], "little")
        h = ((h ^ w) * 0x100000001b3) & mask
        h = ((h << 29) | (h >> 35)) & mask
    return h


def _tiny_factor_file(**bad):
    import struct
    f = dict(L=0, m=0, nvl=1, nul=1, mvnp=1, munp=1, mvr=1, mur=1, rows=1, ld=4, vleaf=(0, 0, 1, 1, 0),
             uleaf=(0, 0, 1, 1, 0), vidx=0, uidx=0, s_elems=1, nparts=1)
    f.update(bad)

    def vec(fmt, vals):
        return struct.pack("<Q", len(vals)) + b"".join(struct.pack("<" + fmt, v) for v in vals)

    p = b"MBFFACT1" + struct.pack("<II", 2, 1 << 1) + struct.pack("<qqq", 1, 1, 0) + struct.pack("<I", f["nparts"])
    p += struct.pack("<8i", f["L"], f["m"], f["nvl"], f["nul"], f["mvnp"], f["munp"], f["mvr"], f["mur"])
    p += struct.pack("<7q", 1, 1, 3, 0, 1, 1, f["s_elems"])
    p += vec("q", [f["rows"]]) + vec("q", [f["ld"]]) + vec("q", []) + vec("q", []) + vec("q", [])
    p += vec("i", [1]) + vec("i", []) + vec("i", [])
    p += struct.pack("<q4i", *f["vleaf"]) + struct.pack("<q4i", *f["uleaf"])
    p += struct.pack("<i", f["vidx"]) + struct.pack("<i", f["uidx"])
    p += struct.pack("<ff", 1.0, 0.0) + struct.pack("<ff", 1.0, 0.0) + struct.pack("<f", 1.0)
    return p + b"MBFEND01" + struct.pack("<QQ", len(p), _hash(p))


@pytest.mark.parametrize("bad", [
    dict(ld=0),                      # leading dimension below the state rows
    dict(rows=-1),                   # negative state rows
    dict(vleaf=(5, 0, 1, 1, 0)),     # leaf factor outside the leaf array
    dict(uleaf=(0, 3, 1, 1, 0)),     # leaf points outside the point-index array
    dict(vleaf=(0, 0, 1, 1, 2)),     # leaf state rows outside stage 0
    dict(vidx=7),                    # Omega point index outside [0, nxi)
    dict(uidx=-2),                   # X point index outside [0, nx)
    dict(s_elems=2),                 # middle scaling longer than the middle state
    dict(mvnp=4),                    # leaf maxima that disagree with the leaves
    dict(m=3),                       # middle level deeper than the tree
    dict(nparts=0),                  # no parts
])
def test_load_refuses_inconsistent_factor_files(tmp_path, bad):
    path = tmp_path / "bad.mbf"
    path.write_bytes(_tiny_factor_file(**bad))
    with pytest.raises(mbf.MBFError) as e:
        mbf.Factor.load(str(path))
    assert e.value.status == -7, str(e.value)


def test_hand_written_factor_file_parses(tmp_path):
    """The well-formed tiny file passes every check on the host; without a GPU
    the load then stops at the first device allocation (not an I/O error)."""
    path = tmp_path / "ok.mbf"
    path.write_bytes(_tiny_factor_file())
    try:
        torch = __import__("torch")
        has_gpu = torch.cuda.is_available()
    except ImportError:
        has_gpu = False
    if has_gpu:
        F = mbf.Factor.load(str(path))
        assert F.info().nnz == 3
    else:
        with pytest.raises(mbf.MBFError) as e:
            mbf.Factor.load(str(path))
        assert e.value.status != -7, str(e.value)


def test_column_bar_catches_one_bad_column():
    """The GPU parity check flags a single column 10x over the bar among
    300 correct ones (a whole-block norm would not)."""
    from tests.bars import assert_columns_close
    rng = np.random.default_rng(0)
    ref = rng.standard_normal((500, 300)) + 1j * rng.standard_normal((500, 300))
    got = ref * (1 + 1e-8)
    assert_columns_close(got, ref, 1e-6)
    got[:, 17] = ref[:, 17] * (1 + 1e-5)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-6  # the block norm misses it
    with pytest.raises(AssertionError):
        assert_columns_close(got, ref, 1e-6)
    got = ref.copy()
    got[3, 5] += 1e-3 * np.abs(ref[:, 5]).max()  # one wrong entry
    with pytest.raises(AssertionError):
        assert_columns_close(got, ref, 1e-6)


def test_matvec_build_rejects_bad_options_and_reports_callback_errors():
    """mbf_build_matvec: oversample 0 and the device builder are refused
    before the black box is called; a black box that fails aborts the build
    with MBF_ERR_CALLBACK and leaves the handle null."""
    lib = mbf.lib()
    n = 8
    x = np.ascontiguousarray(W.grid_x_integer(n))
    xi = np.ascontiguousarray(W.grid_omega(n))
    calls = []
    cb = mbf.MATVEC_CB(lambda user, adj, ncols, src, dst: calls.append(adj) or 5)
    h = ctypes.c_void_p(12345)
    o = mbf._Opts(1e-6, 8, 0, 1, n, 0, 16, 0, 0, 2, 1, 0, 0)  # oversample 0
    assert lib.mbf_build_matvec(2, n * n, x.ctypes.data, n * n, xi.ctypes.data, cb, None, ctypes.byref(o), None,
                                None, ctypes.byref(h)) == -1
    assert not h.value
    o = mbf._Opts(1e-6, 8, 0, 1, n, 0, 16, 4, 0, 2, 1, 1, 0)  # device builder
    assert lib.mbf_build_matvec(2, n * n, x.ctypes.data, n * n, xi.ctypes.data, cb, None, ctypes.byref(o), None,
                                None, ctypes.byref(h)) == -5
    assert not calls
    o = mbf._Opts(1e-6, 8, 0, 1, n, 0, 16, 4, 0, 2, 1, 0, 0)
    h = ctypes.c_void_p(12345)
    assert lib.mbf_build_matvec(2, n * n, x.ctypes.data, n * n, xi.ctypes.data, cb, None, ctypes.byref(o), None,
                                None, ctypes.byref(h)) == -3
    assert calls == [0] and not h.value
    assert "matvec callback" in lib.mbf_last_error().decode()


def test_matvec_build_probes_are_zero_padded_gaussians():
    """The library's case (i) products (Section 2.3): one block of q columns
    per middle-level Omega node B holding the given C on the points of B and
    zeros elsewhere (the B cover Omega once), one per middle-level X node A
    holding R likewise.  The host factorization then runs to the end (on a
    machine without a GPU the upload of the factors fails)."""
    n, rmax, os_ = 8, 6, 4
    x, xi = W.grid_x_integer(n), W.grid_omega(n)
    N, q = n * n, rmax + os_
    D = kernels.dft(n)(x, xi)
    rng = np.random.default_rng(0)
    C = rng.standard_normal((N, q)) + 1j * rng.standard_normal((N, q))
    R = rng.standard_normal((N, q)) + 1j * rng.standard_normal((N, q))
    seen = {0: [], 1: []}

    def mv(adj, blk):
        seen[int(adj)].append(np.array(blk))
        return D.conj().T @ blk if adj else D @ blk

    try:
        mbf.Factor.build_matvec(x, xi, n, mv, tol=1e-10, max_rank=rmax, oversample=os_, leaf_side=1, split="none",
                                probes=(C, R), precs=["c128"])
    except mbf.MBFError as e:
        assert e.status in (-2, -4), e
    for adj, P, npts in ((0, C, 4), (1, R, 16)):  # L = 3: Omega level 2 (4 points), X level 1 (16 points)
        blk = np.hstack(seen[adj])
        assert blk.shape[1] % q == 0
        covered = np.zeros(N, int)
        for b in range(blk.shape[1] // q):
            part = blk[:, b * q:(b + 1) * q]
            rows = np.flatnonzero(np.abs(part).sum(axis=1))
            assert rows.size == npts
            np.testing.assert_array_equal(part[rows], P[rows])
            covered[rows] += 1
        assert np.all(covered == 1)


def test_point_set_kernel_matches_oracle_definition():
    """mbf_kernel_fio_points (general point sets) against the oracle's
    direct evaluation of eq. (example1phi) on clustered x and non-grid xi,
    and against the grid kernel on grid points."""
    x = W.clustered_points(300, seed=3)
    xi = W.disk_frequencies(200, 32.0, seed=4)
    rows, cols = np.arange(0, 300, 7), np.arange(0, 200, 3)
    got = _call_kernel("mbf_kernel_fio_points", 0, x, xi, rows, cols)
    np.testing.assert_allclose(got, kernels.fio_points()(x[rows], xi[cols]), atol=1e-11)
    n = 32
    xu, xg = W.grid_x_unit(n), W.grid_omega(n)
    rows, cols = W.sample_rows(n * n, 40, seed=1), W.sample_rows(n * n, 30, seed=2)
    got = _call_kernel("mbf_kernel_fio_points", n, xu, xg, rows, cols)
    np.testing.assert_allclose(got, kernels.fio_radon(n)(xu[rows], xg[cols]), atol=1e-11)


def test_general_point_set_options_and_host_build_without_gpu():
    """grid_n = 0 (general point sets) needs a depth, refuses the multiscale
    split and the device builder before any work; with valid options the
    host build runs its whole factorization (on a machine without a GPU the
    upload of the factors then fails)."""
    x = np.ascontiguousarray(W.clustered_points(256, seed=5))
    xi = np.ascontiguousarray(W.disk_frequencies(256, 8.0, seed=6))
    with pytest.raises(mbf.MBFError) as e:
        mbf.Factor.build(x, xi, 0, kernel="fio_points", depth=0)
    assert e.value.status == -1 and "depth" in str(e.value)
    with pytest.raises(mbf.MBFError) as e:
        mbf.Factor.build(x, xi, 0, kernel="fio_points", depth=3, split="multiscale")
    assert e.value.status == -1
    with pytest.raises(mbf.MBFError) as e:
        mbf.Factor.build(x, xi, 0, kernel="fio_points", depth=3, builder="device")
    assert e.value.status == -5
    for split in ("none", "polar"):
        try:
            mbf.Factor.build(x, xi, 0, kernel="fio_points", depth=3, split=split, tol=1e-8, builder="host")
        except mbf.MBFError as e:
            assert e.status in (-2, -4), e


def test_general_point_sets_refuse_non_finite_coordinates():
    x = np.ascontiguousarray(W.clustered_points(64, seed=7))
    xi = np.ascontiguousarray(W.disk_frequencies(64, 4.0, seed=8))
    for bad_x, bad_xi in ((True, False), (False, True)):
        xb, xib = x.copy(), xi.copy()
        (xb if bad_x else xib)[3, 1] = np.nan
        for split in ("none", "polar"):
            with pytest.raises(mbf.MBFError) as e:
                mbf.Factor.build(xb, xib, 0, kernel="fio_points", depth=2, split=split, builder="host")
            assert e.value.status == -1 and "non-finite" in str(e.value)
