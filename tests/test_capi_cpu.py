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
