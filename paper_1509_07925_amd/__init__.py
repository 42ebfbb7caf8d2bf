"""Python binding of libmbf (argument marshalling only).

Every step of the apply runs in the library's HIP kernels; PyTorch provides
device memory and streams.  The binding loads ``libmbf.so`` from this
directory and raises if it is missing: there is no fallback path.

Vectors are complex column-major matrices (N, nrhs) on the GPU, i.e.
tensors with ``stride(0) == 1`` (e.g. ``torch.empty(nrhs, N).t()``), or
1-D tensors of length N.  Row i follows the caller's point order.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# MBF_LIB selects another build of the library (e.g. the sanitizer build)
LIB_PATH = os.environ.get("MBF_LIB") or os.path.join(_HERE, "libmbf.so")

PREC = {"c128": 0, "c64": 1, "bf16x3": 2}
SPLIT = {"none": 0, "polar": 1, "multiscale": 2}
BUILDER = {"host": 0, "device": 1}

_lib = None


class MBFError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("mbf status %d: %s" % (status, msg))
        self.status = status


class _Opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_rank", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("leaf_side", ctypes.c_int32), ("grid_n", ctypes.c_int32), ("split", ctypes.c_int32),
                ("center_side", ctypes.c_int32), ("oversample", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("prec_mask", ctypes.c_uint32), ("threads", ctypes.c_int32),
                ("builder", ctypes.c_int32), ("device_mem_gb", ctypes.c_int32)]


class _KParams(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("c_scale", ctypes.c_double),
                ("x", ctypes.POINTER(ctypes.c_double)), ("xi", ctypes.POINTER(ctypes.c_double))]


class _ImportDesc(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int32), ("nx", ctypes.c_int64), ("nxi", ctypes.c_int64),
                ("x_leaf_code", ctypes.c_void_p), ("xi_leaf_code", ctypes.c_void_p),
                ("ranks", ctypes.c_void_p), ("v_leaf", ctypes.c_void_p), ("h_blocks", ctypes.c_void_p),
                ("s_mid", ctypes.c_void_p), ("g_blocks", ctypes.c_void_p), ("u_leaf", ctypes.c_void_p)]


class Info(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int32), ("mid", ctypes.c_int32), ("nparts", ctypes.c_int32),
                ("max_rank", ctypes.c_int32 * 33), ("nx", ctypes.c_int64), ("nxi", ctypes.c_int64),
                ("nnz", ctypes.c_int64), ("nnz_stage_max", ctypes.c_int64),
                ("state_rows_max", ctypes.c_int64), ("prec_mask", ctypes.c_uint32),
                ("device_bytes", ctypes.c_size_t)]


class LaunchRecord(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("part", ctypes.c_int32), ("stage", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("ms", ctypes.c_double), ("flops", ctypes.c_double),
                ("bytes", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("requests", ctypes.c_int64), ("rhs", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("max_concurrent_batches", ctypes.c_int64), ("graphs_captured", ctypes.c_int64),
                ("graph_batches", ctypes.c_int64), ("p50_us", ctypes.c_double),
                ("p99_us", ctypes.c_double), ("mean_us", ctypes.c_double), ("wall_s", ctypes.c_double)]


ENTRY_CB = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64),
                            ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double))
MATVEC_CB = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                             ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double))

EXPORTS = ["mbf_build", "mbf_import", "mbf_multiscale_assemble", "mbf_workspace_size", "mbf_apply",
           "mbf_apply_adjoint", "mbf_info", "mbf_destroy", "mbf_last_error", "mbf_kernel_dft",
           "mbf_kernel_fio", "mbf_kernel_fio_points", "mbf_profile_begin", "mbf_profile_end", "mbf_server_create",
           "mbf_server_submit", "mbf_server_poll", "mbf_server_drain", "mbf_server_stats",
           "mbf_server_destroy", "mbf_save", "mbf_load", "mbf_autotune", "mbf_apply_scratch", "mbf_scratch_bytes",
           "mbf_build_matvec"]


def lib():
    """Load libmbf.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libmbf.so not found at %s: run __graft_entry__.build() or "
                          "python -m paper_1509_07925_amd.build" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, u32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32
    L.mbf_build.argtypes = [i32, i64, vp, i64, vp, ENTRY_CB, vp, ctypes.POINTER(_Opts), vp, ctypes.POINTER(vp)]
    L.mbf_build_matvec.argtypes = [i32, i64, vp, i64, vp, MATVEC_CB, vp, ctypes.POINTER(_Opts), vp, vp,
                                   ctypes.POINTER(vp)]
    L.mbf_import.argtypes = [ctypes.POINTER(_ImportDesc), u32, vp, ctypes.POINTER(vp)]
    L.mbf_multiscale_assemble.argtypes = [i32, ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_void_p),
                                          ctypes.POINTER(i64), i64, i64, vp, vp, u32, vp, ctypes.POINTER(vp)]
    L.mbf_workspace_size.argtypes = [vp, i32, i64, ctypes.POINTER(ctypes.c_size_t)]
    L.mbf_apply.argtypes = [vp, i32, i64, vp, i64, vp, i64, vp, ctypes.c_size_t, vp]
    L.mbf_apply_adjoint.argtypes = [vp, i32, i64, vp, i64, vp, i64, vp, ctypes.c_size_t, vp]
    L.mbf_apply_scratch.argtypes = [vp, i32, i64, vp, i64, vp, i64, vp]
    L.mbf_scratch_bytes.argtypes = []
    L.mbf_scratch_bytes.restype = ctypes.c_size_t
    L.mbf_info.argtypes = [vp, ctypes.POINTER(Info)]
    L.mbf_profile_begin.argtypes = [vp, i32]
    L.mbf_profile_end.argtypes = [vp, ctypes.POINTER(LaunchRecord), i32, ctypes.POINTER(i32)]
    L.mbf_server_create.argtypes = [ctypes.c_size_t, i32, i64, ctypes.c_uint32, ctypes.POINTER(vp)]
    L.mbf_server_submit.argtypes = [vp, vp, i32, i64, vp, i64, vp, i64, vp, ctypes.POINTER(ctypes.c_uint64)]
    L.mbf_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]
    L.mbf_server_drain.argtypes = [vp]
    L.mbf_server_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    L.mbf_server_destroy.argtypes = [vp]
    L.mbf_server_destroy.restype = None
    L.mbf_save.argtypes = [vp, u32, ctypes.c_char_p]
    L.mbf_autotune.argtypes = [vp, i32, i64, vp, ctypes.c_size_t, vp, ctypes.POINTER(i32)]
    L.mbf_load.argtypes = [ctypes.c_char_p, u32, vp, ctypes.POINTER(vp)]
    L.mbf_destroy.argtypes = [vp]
    L.mbf_destroy.restype = None
    L.mbf_last_error.restype = ctypes.c_char_p
    for name in ("mbf_build", "mbf_build_matvec", "mbf_import", "mbf_multiscale_assemble", "mbf_workspace_size", "mbf_apply",
                 "mbf_apply_adjoint", "mbf_apply_scratch", "mbf_info", "mbf_profile_begin", "mbf_profile_end",
                 "mbf_server_create", "mbf_server_submit", "mbf_server_poll", "mbf_server_drain",
                 "mbf_server_stats", "mbf_save", "mbf_load", "mbf_autotune"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(st):
    if st != 0:
        raise MBFError(st, lib().mbf_last_error().decode())


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _mask(precs):
    m = 0
    for p in precs:
        m |= 1 << PREC[p]
    return m


class Factor:
    """A factorization resident in GPU memory (an ``mbf_factor`` handle)."""

    def __init__(self, handle, keep=None):
        self._h = handle
        self._keep = keep

    # ----------------------------------------------------------- creation
    @classmethod
    def import_factors(cls, depth, x_leaf_code, xi_leaf_code, ranks, v_leaf, h_blocks, s_mid, g_blocks,
                       u_leaf, precs=("c64",)):
        """mbf_import: factors of eq. (gbf) in the order documented in mbf.h."""
        arrs = dict(x=np.ascontiguousarray(x_leaf_code, np.int64), xi=np.ascontiguousarray(xi_leaf_code, np.int64),
                    r=np.ascontiguousarray(ranks, np.int32), v=np.ascontiguousarray(v_leaf, np.complex128),
                    h=np.ascontiguousarray(h_blocks, np.complex128), s=np.ascontiguousarray(s_mid, np.float64),
                    g=np.ascontiguousarray(g_blocks, np.complex128), u=np.ascontiguousarray(u_leaf, np.complex128))
        d = _ImportDesc(depth, arrs["x"].size, arrs["xi"].size, arrs["x"].ctypes.data, arrs["xi"].ctypes.data,
                        arrs["r"].ctypes.data, arrs["v"].ctypes.data,
                        arrs["h"].ctypes.data if arrs["h"].size else None, arrs["s"].ctypes.data,
                        arrs["g"].ctypes.data if arrs["g"].size else None, arrs["u"].ctypes.data)
        h = ctypes.c_void_p()
        _check(lib().mbf_import(ctypes.byref(d), _mask(precs), None, ctypes.byref(h)))
        return cls(h)

    @classmethod
    def build(cls, x, xi, n, kernel="dft", c_scale=1.0, tol=1e-6, max_rank=1024, leaf_side=4, depth=0,
              split="none", center_side=16, oversample=10, seed=0, precs=("c64",), threads=0, builder=None,
              device_mem_gb=0):
        """mbf_build from point sets and a kernel-entry callback.

        ``n`` is the side of the grids; 0 builds on general point sets (the
        trees cover the points' bounding squares to ``depth`` levels).

        ``kernel`` is "dft", "fio", "fio_points" (built-in C callbacks; the
        last one for general point sets) or a Python
        callable f(rows, cols) -> complex128 array (rows x cols) taking
        index arrays into x / xi.  ``builder`` is "device" (FP64 on the GPU;
        built-in kernels only, tol >= 1e-7) or "host"; by default built-in
        kernels build on the device and Python callables on the host.
        """
        if builder is None:
            builder = "device" if kernel in ("dft", "fio") and n > 0 else "host"
        x = np.ascontiguousarray(x, np.float64)
        xi = np.ascontiguousarray(xi, np.float64)
        L = lib()
        keep = [x, xi]
        if kernel in ("dft", "fio", "fio_points"):
            params = _KParams(n, c_scale, x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                              xi.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
            fn = getattr(L, "mbf_kernel_" + kernel)
            cb = ctypes.cast(fn, ENTRY_CB)
            user = ctypes.cast(ctypes.byref(params), ctypes.c_void_p)
            keep += [params]
        else:
            pyfn = kernel

            def _cb(_user, m, rows, k, cols, out):
                try:
                    r = np.ctypeslib.as_array(rows, (m,)).copy()
                    c = np.ctypeslib.as_array(cols, (k,)).copy()
                    vals = np.asarray(pyfn(r, c), np.complex128)
                    o = np.ctypeslib.as_array(out, (2 * m * k,))
                    o[:] = np.asfortranarray(vals).ravel(order="F").view(np.float64)
                    return 0
                except Exception:  # any error aborts the build
                    return 1

            cb = ENTRY_CB(_cb)
            user = None
            threads = 1  # Python callbacks hold the GIL
        keep.append(cb)
        o = _Opts(tol, max_rank, depth, leaf_side, n, SPLIT[split], center_side, oversample, seed,
                  _mask(precs), threads, BUILDER[builder], device_mem_gb)
        h = ctypes.c_void_p()
        _check(L.mbf_build(2, x.shape[0], x.ctypes.data, xi.shape[0], xi.ctypes.data, cb, user,
                           ctypes.byref(o), None, ctypes.byref(h)))
        return cls(h)

    @classmethod
    def build_matvec(cls, x, xi, n, matvec, tol=1e-6, max_rank=20, oversample=10, leaf_side=1, depth=0,
                     split="polar", center_side=16, seed=0, precs=("c64",), probes=None, threads=0):
        """mbf_build_matvec (build case (i)): the factorization of a K known
        only through ``matvec(adjoint, block)``, which returns K @ block
        (block: nxi x ncols) or K^* @ block (block: nx x ncols) as complex128
        arrays.  ``probes``: optional (C, R) Gaussian matrices of
        max_rank + oversample columns (nxi and nx rows); by default the
        library draws them from ``seed``.  Host FP64 builder."""
        x = np.ascontiguousarray(x, np.float64)
        xi = np.ascontiguousarray(xi, np.float64)
        nx, nxi = x.shape[0], xi.shape[0]
        L = lib()

        errs = []

        def _mv(_user, adjoint, ncols, src, dst):
            try:
                rin, rout = (nx, nxi) if adjoint else (nxi, nx)
                blk = np.ctypeslib.as_array(src, (2 * rin * ncols,)).view(np.complex128).reshape(ncols, rin).T
                res = np.asarray(matvec(bool(adjoint), blk), np.complex128)
                if res.shape != (rout, ncols):
                    return 2
                o = np.ctypeslib.as_array(dst, (2 * rout * ncols,))
                o[:] = np.asfortranarray(res).ravel(order="F").view(np.float64)
                return 0
            except Exception as ex:  # any error aborts the build; re-raised below as the cause
                errs.append(ex)
                return 1

        cb = MATVEC_CB(_mv)
        pr = None
        if probes is not None:
            C, R = (np.asarray(a, np.complex128) for a in probes)
            q = max_rank + oversample
            if C.shape != (nxi, q) or R.shape != (nx, q):
                raise ValueError("probes must be (nxi x q, nx x q) with q = max_rank + oversample")
            pr = np.concatenate([np.asfortranarray(C).ravel(order="F"), np.asfortranarray(R).ravel(order="F")])
        o = _Opts(tol, max_rank, depth, leaf_side, n, SPLIT[split], center_side, oversample, seed,
                  _mask(precs), threads, BUILDER["host"], 0)
        h = ctypes.c_void_p()
        st = L.mbf_build_matvec(2, nx, x.ctypes.data, nxi, xi.ctypes.data, cb, None, ctypes.byref(o),
                                pr.ctypes.data if pr is not None else None, None, ctypes.byref(h))
        if st != 0 and errs:
            raise MBFError(st, lib().mbf_last_error().decode()) from errs[0]
        _check(st)
        return cls(h)

    @classmethod
    def load(cls, path, precs=()):
        """mbf_load: a factorization saved by ``save`` (precs=() keeps all stored)."""
        h = ctypes.c_void_p()
        _check(lib().mbf_load(os.fsencode(path), _mask(precs), None, ctypes.byref(h)))
        return cls(h)

    def save(self, path, precs=()):
        """mbf_save: write the given precisions (default: all held) to ``path``."""
        _check(lib().mbf_save(self._h, _mask(precs), os.fsencode(path)))

    # ------------------------------------------------------------ queries
    def info(self):
        inf = Info()
        _check(lib().mbf_info(self._h, ctypes.byref(inf)))
        return inf

    def workspace_size(self, prec, nrhs):
        b = ctypes.c_size_t()
        _check(lib().mbf_workspace_size(self._h, PREC[prec], nrhs, ctypes.byref(b)))
        return b.value

    def _dims(self):
        # (nx, nxi) of the handle, fixed for its lifetime
        if getattr(self, "_nx_nxi", None) is None:
            inf = self.info()
            self._nx_nxi = (inf.nx, inf.nxi)
        return self._nx_nxi

    def _ws_size(self, prec, nrhs):
        cache = self.__dict__.setdefault("_ws_cache", {})
        key = (prec, nrhs)
        if key not in cache:
            cache[key] = self.workspace_size(prec, nrhs)
        return cache[key]

    # -------------------------------------------------------------- apply
    def _run(self, adj, x, out, prec, workspace, stream):
        import torch
        nx, nxi = self._dims()
        nin, nout = (nx, nxi) if adj else (nxi, nx)
        vec = x.dim() == 1
        X = x.reshape(-1, 1) if vec else x
        if X.shape[0] != nin or X.stride(0) != 1 or not X.is_cuda:
            raise ValueError("input must be a column-major CUDA tensor with %d rows" % nin)
        want = torch.complex128 if prec == "c128" else torch.complex64
        if X.dtype != want:
            raise ValueError("precision %s needs %s vectors" % (prec, want))
        nrhs = X.shape[1]
        if out is None:
            out = torch.empty((nrhs, nout), dtype=want, device=X.device).t()
        O = out.reshape(-1, 1) if out.dim() == 1 else out
        if O.shape != (nout, nrhs) or O.stride(0) != 1 or O.dtype != want:
            raise ValueError("bad output tensor")
        need = self._ws_size(prec, nrhs)
        if workspace is None or workspace.numel() * workspace.element_size() < need:
            workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=X.device)
        ldx = X.stride(1) if nrhs > 1 else nin
        ldo = O.stride(1) if nrhs > 1 else nout
        fn = lib().mbf_apply_adjoint if adj else lib().mbf_apply
        _check(fn(self._h, PREC[prec], nrhs, ctypes.c_void_p(X.data_ptr()), ldx, ctypes.c_void_p(O.data_ptr()),
                  ldo, ctypes.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size(),
                  _stream_ptr(stream)))
        return out

    def apply(self, g, out=None, prec="c64", workspace=None, stream=None):
        """u = K g (mbf_apply)."""
        return self._run(False, g, out, prec, workspace, stream)

    def apply_adjoint(self, h, out=None, prec="c64", workspace=None, stream=None):
        """v = K^* h (mbf_apply_adjoint)."""
        return self._run(True, h, out, prec, workspace, stream)

    def autotune(self, prec="c64", nrhs=256, workspace=None, stream=None):
        """mbf_autotune: time the stage-kernel variants for this RHS count; returns shapes tuned."""
        import torch
        need = self.workspace_size(prec, nrhs)
        if workspace is None or workspace.numel() * workspace.element_size() < need:
            workspace = torch.empty(max(need, 1), dtype=torch.uint8, device="cuda")
        n = ctypes.c_int32()
        _check(lib().mbf_autotune(self._h, PREC[prec], nrhs, ctypes.c_void_p(workspace.data_ptr()),
                                  workspace.numel() * workspace.element_size(), _stream_ptr(stream), ctypes.byref(n)))
        return n.value

    def profile_begin(self, max_launches):
        _check(lib().mbf_profile_begin(self._h, max_launches))

    def profile_end(self, cap=1 << 16):
        """Per-launch records (kind, part, stage, prec, ms, flops, bytes) as dicts."""
        buf = (LaunchRecord * cap)()
        n = ctypes.c_int32()
        _check(lib().mbf_profile_end(self._h, buf, cap, ctypes.byref(n)))
        return [dict(kind=r.kind, part=r.part, stage=r.stage, prec=r.prec, ms=r.ms, flops=r.flops,
                     bytes=r.bytes) for r in buf[:n.value]]

    def close(self):
        if self._h is not None and self._h.value:
            lib().mbf_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def multiscale_assemble(parts, part_idx, nxi, center_idx, center, precs=("c64",)):
    """mbf_multiscale_assemble; takes ownership of ``parts`` (Factor list)."""
    n = len(parts)
    hs = (ctypes.c_void_p * n)(*[p._h for p in parts])
    idx = [np.ascontiguousarray(i, np.int64) for i in part_idx]
    ip = (ctypes.c_void_p * n)(*[i.ctypes.data for i in idx])
    pn = (ctypes.c_int64 * n)(*[i.size for i in idx])
    ci = np.ascontiguousarray(center_idx, np.int64)
    C = np.asfortranarray(center, np.complex128)
    h = ctypes.c_void_p()
    st = lib().mbf_multiscale_assemble(n, hs, ip, pn, nxi, ci.size, ci.ctypes.data if ci.size else None,
                                       C.ctypes.data if ci.size else None, _mask(precs), None, ctypes.byref(h))
    for p in parts:
        p._h = None
    _check(st)
    return Factor(h)


class Server:
    """Request loop with continuous batching and memory admission (mbf_server_*).

    ``graphs=True`` runs every batch's apply as one launch of a HIP graph
    captured per (factor, precision, batch width) on fixed per-slot buffers
    (MBF_SERVER_GRAPHS)."""

    GRAPHS = 1

    def __init__(self, mem_budget, nslots=4, max_batch_rhs=256, graphs=False):
        self._h = ctypes.c_void_p()
        _check(lib().mbf_server_create(int(mem_budget), nslots, max_batch_rhs, self.GRAPHS if graphs else 0,
                                       ctypes.byref(self._h)))
        self._live = {}

    def submit(self, factor, g, out, prec="c64", ready=True):
        """Queue u = K g (g, out: column-major CUDA tensors); returns the request id.

        With ``ready=True`` an event is recorded on the current stream and
        the request's batch waits for it before reading g (work that
        produced g on that stream is ordered before the request).
        """
        import torch
        G = g.reshape(-1, 1) if g.dim() == 1 else g
        O = out.reshape(-1, 1) if out.dim() == 1 else out
        nrhs = G.shape[1]
        if G.stride(0) != 1 or O.stride(0) != 1 or O.shape[1] != nrhs:
            raise ValueError("column-major tensors with matching columns required")
        ldg = G.stride(1) if nrhs > 1 else G.shape[0]
        ldo = O.stride(1) if nrhs > 1 else O.shape[0]
        ev = None
        if ready:
            ev = torch.cuda.Event()
            ev.record()
        rid = ctypes.c_uint64()
        _check(lib().mbf_server_submit(self._h, factor._h, PREC[prec], nrhs, ctypes.c_void_p(G.data_ptr()), ldg,
                                       ctypes.c_void_p(O.data_ptr()), ldo,
                                       ctypes.c_void_p(ev.cuda_event) if ev is not None else None,
                                       ctypes.byref(rid)))
        self._live[rid.value] = (factor, g, out, ev)
        return rid.value

    def poll(self, rid):
        """(done, latency_us); raises MBFError when the request failed."""
        done = ctypes.c_int32()
        lat = ctypes.c_double()
        st = lib().mbf_server_poll(self._h, rid, ctypes.byref(done), ctypes.byref(lat))
        if done.value:
            self._live.pop(rid, None)
        _check(st)
        return bool(done.value), lat.value

    def drain(self):
        _check(lib().mbf_server_drain(self._h))
        self._live.clear()

    def stats(self):
        st = ServerStats()
        _check(lib().mbf_server_stats(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def close(self):
        if self._h is not None and self._h.value:
            lib().mbf_server_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
