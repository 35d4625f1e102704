"""Python binding of the MI355X H^2 strong recursive skeletonization solver.

Argument marshalling only: every step of the factorization, solve, matvec and
refinement runs in the HIP library libh2rss.so (built in-tree by build.py)
behind the C ABI of include/h2.h.  PyTorch provides device memory and the
stream.  Importing this package fails loudly when the library is missing.

Vectors are torch float64 CUDA tensors of shape (N, nrhs) in original point
order; they are handed to the library column-major (leading dimension N).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libh2rss.so")

H2_PREC_FP64 = 0
H2_PREC_FP32 = 1
H2_PREC_FP32_GRAM = 2
H2_PREC_FP32_QR = 3
(INT_SIZES, INT_RANKS, INT_COLORS, INT_FILL, INT_NTOP, INT_LEVELS, INT_OFFSETS,
 INT_CLUSTER_OFFSETS, INT_OWNERS) = range(9)
MAT_Q, MAT_BLOCK, MAT_TOP = range(3)

STATUS = {
    0: "success", 1: "invalid argument", 2: "format", 3: "out of memory", 4: "singular",
    5: "numeric", 6: "hip", 7: "not converged", 8: "unsupported",
}


class H2Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class _IROpts(ctypes.Structure):
    _fields_ = [("target_bkwd", ctypes.c_double), ("restart", ctypes.c_int),
                ("max_outer", ctypes.c_int), ("inner_rtol", ctypes.c_double)]


class _IRReport(ctypes.Structure):
    _fields_ = [("outer_iterations", ctypes.c_int), ("inner_iterations", ctypes.c_int),
                ("max_bkwd", ctypes.c_double)]


# factorization phases of h2_stats (indices 0..7 are device phases, one
# kernel each; 8 = host planning the stream waited for, 9 = total wall)
H2_PHASES = 10
PHASES = ["fill_row_qr", "augment", "project", "lu", "multipliers", "schur", "close_out",
          "top_lu", "host_planning", "total"]


class _Stats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("max_colors", ctypes.c_int32),
                ("n_top", ctypes.c_int64), ("factor_bytes", ctypes.c_int64),
                ("peak_bytes", ctypes.c_int64), ("factor_flops", ctypes.c_double),
                ("solve_flops_per_rhs", ctypes.c_double), ("time_ms", ctypes.c_double * H2_PHASES),
                ("phase_flops", ctypes.c_double * H2_PHASES),
                ("phase_bytes", ctypes.c_double * H2_PHASES),
                ("launches", ctypes.c_int64 * H2_PHASES),
                ("solves", ctypes.c_int64), ("solve_graph_launches", ctypes.c_int64)]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                            ctypes.c_void_p)


class _CtxOpts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("stream", ctypes.c_void_p), ("alloc", _ALLOC_FN),
                ("free", _FREE_FN), ("user", ctypes.c_void_p)]


class _FactorOpts(ctypes.Structure):
    _fields_ = [("norm2", ctypes.c_double), ("pool_bytes", ctypes.c_int64),
                ("keep_owner_lists", ctypes.c_int32), ("lds_limit_kib", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("dim", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("top_level", ctypes.c_int32), ("n_nodes", ctypes.c_int32),
                ("norm2", ctypes.c_double), ("device_bytes", ctypes.c_int64)]


# exported symbols of include/h2.h with (restype, argtypes)
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_SIG = {
    "h2_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "h2_context_create": (ctypes.c_int, [ctypes.POINTER(_CtxOpts), ctypes.POINTER(_P)]),
    "h2_blob_check": (ctypes.c_int, [_P, ctypes.c_size_t, ctypes.c_char_p, ctypes.c_size_t]),
    "h2_context_destroy": (ctypes.c_int, [_P]),
    "h2_last_error": (ctypes.c_char_p, [_P]),
    "h2_sync": (ctypes.c_int, [_P]),
    "h2_matrix_load": (ctypes.c_int, [_P, _P, ctypes.c_size_t, ctypes.POINTER(_P)]),
    "h2_matrix_destroy": (ctypes.c_int, [_P]),
    "h2_matrix_get_info": (ctypes.c_int, [_P, ctypes.POINTER(_Info)]),
    "h2_matvec": (ctypes.c_int, [_P, _P, _P, _I64, ctypes.c_int, _P, _I64]),
    "h2_matvec_noalloc": (ctypes.c_int, [_P, _P, _P, _I64, ctypes.c_int, _P, _I64]),
    "h2_factor": (ctypes.c_int, [_P, _P, ctypes.c_double, ctypes.c_int,
                                 ctypes.POINTER(_FactorOpts), ctypes.POINTER(_P)]),
    "h2_factor_destroy": (ctypes.c_int, [_P]),
    "h2_solve": (ctypes.c_int, [_P, _P, _P, _I64, ctypes.c_int, _P, _I64]),
    "h2_solve_ir": (ctypes.c_int, [_P, _P, _P, _P, _I64, ctypes.c_int, _P, _I64,
                                   ctypes.POINTER(_IROpts), ctypes.POINTER(_IRReport)]),
    "h2_factor_batched": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(_P), ctypes.c_double,
                                         ctypes.c_int, ctypes.POINTER(_FactorOpts),
                                         ctypes.POINTER(_P)]),
    "h2_solve_batched": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(_P), ctypes.POINTER(_P),
                                        ctypes.POINTER(_I64), ctypes.c_int, ctypes.POINTER(_P),
                                        ctypes.POINTER(_I64)]),
    "h2_factor_export_ints": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int,
                                             ctypes.POINTER(_I64), _I64, ctypes.POINTER(_I64)]),
    "h2_factor_get_stats": (ctypes.c_int, [_P, ctypes.POINTER(_Stats)]),
    "h2_factor_export_matrix": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                               ctypes.c_int, _P, _I64, ctypes.POINTER(_I64),
                                               ctypes.POINTER(_I64)]),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library {LIB_PATH} is not built (run python paper_2509_11152_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIG.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


# Handles that the garbage collector releases while the library is inside one
# of its allocator callbacks (a collection can run in the callback's Python
# code) are destroyed once the library call has returned, never from inside
# it: the library is not re-entrant.
# A context released by the collector is destroyed at the next library call,
# after any matrix or factor that the same collection released (they must go
# first).
_in_callback = [0]
_deferred = []  # (order, destroy function, handle): factors, matrices, contexts


def _release(order, fn, ptr, keep=None):
    """keep: objects the destroy call needs alive (a context's allocator
    callbacks)."""
    if _in_callback[0] or order == 2:
        _deferred.append((order, fn, ptr, keep))
    else:
        fn(ptr)


def _flush_deferred():
    if not _deferred or _in_callback[0]:
        return
    items = sorted(_deferred, key=lambda x: x[0])
    _deferred.clear()
    for _, fn, ptr, _keep in items:
        try:
            fn(ptr)
        except Exception:
            pass


def _check(code, ctx=None):
    _flush_deferred()
    if code != 0:
        msg = lib.h2_last_error(ctx.ptr).decode() if ctx is not None else ""
        raise H2Error(code, msg)


def _colmajor(X):
    """(N, nrhs) tensor -> contiguous (nrhs, N) tensor = column-major N x nrhs."""
    import torch

    if X.dim() == 1:
        X = X[:, None]
    return X.t().contiguous().to(torch.float64)


class Context:
    """A library context on one device.

    stream: None lets the library create its own stream (ordered with the
    legacy default stream, which is torch's default); or a torch.cuda.Stream
    to enqueue on.  allocator: "torch" backs every device byte the library
    holds with torch's caching allocator; "pool" uses the device's
    stream-ordered memory pool."""

    def __init__(self, device=0, stream=None, allocator="torch"):
        import torch

        self.device = device
        self.torch_stream = stream
        self._cbs = None
        opts = _CtxOpts()
        opts.device = device
        opts.stream = stream.cuda_stream if stream is not None else None
        if allocator == "torch":
            def _alloc(nbytes, strm, user):
                _in_callback[0] += 1
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), device, int(strm or 0))
                except Exception:
                    return None
                finally:
                    _in_callback[0] -= 1

            def _free(ptr, nbytes, strm, user):
                _in_callback[0] += 1
                try:
                    torch.cuda.caching_allocator_delete(int(ptr))
                except Exception:
                    pass
                finally:
                    _in_callback[0] -= 1

            self._cbs = (_ALLOC_FN(_alloc), _FREE_FN(_free))
            opts.alloc, opts.free = self._cbs
        elif allocator != "pool":
            raise ValueError(f"unknown allocator {allocator!r}")
        self.ptr = _P()
        _check(lib.h2_context_create(ctypes.byref(opts), ctypes.byref(self.ptr)))

    def sync(self):
        _check(lib.h2_sync(self.ptr), self)

    def close(self):
        if self.ptr:
            _release(2, lib.h2_context_destroy, self.ptr, self._cbs)
            self.ptr = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Matrix:
    """A serialized H^2 matrix (uint8 numpy blob) loaded onto the device."""

    def __init__(self, ctx, blob):
        self.ctx = ctx
        buf = np.ascontiguousarray(np.asarray(blob, dtype=np.uint8))
        self.ptr = _P()
        _check(lib.h2_matrix_load(ctx.ptr, buf.ctypes.data_as(_P), buf.nbytes,
                                  ctypes.byref(self.ptr)), ctx)
        info = _Info()
        _check(lib.h2_matrix_get_info(self.ptr, ctypes.byref(info)), ctx)
        self.n = info.n
        self.depth = info.depth
        self.top_level = info.top_level
        self.norm2 = info.norm2
        self.device_bytes = info.device_bytes

    def matvec(self, X):
        import torch

        Xc = _colmajor(X)
        nrhs = Xc.shape[0]
        Y = torch.empty_like(Xc)
        _check(lib.h2_matvec(self.ctx.ptr, self.ptr, _P(Xc.data_ptr()), self.n, nrhs,
                             _P(Y.data_ptr()), self.n), self.ctx)
        self.ctx.sync()
        return Y.t()

    def matvec_noalloc(self, X):
        """The product through h2_matvec_noalloc (work arrays in the library's
        static device scratch; the output tensor is the caller's)."""
        import torch

        Xc = _colmajor(X)
        nrhs = Xc.shape[0]
        Y = torch.empty_like(Xc)
        _check(lib.h2_matvec_noalloc(self.ctx.ptr, self.ptr, _P(Xc.data_ptr()), self.n, nrhs,
                                     _P(Y.data_ptr()), self.n), self.ctx)
        return Y.t()

    def __del__(self):
        try:
            if self.ptr:
                _release(1, lib.h2_matrix_destroy, self.ptr)
                self.ptr = _P()
        except Exception:
            pass


def _factor_opts(norm2=None, pool_bytes=None, keep_owner_lists=False, lds_limit_kib=0):
    return _FactorOpts(float(norm2 or 0.0), int(pool_bytes or 0), int(bool(keep_owner_lists)),
                       int(lds_limit_kib))


class Factor:
    def __init__(self, ctx, H, tol, prec=H2_PREC_FP64, _ptr=None, **opts):
        self.ctx = ctx
        self.n = H.n
        self.prec = prec
        if _ptr is not None:
            self.ptr = _ptr
        else:
            self.ptr = _P()
            o = _factor_opts(**opts)
            _check(lib.h2_factor(ctx.ptr, H.ptr, float(tol), prec, ctypes.byref(o),
                                 ctypes.byref(self.ptr)), ctx)

    def solve(self, B, out=None):
        import torch

        Bc = _colmajor(B)
        nrhs = Bc.shape[0]
        X = torch.empty_like(Bc) if out is None else out
        _check(lib.h2_solve(self.ctx.ptr, self.ptr, _P(Bc.data_ptr()), self.n, nrhs,
                            _P(X.data_ptr()), self.n), self.ctx)
        self.ctx.sync()
        return X.t()

    def solve_colmajor(self, Bc, Xc):
        """Solve on preallocated (nrhs, N) buffers without syncing (timing loops)."""
        _check(lib.h2_solve(self.ctx.ptr, self.ptr, _P(Bc.data_ptr()), self.n, Bc.shape[0],
                            _P(Xc.data_ptr()), self.n), self.ctx)

    def ints(self, level, kind):
        n = ctypes.c_int64(0)
        _check(lib.h2_factor_export_ints(self.ptr, level, kind, None, 0, ctypes.byref(n)))
        buf = (ctypes.c_int64 * max(n.value, 1))()
        _check(lib.h2_factor_export_ints(self.ptr, level, kind, buf, n.value, ctypes.byref(n)))
        return np.array(buf[:n.value], dtype=np.int64)

    def matrix(self, level, kind, i=0, j=0):
        """Copy a factor matrix (Q~ of cluster i, near block (i, j), or the LU'd top block)."""
        m, n = ctypes.c_int64(0), ctypes.c_int64(0)
        _check(lib.h2_factor_export_matrix(self.ptr, level, kind, i, j, None, 0, ctypes.byref(m),
                                           ctypes.byref(n)))
        out = np.zeros((n.value, m.value))
        if m.value * n.value:
            _check(lib.h2_factor_export_matrix(self.ptr, level, kind, i, j, out.ctypes.data_as(_P),
                                               out.size, ctypes.byref(m), ctypes.byref(n)))
        return out.T

    def levels(self):
        return [int(x) for x in self.ints(0, INT_LEVELS)]

    def stats(self):
        s = _Stats()
        _check(lib.h2_factor_get_stats(self.ptr, ctypes.byref(s)))
        return {"levels": s.levels, "max_colors": s.max_colors, "n_top": s.n_top,
                "factor_bytes": s.factor_bytes, "peak_bytes": s.peak_bytes,
                "factor_flops": s.factor_flops, "solve_flops_per_rhs": s.solve_flops_per_rhs,
                "time_ms": list(s.time_ms),
                "phase_flops": list(s.phase_flops), "phase_bytes": list(s.phase_bytes),
                "launches": list(s.launches), "solves": s.solves,
                "solve_graph_launches": s.solve_graph_launches}

    def __del__(self):
        try:
            if self.ptr:
                _release(0, lib.h2_factor_destroy, self.ptr)
                self.ptr = _P()
        except Exception:
            pass


def blob_check(blob):
    """Host-side validation of a serialized matrix: (status code, message)."""
    buf = np.ascontiguousarray(np.asarray(blob, dtype=np.uint8))
    msg = ctypes.create_string_buffer(512)
    code = lib.h2_blob_check(buf.ctypes.data_as(_P), buf.nbytes, msg, 512)
    return code, msg.value.decode()


def solve_ir(ctx, H, F, B, target=1e-12, restart=30, max_outer=20, inner_rtol=1e-3):
    """GMRES-IR: returns (X, report dict); raises on errors other than NOT_CONVERGED."""
    import torch

    Bc = _colmajor(B)
    nrhs = Bc.shape[0]
    X = torch.empty_like(Bc)
    opts = _IROpts(target, restart, max_outer, inner_rtol)
    rep = _IRReport()
    code = lib.h2_solve_ir(ctx.ptr, H.ptr, F.ptr, _P(Bc.data_ptr()), H.n, nrhs, _P(X.data_ptr()),
                           H.n, ctypes.byref(opts), ctypes.byref(rep))
    if code not in (0, 7):
        _check(code, ctx)
    return X.t(), {"outer": rep.outer_iterations, "inner": rep.inner_iterations,
                   "max_bkwd": rep.max_bkwd, "converged": code == 0}


def factor_batched(ctx, Hs, tol, prec=H2_PREC_FP64, **opts):
    arr = (_P * len(Hs))(*[H.ptr for H in Hs])
    out = (_P * len(Hs))()
    o = _factor_opts(**opts)
    _check(lib.h2_factor_batched(ctx.ptr, len(Hs), arr, float(tol), prec, ctypes.byref(o), out),
           ctx)
    return [Factor(ctx, H, tol, prec, _ptr=_P(out[i])) for i, H in enumerate(Hs)]


def solve_batched(ctx, Fs, Bs):
    """Bs: list of (N_i, nrhs) tensors with the same nrhs; returns list of X_i."""
    import torch

    Bcs = [_colmajor(B) for B in Bs]
    nrhs = Bcs[0].shape[0]
    Xcs = [torch.empty_like(b) for b in Bcs]
    n = len(Fs)
    fa = (_P * n)(*[F.ptr for F in Fs])
    ba = (_P * n)(*[_P(b.data_ptr()) for b in Bcs])
    xa = (_P * n)(*[_P(x.data_ptr()) for x in Xcs])
    lb = (_I64 * n)(*[F.n for F in Fs])
    _check(lib.h2_solve_batched(ctx.ptr, n, fa, ba, lb, nrhs, xa, lb), ctx)
    ctx.sync()
    return [x.t() for x in Xcs]
