"""Python binding of libpipesafe (ctypes; argument marshalling only).

Every step of a solve runs in the library's HIP kernels.  PyTorch is used,
where the caller wants device buffers, only to provide device memory and the
current stream (``solve_dev`` / ``spmv_dev`` take torch CUDA tensors).  There
is no CPU fallback: if the library is missing or no gfx950 GPU is present,
the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpipesafe.so")

VARIANTS = {"ssbicgsafe2": 0, "pbicgsafe": 1, "pbicgsafe_rr": 2, "pbicgstab": 3}
CONVERGED, MAXIT, BREAKDOWN, NONFINITE = 0, 1, 2, 3
STATUS_NAMES = {0: "converged", 1: "maxit", 2: "breakdown", 3: "nonfinite"}
# ps_options.precision: the matrix values the products read (include/pipesafe.h)
PRECISIONS = {"fp64": 0, "fp32_matrix": 1, "fp32_krylov": 2, "fp32_vectors": 3}
VEC = ["x", "r", "rs", "s", "y", "t", "p", "u", "z", "w", "l", "g", "q", "o", "As", "v", "b"]
SCAL = ["alpha", "beta", "zeta", "eta", "omega", "f", "rhoref", "rho", "pending", "gs", "gw", "gz"]
KERNEL_CLASSES = {"spmv": 0, "dots": 1, "update": 2, "spmv_fused": 3, "other": 4, "dots_finish": 5}


class PipesafeError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {_lib().ps_strerror(code).decode()} ({code})")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("rr_m", ctypes.c_int32), ("rr_M", ctypes.c_int32), ("norm_ref", ctypes.c_int32),
                ("batch_iters", ctypes.c_int32), ("overlap", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("resume", ctypes.c_int32),
                ("resume_iter", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("x0_fallback", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("stream", ctypes.c_void_p)]


class Info(ctypes.Structure):
    _fields_ = [("format", ctypes.c_int32), ("spmv_shape", ctypes.c_int32), ("n", ctypes.c_int64),
                ("nnz", ctypes.c_int64), ("slots", ctypes.c_int64), ("spmv_blocks", ctypes.c_int32),
                ("dot_grid", ctypes.c_int32), ("matrix_bytes", ctypes.c_int64),
                ("auto_overlap", ctypes.c_int32), ("auto_schedule", ctypes.c_int32),
                ("nsys", ctypes.c_int32), ("streaming", ctypes.c_int32), ("n_padded", ctypes.c_int64),
                ("index_bits", ctypes.c_int32), ("gather_sort", ctypes.c_int32)]


FORMATS = {0: "csr", 1: "sell"}
FORMAT_IDS = {"csr": 0, "sell": 1}


class Layout(ctypes.Structure):
    """ps_layout: an explicit device layout; -1 = automatic."""
    _fields_ = [("format", ctypes.c_int32), ("sell_rows_per_lane", ctypes.c_int32),
                ("spmv_shape", ctypes.c_int32), ("index_bits", ctypes.c_int32),
                ("gather_sort", ctypes.c_int32)]


def layout(format=-1, sell_rows_per_lane=-1, spmv_shape=-1, index_bits=-1, gather_sort=-1) -> Layout:
    return Layout(FORMAT_IDS.get(format, format), sell_rows_per_lane, spmv_shape, index_bits,
                  gather_sort)


class TuneEntry(ctypes.Structure):
    _fields_ = [("layout", Layout), ("schedule", ctypes.c_int32), ("overlap", ctypes.c_int32),
                ("streaming", ctypes.c_int32), ("batch_iters", ctypes.c_int32),
                ("us", ctypes.c_double)]


class TuneReport(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("best", ctypes.c_int32), ("entry", TuneEntry * 48)]

    def rows(self) -> list:
        out = []
        for k in range(self.count):
            e = self.entry[k]
            r = {"us": e.us, "best": k == self.best}
            if e.layout.format >= 0:
                r.update(format=FORMATS[e.layout.format], sell_rows_per_lane=e.layout.sell_rows_per_lane,
                         spmv_shape=e.layout.spmv_shape, index_bits=e.layout.index_bits,
                         gather_sort=e.layout.gather_sort)
            else:
                r.update(schedule=e.schedule, overlap=e.overlap, streaming=e.streaming,
                         batch_iters=e.batch_iters)
            out.append(r)
        return out

_L = None


def _lib():
    global _L
    if _L is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        Pi32, Pi64, Pf64 = ctypes.POINTER(i32), ctypes.POINTER(i64), ctypes.POINTER(f64)
        L.ps_default_options.argtypes = [ctypes.POINTER(Options)]
        L.ps_default_options.restype = None
        L.ps_create.argtypes = [ctypes.POINTER(P), i64, i64, P, P, P]
        L.ps_solve.argtypes = [P, P, P, f64, i32, i32, ctypes.POINTER(Options), P, Pi32, P, Pi32]
        L.ps_solve_dev.argtypes = L.ps_solve.argtypes
        L.ps_solve_dev_static.argtypes = L.ps_solve.argtypes
        L.ps_create_batch.argtypes = [ctypes.POINTER(P), i32, P, i64, i64, P, P, P]
        L.ps_solve_batch.argtypes = [P, P, P, f64, i32, i32, ctypes.POINTER(Options), P, P, P, P]
        L.ps_solve_batch_dev.argtypes = L.ps_solve_batch.argtypes
        L.ps_spmv_dev.argtypes = [P, P, P, P]
        L.ps_get_state.argtypes = [P, i32, P]
        L.ps_set_state.argtypes = [P, i32, P]
        L.ps_get_scalars.argtypes = [P, P]
        L.ps_set_scalars.argtypes = [P, P]
        L.ps_kernel_stats.argtypes = [P, i32, Pf64, Pi64]
        L.ps_kernel_streams.argtypes = [P, i32, Pi64]
        L.ps_matrix_info.argtypes = [P, ctypes.POINTER(Info)]
        L.ps_stream_copy.argtypes = [P, P, i64, P]
        L.ps_destroy.argtypes = [P]
        L.ps_create_ex.argtypes = [ctypes.POINTER(P), i64, i64, P, P, P, ctypes.POINTER(Layout)]
        L.ps_create_batch_ex.argtypes = [ctypes.POINTER(P), i32, P, i64, i64, P, P, P,
                                         ctypes.POINTER(Layout)]
        L.ps_autotune_layout.argtypes = [ctypes.POINTER(P), i32, P, i64, i64, P, P, P, i32,
                                         ctypes.POINTER(TuneReport)]
        L.ps_tune_options.argtypes = [P, P, i32, i32, ctypes.POINTER(Options),
                                      ctypes.POINTER(TuneReport)]
        L.ps_strerror.argtypes = [ctypes.c_int]
        L.ps_strerror.restype = ctypes.c_char_p
        L.ps_version.restype = ctypes.c_char_p
        for name in ("ps_create", "ps_create_batch", "ps_solve_batch", "ps_solve_batch_dev",
                     "ps_solve", "ps_solve_dev", "ps_solve_dev_static", "ps_spmv_dev", "ps_get_state",
                     "ps_set_state", "ps_get_scalars", "ps_set_scalars", "ps_kernel_stats",
                     "ps_kernel_streams", "ps_matrix_info",
                     "ps_stream_copy", "ps_destroy", "ps_create_ex", "ps_create_batch_ex",
                     "ps_autotune_layout", "ps_tune_options"):
            getattr(L, name).restype = ctypes.c_int
        _L = L
    return _L


def library():
    """The loaded ctypes library (raises ImportError if it is not built)."""
    return _lib()


def _check(rc: int, what: str):
    if rc != 0:
        raise PipesafeError(rc, what)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _vid(variant) -> int:
    return VARIANTS[variant] if isinstance(variant, str) else int(variant)


def options(**kw) -> Options:
    o = Options()
    _lib().ps_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if k == "profile" and isinstance(v, (list, tuple, set)):
            v = sum(1 << KERNEL_CLASSES[c] for c in v)
        if k == "precision" and isinstance(v, str):
            v = PRECISIONS[v]
        setattr(o, k, v)
    return o


@dataclass
class SolveResult:
    x: object
    iters: int
    status: int
    hist: np.ndarray

    @property
    def status_name(self) -> str:
        return STATUS_NAMES.get(self.status, str(self.status))


class Matrix:
    """A CSR matrix resident on the current HIP device, with its solver workspace."""

    def __init__(self, n: int, rowptr, col, val, layout: Layout | None = None, _handle=None):
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        self.n = int(n)
        self.nnz = int(rowptr[-1]) if rowptr.size else 0
        if _handle is not None:
            self._h = _handle
            return
        col = np.ascontiguousarray(col, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float64)
        h = ctypes.c_void_p()
        _check(_lib().ps_create_ex(ctypes.byref(h), self.n, self.nnz, _ptr(rowptr), _ptr(col),
                                   _ptr(val), None if layout is None else ctypes.byref(layout)),
               "ps_create_ex")
        self._h = h

    @classmethod
    def from_csr(cls, A, layout: Layout | None = None) -> "Matrix":
        return cls(A.n, A.rowptr, A.col, A.val, layout)

    @classmethod
    def autotuned(cls, A, reps: int = 20):
        """ps_autotune_layout: the layout with the fastest p-BiCGSafe iterations on A.
        Returns (Matrix, rows of the tuning report)."""
        rowptr = np.ascontiguousarray(A.rowptr, dtype=np.int64)
        col = np.ascontiguousarray(A.col, dtype=np.int32)
        val = np.ascontiguousarray(A.val, dtype=np.float64)
        h, rep = ctypes.c_void_p(), TuneReport()
        _check(_lib().ps_autotune_layout(ctypes.byref(h), 1, None, A.n, int(rowptr[-1]),
                                         _ptr(rowptr), _ptr(col), _ptr(val), int(reps),
                                         ctypes.byref(rep)), "ps_autotune_layout")
        return cls(A.n, rowptr, None, None, _handle=h), rep.rows()

    def tune_options(self, b, variant="pbicgsafe", iters=50, **base):
        """ps_tune_options from device b (torch CUDA float64, length n): returns (dict of the
        chosen schedule / overlap / batch_iters, rows of the tuning report)."""
        import torch
        if b.dtype != torch.float64 or not b.is_cuda or not b.is_contiguous():
            raise ValueError("expected a contiguous float64 CUDA tensor")
        o, rep = options(**base), TuneReport()
        _check(_lib().ps_tune_options(self._h, ctypes.c_void_p(b.data_ptr()), _vid(variant),
                                      int(iters), ctypes.byref(o), ctypes.byref(rep)),
               "ps_tune_options")
        return {"schedule": o.schedule, "overlap": o.overlap, "batch_iters": o.batch_iters}, rep.rows()

    def close(self):
        if getattr(self, "_h", None):
            _lib().ps_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -------------------------------------------------------------- solves
    def solve(self, b, x0=None, tol=1e-8, maxit=10_000, variant="pbicgsafe", hist=True, **opt):
        """Solve from host (numpy) buffers; returns SolveResult with a numpy x."""
        b = np.ascontiguousarray(b, dtype=np.float64)
        x0a = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
        x = np.empty(self.n)
        h = np.empty(maxit + 1) if hist else None
        iters, status = ctypes.c_int32(), ctypes.c_int32()
        o = options(**opt)
        _check(_lib().ps_solve(self._h, _ptr(b), None if x0a is None else _ptr(x0a), float(tol),
                               int(maxit), _vid(variant), ctypes.byref(o), _ptr(x),
                               ctypes.byref(iters), None if h is None else _ptr(h),
                               ctypes.byref(status)), "ps_solve")
        it = iters.value
        return SolveResult(x, it, status.value, h[: it + 1] if h is not None else None)

    def solve_dev(self, b, x0=None, x=None, tol=1e-8, maxit=10_000, variant="pbicgsafe",
                  hist=True, stream=None, **opt):
        """Solve with torch CUDA tensors b, x0 (or None), x (allocated if None), float64.

        Work is ordered on ``stream`` (default: torch's current stream)."""
        return self._solve_dev("ps_solve_dev", b, x0, x, tol, maxit, variant, hist, stream, opt)

    def solve_dev_static(self, b, x0=None, x=None, tol=1e-8, maxit=10_000, variant="pbicgsafe",
                         hist=True, stream=None, **opt):
        """solve_dev through ps_solve_dev_static: the library allocates nothing during the call
        (its per-solve blocks live in a static device workspace; x must be given for a caller
        that cannot allocate either)."""
        return self._solve_dev("ps_solve_dev_static", b, x0, x, tol, maxit, variant, hist, stream,
                               opt)

    def _solve_dev(self, entry, b, x0, x, tol, maxit, variant, hist, stream, opt):
        import torch
        for t in (b, x0, x):
            if t is not None and (t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous()
                                  or t.numel() != self.n):
                raise ValueError("expected contiguous float64 CUDA tensors of length n")
        if x is None:
            x = torch.empty(self.n, dtype=torch.float64, device=b.device)
        if stream is None:
            stream = torch.cuda.current_stream(b.device).cuda_stream
        h = np.empty(maxit + 1) if hist else None
        iters, status = ctypes.c_int32(), ctypes.c_int32()
        o = options(stream=stream, **opt)
        _check(getattr(_lib(), entry)(self._h, ctypes.c_void_p(b.data_ptr()),
                                      None if x0 is None else ctypes.c_void_p(x0.data_ptr()),
                                      float(tol), int(maxit), _vid(variant), ctypes.byref(o),
                                      ctypes.c_void_p(x.data_ptr()), ctypes.byref(iters),
                                      None if h is None else _ptr(h), ctypes.byref(status)),
               entry)
        it = iters.value
        return SolveResult(x, it, status.value, h[: it + 1] if h is not None else None)

    def spmv_dev(self, x, y=None, stream=None):
        import torch
        if y is None:
            y = torch.empty_like(x)
        if stream is None:
            stream = torch.cuda.current_stream(x.device).cuda_stream
        _check(_lib().ps_spmv_dev(self._h, ctypes.c_void_p(x.data_ptr()),
                                  ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(stream)),
               "ps_spmv_dev")
        return y

    # --------------------------------------------------------------- state
    def get_state(self, name: str) -> np.ndarray:
        out = np.empty(self.n)
        _check(_lib().ps_get_state(self._h, VEC.index(name), _ptr(out)), "ps_get_state")
        return out

    def set_state(self, name: str, values):
        a = np.ascontiguousarray(values, dtype=np.float64)
        assert a.size == self.n
        _check(_lib().ps_set_state(self._h, VEC.index(name), _ptr(a)), "ps_set_state")

    def get_scalars(self) -> dict:
        out = np.empty(len(SCAL))
        _check(_lib().ps_get_scalars(self._h, _ptr(out)), "ps_get_scalars")
        return dict(zip(SCAL, out.tolist()))

    def set_scalars(self, values: dict):
        cur = np.empty(len(SCAL))
        _check(_lib().ps_get_scalars(self._h, _ptr(cur)), "ps_get_scalars")
        for k, v in values.items():
            cur[SCAL.index(k)] = v
        _check(_lib().ps_set_scalars(self._h, _ptr(cur)), "ps_set_scalars")

    def info(self) -> dict:
        """The device layout ps_create chose (format, slots, product grid, matrix bytes)."""
        i = Info()
        _check(_lib().ps_matrix_info(self._h, ctypes.byref(i)), "ps_matrix_info")
        d = {k: getattr(i, k) for k, _ in Info._fields_}
        d["format"] = FORMATS.get(d["format"], d["format"])
        return d

    def kernel_stats(self) -> dict:
        """{class: (total_ms, launches)} of the last profiled solve."""
        out = {}
        for name, c in KERNEL_CLASSES.items():
            ms, cnt = ctypes.c_double(), ctypes.c_int64()
            _check(_lib().ps_kernel_stats(self._h, c, ctypes.byref(ms), ctypes.byref(cnt)),
                   "ps_kernel_stats")
            out[name] = (ms.value, cnt.value)
        return out

    def kernel_streams(self) -> dict:
        """{class: launches on the second stream} of the last profiled solve."""
        out = {}
        for name, c in KERNEL_CLASSES.items():
            cnt = ctypes.c_int64()
            _check(_lib().ps_kernel_streams(self._h, c, ctypes.byref(cnt)), "ps_kernel_streams")
            out[name] = cnt.value
        return out


@dataclass
class BatchResult:
    x: object                 # concatenated solutions (numpy or torch, like the inputs)
    iters: np.ndarray         # int32[nsys]
    status: np.ndarray        # int32[nsys]
    hist: np.ndarray | None   # [nsys, maxit+1]; row k valid up to iters[k]

    def system_hist(self, k: int) -> np.ndarray:
        return self.hist[k, : int(self.iters[k]) + 1]


class BatchMatrix(Matrix):
    """Independent systems solved together (ps_create_batch / ps_solve_batch)."""

    def __init__(self, sys_ptr, n: int, rowptr, col, val, layout: Layout | None = None,
                 _handle=None):
        sys_ptr = np.ascontiguousarray(sys_ptr, dtype=np.int64)
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        self.n = int(n)
        self.nnz = int(rowptr[-1]) if rowptr.size else 0
        self.nsys = int(sys_ptr.size - 1)
        self.sys_ptr = sys_ptr
        if _handle is not None:
            self._h = _handle
            return
        col = np.ascontiguousarray(col, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float64)
        h = ctypes.c_void_p()
        _check(_lib().ps_create_batch_ex(ctypes.byref(h), self.nsys, _ptr(sys_ptr), self.n,
                                         self.nnz, _ptr(rowptr), _ptr(col), _ptr(val),
                                         None if layout is None else ctypes.byref(layout)),
               "ps_create_batch_ex")
        self._h = h

    @classmethod
    def from_batch(cls, B, layout: Layout | None = None) -> "BatchMatrix":
        """From a workloads.Batch (its block-diagonal concatenation)."""
        C = B.concat()
        return cls(B.sys_ptr(), C.n, C.rowptr, C.col, C.val, layout)

    @classmethod
    def autotuned(cls, B, reps: int = 20):
        """ps_autotune_layout for a workloads.Batch: returns (BatchMatrix, report rows)."""
        C = B.concat()
        sys_ptr = np.ascontiguousarray(B.sys_ptr(), dtype=np.int64)
        rowptr = np.ascontiguousarray(C.rowptr, dtype=np.int64)
        col = np.ascontiguousarray(C.col, dtype=np.int32)
        val = np.ascontiguousarray(C.val, dtype=np.float64)
        h, rep = ctypes.c_void_p(), TuneReport()
        _check(_lib().ps_autotune_layout(ctypes.byref(h), int(sys_ptr.size - 1), _ptr(sys_ptr),
                                         C.n, int(rowptr[-1]), _ptr(rowptr), _ptr(col), _ptr(val),
                                         int(reps), ctypes.byref(rep)), "ps_autotune_layout")
        return cls(sys_ptr, C.n, rowptr, None, None, _handle=h), rep.rows()

    def solve(self, b, x0=None, tol=1e-8, maxit=10_000, variant="pbicgsafe", hist=True, **opt):
        b = np.ascontiguousarray(b, dtype=np.float64)
        x0a = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
        x = np.empty(self.n)
        h = np.empty((self.nsys, maxit + 1)) if hist else None
        iters = np.zeros(self.nsys, dtype=np.int32)
        status = np.zeros(self.nsys, dtype=np.int32)
        o = options(**opt)
        _check(_lib().ps_solve_batch(self._h, _ptr(b), None if x0a is None else _ptr(x0a),
                                     float(tol), int(maxit), _vid(variant), ctypes.byref(o), _ptr(x),
                                     _ptr(iters), None if h is None else _ptr(h), _ptr(status)),
               "ps_solve_batch")
        return BatchResult(x, iters, status, h)

    def solve_dev(self, b, x0=None, x=None, tol=1e-8, maxit=10_000, variant="pbicgsafe",
                  hist=True, stream=None, **opt):
        import torch
        for t in (b, x0, x):
            if t is not None and (t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous()
                                  or t.numel() != self.n):
                raise ValueError("expected contiguous float64 CUDA tensors of length n")
        if x is None:
            x = torch.empty(self.n, dtype=torch.float64, device=b.device)
        if stream is None:
            stream = torch.cuda.current_stream(b.device).cuda_stream
        h = np.empty((self.nsys, maxit + 1)) if hist else None
        iters = np.zeros(self.nsys, dtype=np.int32)
        status = np.zeros(self.nsys, dtype=np.int32)
        o = options(stream=stream, **opt)
        _check(_lib().ps_solve_batch_dev(self._h, ctypes.c_void_p(b.data_ptr()),
                                         None if x0 is None else ctypes.c_void_p(x0.data_ptr()),
                                         float(tol), int(maxit), _vid(variant), ctypes.byref(o),
                                         ctypes.c_void_p(x.data_ptr()), _ptr(iters),
                                         None if h is None else _ptr(h), _ptr(status)),
               "ps_solve_batch_dev")
        return BatchResult(x, iters, status, h)


def stream_copy(dst, src, stream=None):
    """dst[:] = src[:] for torch CUDA tensors with the library's streaming copy kernel."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(src.device).cuda_stream
    nbytes = src.numel() * src.element_size()
    _check(_lib().ps_stream_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()),
                                 nbytes, ctypes.c_void_p(stream)), "ps_stream_copy")
