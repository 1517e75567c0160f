"""ctypes front end of the FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and
the benchmark's CPU-baseline leg, never by the product path.  It shares no
code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "oracle.c")
LIB = os.path.join(_HERE, "liboracle.so")

SSBICGSAFE2, PBICGSAFE, PBICGSAFE_RR, PBICGSTAB, BICGSTAB = 0, 1, 2, 3, 4
VARIANTS = {"ssbicgsafe2": 0, "pbicgsafe": 1, "pbicgsafe_rr": 2, "pbicgstab": 3, "bicgstab": 4}
CONVERGED, MAXIT, BREAKDOWN, NONFINITE = 0, 1, 2, 3

# state layout (follows the enums at the top of oracle.c)
VEC = ["x", "r", "rs", "s", "y", "t", "p", "u", "z", "w", "l", "g", "q", "o", "As", "Aw", "v", "tmp"]
SCAL = ["alpha", "beta", "zeta", "eta", "omega", "f", "rhoref", "rho", "nspmv", "ndot", "nphase",
        "pending_breakdown", "gs", "gw", "gz"]
NCOEF = 8
COEF = ["alpha", "beta", "zeta", "eta", "omega", "rho", "f", "spare"]
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared"]


def build(src: str = SRC, out: str = LIB) -> str:
    """Compile the oracle with gcc (plain -O2, no FMA contraction, OpenMP)."""
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, src, "-lm"])
    os.replace(tmp, out)
    return out


def _vid(variant):
    return VARIANTS[variant] if isinstance(variant, str) else int(variant)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _csr(A):
    rowptr = np.ascontiguousarray(A.rowptr, dtype=np.int64)
    col = np.ascontiguousarray(A.col, dtype=np.int32)
    val = np.ascontiguousarray(A.val, dtype=np.float64)
    return rowptr, col, val


class Result:
    def __init__(self, **kw):
        self.__dict__.update(kw)


class State:
    """The oracle's full iteration state: NV vectors and NS scalars."""

    def __init__(self, n):
        self.n = n
        self.V = np.zeros((len(VEC), n))
        self.S = np.zeros(len(SCAL))

    def vec(self, name):
        return self.V[VEC.index(name)]

    def scal(self, name):
        return float(self.S[SCAL.index(name)])

    def set_scal(self, name, value):
        self.S[SCAL.index(name)] = value

    def copy(self):
        s = State(self.n)
        s.V[...] = self.V
        s.S[...] = self.S
        return s


class Oracle:
    """One loaded build of ``oracle.c``."""

    def __init__(self, path: str = LIB):
        if not os.path.exists(path):
            if path == LIB:
                build()
            else:
                raise FileNotFoundError(path)
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i64, f64, cint = ctypes.c_int64, ctypes.c_double, ctypes.c_int
        L.orc_setup.argtypes = [cint, cint, i64, P, P, P, P, P, cint, cint, P, P]
        L.orc_setup.restype = cint
        L.orc_run.argtypes = [cint, cint, i64, P, P, P, P, P, P, i64, i64, f64, i64, i64, P, P, P, P]
        L.orc_run.restype = cint
        L.orc_solve.argtypes = [cint, cint, i64, P, P, P, P, P, cint, f64, i64, i64, i64, cint, P, P, P,
                                P, P, P]
        L.orc_solve.restype = cint
        L.orc_spmv.argtypes = [i64, P, P, P, P, P]
        L.orc_spmv.restype = None
        L.orc_dot.argtypes = [i64, P, P]
        L.orc_dot.restype = f64
        L.orc_set_threads.argtypes = [cint]
        L.orc_set_threads.restype = None
        L.orc_threads.argtypes = []
        L.orc_threads.restype = cint
        if L.orc_nv() != len(VEC) or L.orc_ns() != len(SCAL):
            raise RuntimeError("oracle state layout mismatch")
        self.L = L

    def spmv(self, A, x):
        rowptr, col, val = _csr(A)
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.empty(A.n)
        self.L.orc_spmv(A.n, _p(rowptr), _p(col), _p(val), _p(x), _p(y))
        return y

    def dot(self, u, v):
        """The oracle's inner product (u, v): the exact sum of the products rounded once."""
        u = np.ascontiguousarray(u, dtype=np.float64)
        v = np.ascontiguousarray(v, dtype=np.float64)
        assert u.shape == v.shape and u.ndim == 1
        return float(self.L.orc_dot(u.size, _p(u), _p(v)))

    def set_threads(self, n):
        """OpenMP threads of later calls (results do not depend on it)."""
        self.L.orc_set_threads(int(n))

    def threads(self):
        return int(self.L.orc_threads())

    def solve(self, A, b=None, x0=None, tol=1e-8, maxit=10_000, variant="pbicgsafe", rr_m=100,
              rr_M=None, norm_ref=0, precision=0, x0_mode=0):
        """Full solve: x, iters, status, hist[0..iters], coef[0..iters) and operation counters.

        precision: 0 FP64; 1 every product with the matrix values rounded to FP32;
        2 the residual statements (set-up, replacement steps) with the FP64 values and every
        other product with the rounded ones; 3 as 2 with p, u, z held in FP32 (p-BiCGSafe(-rr)).
        x0_mode (with x0): 0 as given; 1 replaced by 0 if ||b - A x0|| > ||b||; 2 first
        scaled by (A x0, b)/(A x0, A x0), then the rule of 1 (see oracle.c)."""
        rowptr, col, val = _csr(A)
        b = np.ascontiguousarray(A.b if b is None else b, dtype=np.float64)
        x0a = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
        x = np.empty(A.n)
        iters = ctypes.c_int64()
        status = ctypes.c_int32()
        hist = np.full(maxit + 1, np.nan)
        coef = np.zeros((maxit + 1, NCOEF))
        counters = np.zeros(3)
        rc = self.L.orc_solve(_vid(variant), precision, A.n, _p(rowptr), _p(col), _p(val), _p(b),
                              _p(x0a), x0_mode, tol, maxit, rr_m, maxit if rr_M is None else rr_M,
                              norm_ref, _p(x),
                              ctypes.byref(iters), _p(hist), _p(coef), ctypes.byref(status),
                              _p(counters))
        if rc != 0:
            raise RuntimeError(f"orc_solve failed: {rc}")
        it = iters.value
        return Result(x=x, iters=it, status=status.value, hist=hist[: it + 1], coef=coef[:it],
                      nspmv=int(counters[0]), ndot=int(counters[1]), nphase=int(counters[2]))

    def setup(self, A, b=None, x0=None, variant="pbicgsafe", norm_ref=0, precision=0,
              x0_mode=0) -> State:
        rowptr, col, val = _csr(A)
        b = np.ascontiguousarray(A.b if b is None else b, dtype=np.float64)
        x0a = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
        st = State(A.n)
        rc = self.L.orc_setup(_vid(variant), precision, A.n, _p(rowptr), _p(col), _p(val), _p(b),
                              _p(x0a), x0_mode, norm_ref, _p(st.V), _p(st.S))
        if rc != 0:
            raise RuntimeError(f"orc_setup failed: {rc}")
        return st

    def run(self, A, st: State, i_begin, maxit, b=None, tol=0.0, variant="pbicgsafe", rr_m=100,
            rr_M=None, precision=0):
        """Advance ``st`` in place from iteration ``i_begin`` until a stop (at the latest i = maxit)."""
        rowptr, col, val = _csr(A)
        b = np.ascontiguousarray(A.b if b is None else b, dtype=np.float64)
        iters = ctypes.c_int64()
        status = ctypes.c_int32()
        hist = np.full(maxit + 1, np.nan)
        coef = np.zeros((maxit + 1, NCOEF))
        rc = self.L.orc_run(_vid(variant), precision, A.n, _p(rowptr), _p(col), _p(val), _p(b),
                            _p(st.V), _p(st.S), i_begin, maxit, tol, rr_m,
                            maxit if rr_M is None else rr_M, ctypes.byref(iters), _p(hist),
                            _p(coef), ctypes.byref(status))
        if rc != 0:
            raise RuntimeError(f"orc_run failed: {rc}")
        return Result(iters=iters.value, status=status.value, hist=hist, coef=coef)

    def state_at(self, A, i, variant="pbicgsafe", b=None, x0=None, rr_m=100, rr_M=None,
                 precision=0):
        """State at the start of iteration ``i`` (the solve stopped there with status MAXIT)."""
        st = self.setup(A, b=b, x0=x0, variant=variant, precision=precision)
        res = self.run(A, st, 0, i, b=b, tol=0.0, variant=variant, rr_m=rr_m, rr_M=rr_M,
                       precision=precision)
        return st, res


_default = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default


def solve(*a, **k):
    return default().solve(*a, **k)


def setup(*a, **k):
    return default().setup(*a, **k)


def run(*a, **k):
    return default().run(*a, **k)


def spmv(*a, **k):
    return default().spmv(*a, **k)


def state_at(*a, **k):
    return default().state_at(*a, **k)
