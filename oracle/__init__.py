"""ORACLE — test infrastructure only.

A plain FP64 CPU implementation of the damped, smoothing-regularised LSQR
solve (Paige & Saunders 1982, the solver the paper's "Solver for the
Large-scale Linear System" section names beside LSMR) of

    min |G x - dt|^2 + w^2 |L x|^2 + lambda^2 |x|^2,

written in plain C (lsqr_oracle.c) with this thin ctypes shim.  Only tests/,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import it.  It imports nothing from the GPU package and shares no code with it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile lsqr_oracle.c with gcc (no FMA contraction, -O2, OpenMP)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-shared", "-fPIC",
                               "-o", tmp, os.path.join(_HERE, "lsqr_oracle.c"), "-lm"])
        os.replace(tmp, _SO)
    return _SO


class _Op(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p),
                ("w", ctypes.c_double), ("damp", ctypes.c_double), ("d", ctypes.c_void_p),
                ("nthreads", ctypes.c_int), ("compensated", ctypes.c_int),
                ("ccol_ptr", ctypes.c_void_p), ("crow", ctypes.c_void_p), ("cval", ctypes.c_void_p)]


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        OP = ctypes.POINTER(_Op)
        lib.oracle_transpose.argtypes = [OP]
        lib.oracle_transpose.restype = ctypes.c_int
        lib.oracle_free.argtypes = [OP]
        lib.oracle_free.restype = None
        lib.oracle_laplacian.argtypes = [ctypes.c_int32] * 3 + [P, P, ctypes.c_int]
        lib.oracle_laplacian.restype = None
        lib.oracle_apply.argtypes = [OP, P, P, P]
        lib.oracle_apply.restype = None
        lib.oracle_apply_t.argtypes = [OP, P, P, P]
        lib.oracle_apply_t.restype = None
        lib.oracle_jacobi.argtypes = [OP, P]
        lib.oracle_jacobi.restype = None
        lib.oracle_lsqr.argtypes = [OP, P, ctypes.c_int, ctypes.c_double, P, P, P, P, P,
                                    ctypes.c_int]
        lib.oracle_lsqr.restype = ctypes.c_int
        lib.oracle_lsqr_ref.argtypes = [OP, P, ctypes.c_int, ctypes.c_double, P, P, P,
                                        ctypes.c_double, P, P, ctypes.c_int]
        lib.oracle_lsqr_ref.restype = ctypes.c_int
        lib.oracle_lsqr_implicit.argtypes = [OP, P, ctypes.c_int, P]
        lib.oracle_lsqr_implicit.restype = ctypes.c_int
        _lib_handle = lib
    return _lib_handle


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


class Operator:
    """Abar D = [G; w L; lambda I] D over a CSR G on an (nx, ny, nz) grid."""

    def __init__(self, row_ptr, col, val, nx, ny, nz, damp, smooth, d=None,
                 compensated=False, nthreads=1):
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.val = np.ascontiguousarray(val, dtype=np.float64)
        self.m = len(self.row_ptr) - 1
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.n = self.nx * self.ny * self.nz
        self.d = None if d is None else np.ascontiguousarray(d, dtype=np.float64)
        self._op = _Op(self.m, self.n, self.nx, self.ny, self.nz, _p(self.row_ptr).value,
                       _p(self.col).value, _p(self.val).value, float(smooth), float(damp),
                       None if self.d is None else _p(self.d).value, int(nthreads),
                       int(bool(compensated)), None, None, None)
        if _lib().oracle_transpose(ctypes.byref(self._op)) != 0:
            raise MemoryError("oracle transpose allocation failed")

    @classmethod
    def from_system(cls, s, d=None, compensated=False, nthreads=1, damp=None, smooth=None):
        return cls(s.row_ptr, s.col, s.val, s.nx, s.ny, s.nz,
                   s.damp if damp is None else damp, s.smooth if smooth is None else smooth,
                   d=d, compensated=compensated, nthreads=nthreads)

    def __del__(self):
        try:
            _lib().oracle_free(ctypes.byref(self._op))
        except Exception:
            pass

    @property
    def mbar(self):
        return self.m + 2 * self.n

    def apply(self, x):
        """ybar = Abar D x (m + 2n entries)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.empty(self.mbar)
        sc = np.empty(self.n)
        _lib().oracle_apply(ctypes.byref(self._op), _p(x), _p(y), _p(sc))
        return y

    def apply_t(self, ybar):
        """x = D Abar^T ybar."""
        ybar = np.ascontiguousarray(ybar, dtype=np.float64)
        assert ybar.shape == (self.mbar,)
        x = np.empty(self.n)
        sc = np.empty(self.n)
        _lib().oracle_apply_t(ctypes.byref(self._op), _p(ybar), _p(x), _p(sc))
        return x

    def jacobi(self):
        """d_j = 1 / |column j of Abar|."""
        d = np.empty(self.n)
        _lib().oracle_jacobi(ctypes.byref(self._op), _p(d))
        return d

    def lsqr(self, dt, iters, tol=0.0, ncap=0):
        """Explicit-block LSQR.  Returns dict(x, hist [K+1, 3], istop, iters, U, V)."""
        dt = np.ascontiguousarray(dt, dtype=np.float64)
        assert dt.shape == (self.m,)
        x = np.empty(self.n)
        hist = np.full((iters + 1, 3), np.nan)
        info = np.zeros(2, dtype=np.int32)
        U = np.zeros((ncap, self.mbar)) if ncap else None
        V = np.zeros((ncap, self.n)) if ncap else None
        rc = _lib().oracle_lsqr(ctypes.byref(self._op), _p(dt), int(iters), float(tol), _p(x),
                                _p(hist), _p(info), _p(U), _p(V), int(ncap))
        if rc != 0:
            raise FloatingPointError(f"oracle_lsqr failed with code {rc}")
        k = int(info[1])
        return dict(x=x, hist=hist[:k + 1], istop=int(info[0]), iters=k, U=U, V=V)

    def lsqr_ref(self, dt, iters, tol, snap_tol, stall=200):
        """LSQR towards a converged reference: stops at eta <= tol, after `iters`,
        or when eta has not reached a new low for `stall` iterations (istop 5);
        also returns the first iterate with eta <= snap_tol (x_snap, k_snap = -1
        if none)."""
        dt = np.ascontiguousarray(dt, dtype=np.float64)
        assert dt.shape == (self.m,)
        x = np.empty(self.n)
        xs = np.full(self.n, np.nan)
        hist = np.full((iters + 1, 3), np.nan)
        info = np.zeros(2, dtype=np.int32)
        ks = np.zeros(1, dtype=np.int32)
        rc = _lib().oracle_lsqr_ref(ctypes.byref(self._op), _p(dt), int(iters), float(tol), _p(x),
                                    _p(hist), _p(info), float(snap_tol), _p(xs), _p(ks),
                                    int(stall))
        if rc != 0:
            raise FloatingPointError(f"oracle_lsqr_ref failed with code {rc}")
        k = int(info[1])
        return dict(x=x, hist=hist[:k + 1], istop=int(info[0]), iters=k, x_snap=xs,
                    k_snap=int(ks[0]))

    def lsqr_implicit(self, dt, iters):
        """Implicit-damp LSQR on [G; w L] with damp lambda (no column scaling)."""
        dt = np.ascontiguousarray(dt, dtype=np.float64)
        x = np.empty(self.n)
        rc = _lib().oracle_lsqr_implicit(ctypes.byref(self._op), _p(dt), int(iters), _p(x))
        if rc != 0:
            raise FloatingPointError(f"oracle_lsqr_implicit failed with code {rc}")
        return x


def laplacian_apply(nx, ny, nz, x, nthreads=1):
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty_like(x)
    _lib().oracle_laplacian(int(nx), int(ny), int(nz), _p(x), _p(y), int(nthreads))
    return y


def lsmr(sys, iters, tol=0.0, d=None, nthreads=1, dt=None):
    """Convenience: explicit-block LSMR (oracle/lsmr.py) on a generated system."""
    from .lsmr import lsmr as _lsmr
    op = Operator.from_system(sys, d=d, nthreads=nthreads)
    return _lsmr(op, sys.dt if dt is None else dt, iters, tol)


def lsqr(sys, iters, tol=0.0, d=None, compensated=False, nthreads=1, ncap=0, dt=None):
    """Convenience: explicit-block LSQR on a generated system."""
    op = Operator.from_system(sys, d=d, compensated=compensated, nthreads=nthreads)
    return op.lsqr(sys.dt if dt is None else dt, iters, tol, ncap)
