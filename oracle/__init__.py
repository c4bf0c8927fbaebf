"""FP64 CPU oracle for the k-means hot path -- test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package.  It shares no code with the GPU library: the arithmetic lives in
``knor_oracle.c`` (plain C, FP64, no FMA contraction), loaded here through
ctypes.  Inputs arrive as float64 arrays (every storage dtype upcasts to FP64
exactly).

Functions and the passage each follows (Mhembere et al., HPDC'17):
  dist2            squared Euclidean distance     -- Section "Nomenclature"
  assign           nearest centroid, strict "<"   -- Algorithm 1
  update           member means, empty keeps      -- Section "Parallel Lloyd's
                                                     Algorithm", Phase II
  fit              Lloyd's loop                   -- Sections "Introduction",
                                                     "Parallel Lloyd's Algorithm"
  mti_fit          Lloyd's with MTI Clauses 1-3   -- Section "Minimal Triangle
                                                     Inequality (MTI) Pruning"
  cc_bounds        s(c) = 1/2 min_{j!=c} d(c, j)  -- same section
  update_exact,    the member mean rounded once   -- Phase II, second reading:
  exact_mean,      (ties to even) from an exact      the mean itself, free of
  fit_exact_mean   fixed-point sum                   any summation order
  canonical_sum    the fixed summation order used for sums of many terms
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "knor_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
          "-shared", "-Wall"]


def build(force: bool = True) -> str:
    """Compile knor_oracle.c into liboracle.so with gcc (FP64, no contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Trace(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("changed", ctypes.c_void_p), ("objective", ctypes.c_void_p),
                ("ndist", ctypes.c_void_p), ("pruned1", ctypes.c_void_p),
                ("label_hist", ctypes.c_void_p),
                ("bound_violations", ctypes.c_int32)]


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


@dataclasses.dataclass
class FitResult:
    C: np.ndarray
    labels: np.ndarray
    iters: int
    converged: bool
    changed: np.ndarray
    objective: np.ndarray | None
    ndist: np.ndarray
    pruned1: np.ndarray
    label_hist: np.ndarray | None
    bound_violations: int


class Oracle:
    """The oracle's entry points bound to one compiled copy of knor_oracle.c
    (the default copy is liboracle.so next to this file)."""

    def __init__(self, path: str = _LIB):
        if path == _LIB and not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i64, f64 = ctypes.c_int64, ctypes.c_double
        L.oracle_dist2.argtypes = [P, P, ctypes.c_int]
        L.oracle_dist2.restype = f64
        L.oracle_assign.argtypes = [P, i64, ctypes.c_int, P, ctypes.c_int, P, P]
        L.oracle_update.argtypes = [P, i64, ctypes.c_int, P, ctypes.c_int, P, P, P]
        for fn in (L.oracle_fit, L.oracle_mti_fit):
            fn.argtypes = [P, i64, ctypes.c_int, ctypes.c_int, P, ctypes.c_int,
                           f64, P, P, ctypes.POINTER(_Trace)]
        L.oracle_update_exact.argtypes = [P, i64, ctypes.c_int, P, ctypes.c_int, P, P, P]
        L.oracle_exact_mean.argtypes = [P, i64]
        L.oracle_exact_mean.restype = f64
        L.oracle_fit_ex.argtypes = [P, i64, ctypes.c_int, ctypes.c_int, P, ctypes.c_int,
                                    f64, ctypes.c_int, ctypes.c_int, P, P,
                                    ctypes.POINTER(_Trace)]
        L.oracle_cc_bounds.argtypes = [P, ctypes.c_int, ctypes.c_int, P]
        L.oracle_canonical_sum.argtypes = [P, i64]
        L.oracle_canonical_sum.restype = f64
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_objective.argtypes = [P, i64, ctypes.c_int, P, P]
        L.oracle_objective.restype = f64
        self.L = L

    def num_threads(self) -> int:
        return int(self.L.oracle_num_threads())

    def set_threads(self, t: int) -> None:
        self.L.oracle_set_threads(int(t))

    def dist2(self, x, c) -> float:
        x, c = _f64(x), _f64(c)
        return float(self.L.oracle_dist2(_ptr(x), _ptr(c), x.shape[-1]))

    def assign(self, X, C):
        """(labels int32[n], D float64[n]) with D = D(x, c_label)."""
        X, C = _f64(X), _f64(C)
        n, d = X.shape
        k = C.shape[0]
        lab = np.empty(n, np.int32)
        D = np.empty(n, np.float64)
        _check(self.L.oracle_assign(_ptr(X), n, d, _ptr(C), k, _ptr(lab),
                                    _ptr(D)), "assign")
        return lab, D

    def update(self, X, labels, C_prev):
        """(C_new float64[k,d], counts int64[k])."""
        X, C_prev = _f64(X), _f64(C_prev)
        labels = np.ascontiguousarray(labels, dtype=np.int32)
        n, d = X.shape
        k = C_prev.shape[0]
        C = np.empty((k, d), np.float64)
        cnt = np.empty(k, np.int64)
        _check(self.L.oracle_update(_ptr(X), n, d, _ptr(labels), k,
                                    _ptr(C_prev), _ptr(C), _ptr(cnt)), "update")
        return C, cnt

    def update_exact(self, X, labels, C_prev):
        """(C_new, counts) with each centroid the exactly rounded mean."""
        X, C_prev = _f64(X), _f64(C_prev)
        labels = np.ascontiguousarray(labels, dtype=np.int32)
        n, d = X.shape
        k = C_prev.shape[0]
        C = np.empty((k, d), np.float64)
        cnt = np.empty(k, np.int64)
        _check(self.L.oracle_update_exact(_ptr(X), n, d, _ptr(labels), k,
                                          _ptr(C_prev), _ptr(C), _ptr(cnt)), "update_exact")
        return C, cnt

    def exact_mean(self, v) -> float:
        v = _f64(v)
        return float(self.L.oracle_exact_mean(_ptr(v), v.size))

    def canonical_sum(self, v) -> float:
        v = _f64(v)
        return float(self.L.oracle_canonical_sum(_ptr(v), v.size))

    def objective(self, X, C, labels) -> float:
        """Canonical sum over points of D(x_p, c_{labels[p]})."""
        X, C = _f64(X), _f64(C)
        labels = np.ascontiguousarray(labels, dtype=np.int32)
        n, d = X.shape
        return float(self.L.oracle_objective(_ptr(X), n, d, _ptr(C),
                                             _ptr(labels)))

    def cc_bounds(self, C):
        C = _f64(C)
        k, d = C.shape
        s = np.empty(k, np.float64)
        _check(self.L.oracle_cc_bounds(_ptr(C), k, d, _ptr(s)), "cc_bounds")
        return s

    def _fit(self, fn, X, C0, max_iters, tol, history, objective, extra=()):
        X, C0 = _f64(X), _f64(C0)
        n, d = X.shape
        k = C0.shape[0]
        C = np.empty((k, d), np.float64)
        lab = np.empty(n, np.int32)
        ch = np.zeros(max_iters, np.int64)
        ob = np.zeros(max_iters, np.float64) if objective else None
        nd = np.zeros(max_iters, np.int64)
        p1 = np.zeros(max_iters, np.int64)
        hist = np.zeros((max_iters, n), np.int32) if history else None
        tr = _Trace(0, 0, ch.ctypes.data,
                    ob.ctypes.data if ob is not None else None,
                    nd.ctypes.data, p1.ctypes.data,
                    hist.ctypes.data if hist is not None else None, 0)
        _check(fn(_ptr(X), n, d, k, _ptr(C0), max_iters, float(tol), *extra, _ptr(C),
                  _ptr(lab), ctypes.byref(tr)), "fit")
        it = tr.iters
        return FitResult(C=C, labels=lab, iters=it,
                         converged=bool(tr.converged), changed=ch[:it],
                         objective=None if ob is None else ob[:it],
                         ndist=nd[:it], pruned1=p1[:it],
                         label_hist=None if hist is None else hist[:it],
                         bound_violations=int(tr.bound_violations))

    def fit(self, X, C0, max_iters, tol=0.0, history=False, objective=True):
        """Plain FP64 Lloyd's from C0."""
        return self._fit(self.L.oracle_fit, X, C0, max_iters, tol, history,
                         objective)

    def mti_fit(self, X, C0, max_iters, tol=0.0, history=False, objective=True,
                exact_mean=False):
        """FP64 Lloyd's with MTI Clauses 1-3 (labels equal plain Lloyd's);
        exact_mean=True: centroids are exactly rounded means."""
        if exact_mean:
            return self._fit(self.L.oracle_fit_ex, X, C0, max_iters, tol, history,
                             objective, extra=(1, 1))
        return self._fit(self.L.oracle_mti_fit, X, C0, max_iters, tol, history,
                         objective)

    def fit_exact_mean(self, X, C0, max_iters, tol=0.0, history=False, objective=True):
        """Plain FP64 Lloyd's with exactly rounded means."""
        return self._fit(self.L.oracle_fit_ex, X, C0, max_iters, tol, history,
                         objective, extra=(0, 1))


_default = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default


def lib():
    return default().L


def num_threads():
    return default().num_threads()


def set_threads(t):
    default().set_threads(t)


def dist2(x, c):
    return default().dist2(x, c)


def assign(X, C):
    return default().assign(X, C)


def update(X, labels, C_prev):
    return default().update(X, labels, C_prev)


def update_exact(X, labels, C_prev):
    return default().update_exact(X, labels, C_prev)


def exact_mean(v):
    return default().exact_mean(v)


def canonical_sum(v):
    return default().canonical_sum(v)


def cc_bounds(C):
    return default().cc_bounds(C)


def objective(X, C, labels):
    return default().objective(X, C, labels)


def fit(X, C0, max_iters, tol=0.0, history=False, objective=True):
    return default().fit(X, C0, max_iters, tol, history, objective)


def mti_fit(X, C0, max_iters, tol=0.0, history=False, objective=True, exact_mean=False):
    return default().mti_fit(X, C0, max_iters, tol, history, objective, exact_mean)


def fit_exact_mean(X, C0, max_iters, tol=0.0, history=False, objective=True):
    return default().fit_exact_mean(X, C0, max_iters, tol, history, objective)
