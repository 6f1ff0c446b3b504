"""Multi-core FP64 CPU tools (``katz_cpu.c``) -- TEST INFRASTRUCTURE ONLY.

Imported by the test suite and the benchmark's CPU leg only.  Three tools:

* :func:`katz_series_mt` -- the oracle at benchmark sizes: the truncated
  Neumann series k_q = sum_{l>=1} (beta A)^l e_q (Section 3.1, eq.
  KatzMatrix applied to e_q) with the rigorous tail bound
  ||v_L|| c / (1 - c) <= tol ||k||, OpenMP over rows, several queries at once;
* :func:`cg_mt` -- the CPU baseline: plain conjugate gradients on
  (I - beta A) k = beta A e_q (eq. LinearSystem; the paper's comparison
  method), multi-RHS, same stop rule as the GPU path (true FP64 residual).

* :func:`lambda_max_mt` -- lambda_max(A) by Lanczos with an OpenMP SpMV,
  for graphs where the single-threaded scipy eigensolve takes minutes
  (Sec. 3.1: beta < 1 / lambda_max; c = beta * lambda_max).

The first two return node-major results as an (n, B) array (column j = query j).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "katz_cpu.c")
_LIB = os.path.join(_HERE, "libkatz_cpu.so")
_lib = None


def build(force: bool = True) -> str:
    """Compiles katz_cpu.c (plain C + OpenMP, host only) next to this file."""
    global _lib
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
        _lib = None
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=False)
    lib = ctypes.CDLL(_LIB)
    i32, dbl, P = ctypes.c_int32, ctypes.c_double, ctypes.c_void_p
    lib.ko_series.restype = ctypes.c_int
    lib.ko_series.argtypes = [i32, P, P, P, dbl, dbl, i32, P, dbl, i32, i32, P, P, P, P]
    lib.ko_lambda_max.restype = ctypes.c_int
    lib.ko_lambda_max.argtypes = [i32, P, P, P, i32, dbl, i32, P, P, P]
    lib.ko_cg.restype = ctypes.c_int
    lib.ko_cg.argtypes = [i32, P, P, P, dbl, i32, P, dbl, i32, i32, P, P, P, P]
    _lib = lib
    return lib


def _csr(row_ptr, col, val):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    vv = None if val is None else np.ascontiguousarray(val, dtype=np.float64)
    return rp, cl, vv


def _ptr(a):
    return None if a is None else a.ctypes.data


def katz_series_mt(n, row_ptr, col, qs, beta, c, val=None, tol=1e-13, max_terms=100000, threads=0):
    """Katz vectors of the queries qs by the truncated Neumann series (see the
    module docstring).  c = beta * lambda_max(A) must be passed by the caller
    (it sets the tail bound).  Returns {"k": (n, B), "terms": (B,),
    "tail": (B,) absolute tail bounds, "threads": OpenMP threads used}."""
    lib = _load()
    rp, cl, vv = _csr(row_ptr, col, val)
    q = np.ascontiguousarray(np.atleast_1d(qs), dtype=np.int32)
    B = len(q)
    k = np.empty((n, B), dtype=np.float64)
    terms = np.zeros(B, dtype=np.int32)
    tail = np.zeros(B, dtype=np.float64)
    used = np.zeros(1, dtype=np.int32)
    rc = lib.ko_series(n, _ptr(rp), _ptr(cl), _ptr(vv), float(beta), float(c), B, _ptr(q), float(tol),
                       int(max_terms), int(threads), _ptr(k), _ptr(terms), _ptr(tail), _ptr(used))
    if rc == -1:
        raise ValueError("ko_series: bad arguments (need 0 < c < 1, beta > 0, ids in range)")
    if rc == -2:
        raise RuntimeError("ko_series: tail bound not reached within %d terms" % max_terms)
    return {"k": k, "terms": terms, "tail": tail, "threads": int(used[0])}


def cg_mt(n, row_ptr, col, qs, beta, val=None, tol=1e-6, max_iter=1000, threads=0):
    """Plain FP64 CG on (I - beta A) k = beta A e_q for the queries qs.
    Returns {"k": (n, B), "iters": (B,), "rel_residual": (B,) true FP64
    residuals, "threads": OpenMP threads used, "converged": bool}."""
    lib = _load()
    rp, cl, vv = _csr(row_ptr, col, val)
    q = np.ascontiguousarray(np.atleast_1d(qs), dtype=np.int32)
    B = len(q)
    x = np.empty((n, B), dtype=np.float64)
    iters = np.zeros(B, dtype=np.int32)
    rel = np.zeros(B, dtype=np.float64)
    used = np.zeros(1, dtype=np.int32)
    rc = lib.ko_cg(n, _ptr(rp), _ptr(cl), _ptr(vv), float(beta), B, _ptr(q), float(tol), int(max_iter),
                   int(threads), _ptr(x), _ptr(iters), _ptr(rel), _ptr(used))
    if rc == -1:
        raise ValueError("ko_cg: bad arguments")
    return {"k": x, "iters": iters, "rel_residual": rel, "threads": int(used[0]), "converged": rc == 0}


def lambda_max_mt(n, row_ptr, col, val=None, tol=1e-12, max_steps=400, threads=0):
    """lambda_max(A) of a symmetric nonnegative CSR matrix by the Lanczos
    iteration from the all-ones vector (see the module docstring).  Stops when
    the largest Ritz value changes by at most `tol` (relative) in two
    consecutive steps.  Returns {"lambda": float, "steps": int, "threads":
    int}; raises if max_steps ended the run first."""
    lib = _load()
    rp, cl, vv = _csr(row_ptr, col, val)
    lam = np.zeros(1, dtype=np.float64)
    steps = np.zeros(1, dtype=np.int32)
    used = np.zeros(1, dtype=np.int32)
    rc = lib.ko_lambda_max(int(n), _ptr(rp), _ptr(cl), _ptr(vv), int(max_steps), float(tol), int(threads),
                           _ptr(lam), _ptr(steps), _ptr(used))
    if rc == -1:
        raise ValueError("ko_lambda_max: bad arguments")
    if rc == -2:
        raise RuntimeError("ko_lambda_max: not converged in %d steps (last %.17g)" % (max_steps, lam[0]))
    return {"lambda": float(lam[0]), "steps": int(steps[0]), "threads": int(used[0])}
