"""Seeded synthetic inputs for the Katz workloads.

This package only *produces inputs*: undirected simple graphs in CSR form and
seeded query-node lists.  It contains none of the Katz method's arithmetic and
is shared, unchanged, by the CPU oracle tests and by the HIP library's tests
and benchmark.  The generators are C (``gen.c``), built into
``libkatz_inputs.so`` next to this file.

Workloads (graph family, sizes, damping ``c = beta * lambda_max``):

* ``sbm2k``    - SBM, 2,000 nodes, 10 communities of 200, p_in 0.05, p_out 0.001;
                 c = 0.5, one query, FP64 to relative residual 1e-10.
* ``cl1m``     - Chung-Lu, 1M nodes, exponent 2.5, mean degree 20;
                 c in {0.1, 0.5, 0.9}, rank 32, one query per solve.
* ``lnsbm4m``  - SBM, 4M nodes, 2,000 communities of lognormal size
                 (median 1,500, sigma 1.0), mean degree 16 of which 85% intra;
                 c = 0.5, 256 queries solved together.
* ``cl8m``     - Chung-Lu, 8M nodes, exponent 2.3, mean degree 12; c = 0.9,
                 512 queries, mixed precision.
* ``dcsbm16m`` - degree-corrected SBM hybrid, 16M nodes, mean degree 25,
                 85% of the edge mass intra-community; c = 0.5, serving.

Every workload accepts a ``scale`` (0 < scale <= 1) that shrinks the node
count while keeping degrees and community shapes, for quick tests.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libkatz_inputs.so")
_lib = None


def build(force: bool = True) -> str:
    """Compiles gen.c into libkatz_inputs.so (plain C, host only)."""
    global _lib
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
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
    P = ctypes.c_void_p
    i32, i64, u64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    pi32 = ctypes.POINTER(ctypes.c_int32)
    pdbl = ctypes.POINTER(ctypes.c_double)
    lib.kg_sbm.restype = P
    lib.kg_sbm.argtypes = [i32, pi32, pdbl, dbl, u64, ctypes.c_int]
    lib.kg_chung_lu.restype = P
    lib.kg_chung_lu.argtypes = [i32, dbl, dbl, u64, ctypes.c_int]
    lib.kg_dcsbm.restype = P
    lib.kg_dcsbm.argtypes = [i32, pi32, dbl, dbl, dbl, u64, ctypes.c_int]
    lib.kg_wrap_csr.restype = P
    lib.kg_wrap_csr.argtypes = [i32, pi32, pi32]
    lib.kg_lognormal_sizes.restype = ctypes.c_int
    lib.kg_lognormal_sizes.argtypes = [i32, i32, dbl, dbl, i32, u64, pi32]
    lib.kg_graph_n.restype = i32
    lib.kg_graph_n.argtypes = [P]
    lib.kg_graph_nnz.restype = i64
    lib.kg_graph_nnz.argtypes = [P]
    lib.kg_graph_ncomm.restype = i32
    lib.kg_graph_ncomm.argtypes = [P]
    lib.kg_graph_copy.restype = None
    lib.kg_graph_copy.argtypes = [P, pi32, pi32, pi32]
    lib.kg_graph_free.restype = None
    lib.kg_graph_free.argtypes = [P]
    lib.kg_sample_queries.restype = i32
    lib.kg_sample_queries.argtypes = [P, i32, u64, pi32]
    _lib = lib
    return lib


def _p32(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _pd(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Graph:
    """Undirected simple graph, symmetric CSR with sorted rows (int32)."""
    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    labels: Optional[np.ndarray] = None
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)


def _take(h, name, meta) -> Graph:
    lib = _load()
    if not h:
        raise RuntimeError("graph generator failed (invalid sizes or out of memory)")
    try:
        n = lib.kg_graph_n(h)
        nnz = lib.kg_graph_nnz(h)
        rp = np.empty(n + 1, np.int32)
        col = np.empty(nnz, np.int32)
        labels = np.empty(n, np.int32) if lib.kg_graph_ncomm(h) > 0 else None
        lib.kg_graph_copy(h, _p32(rp), _p32(col), _p32(labels) if labels is not None else None)
    finally:
        lib.kg_graph_free(h)
    return Graph(n, rp, col, labels, name, meta)


def sbm(sizes, p_in, p_out: float, seed: int, relabel: bool = True, name: str = "sbm") -> Graph:
    sizes = np.ascontiguousarray(sizes, np.int32)
    p_in = np.ascontiguousarray(np.broadcast_to(np.asarray(p_in, np.float64), sizes.shape))
    h = _load().kg_sbm(len(sizes), _p32(sizes), _pd(p_in), float(p_out), seed, int(relabel))
    return _take(h, name, {"family": "sbm", "seed": seed, "p_out": p_out})


def lognormal_sizes(ncomm: int, n_total: int, median: float, sigma: float, seed: int,
                    min_size: int = 2) -> np.ndarray:
    out = np.empty(ncomm, np.int32)
    rc = _load().kg_lognormal_sizes(ncomm, n_total, math.log(median), sigma, min_size, seed, _p32(out))
    if rc != 0:
        raise ValueError("lognormal_sizes: infeasible parameters")
    return out


def chung_lu(n: int, gamma: float, mean_deg: float, seed: int, relabel: bool = True,
             name: str = "chung_lu") -> Graph:
    h = _load().kg_chung_lu(n, gamma, mean_deg, seed, int(relabel))
    return _take(h, name, {"family": "chung_lu", "gamma": gamma, "mean_deg": mean_deg, "seed": seed})


def dcsbm(sizes, gamma: float, mean_deg: float, f_in: float, seed: int, relabel: bool = True,
          name: str = "dcsbm") -> Graph:
    sizes = np.ascontiguousarray(sizes, np.int32)
    h = _load().kg_dcsbm(len(sizes), _p32(sizes), gamma, mean_deg, f_in, seed, int(relabel))
    return _take(h, name, {"family": "dcsbm", "gamma": gamma, "mean_deg": mean_deg, "f_in": f_in,
                           "seed": seed})


def from_edges(n: int, edges) -> Graph:
    """Symmetric CSR from an undirected edge list (self loops and duplicates dropped)."""
    e = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    e = e[e[:, 0] != e[:, 1]]
    u = np.concatenate([e[:, 0], e[:, 1]])
    v = np.concatenate([e[:, 1], e[:, 0]])
    key = np.unique(u * n + v)
    u, v = key // n, key % n
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, u + 1, 1)
    rp = np.cumsum(rp).astype(np.int32)
    return Graph(n, rp, v.astype(np.int32), None, "edges")


def edge_weights(g: Graph, seed: int, lo: float = 0.25, hi: float = 2.0) -> np.ndarray:
    """Positive FP64 weights for the CSR entries of g, one value per undirected
    edge so that the weighted matrix stays symmetric: uniform in [lo, hi) from
    the splitmix64 finaliser of (min(u, v) * n + max(u, v)) xor the seed."""
    rows = np.repeat(np.arange(g.n, dtype=np.int64), g.degrees())
    c = g.col.astype(np.int64)
    key = (np.minimum(rows, c) * np.int64(g.n) + np.maximum(rows, c)).astype(np.uint64)
    with np.errstate(over="ignore"):
        z = key ^ (np.uint64(seed) * np.uint64(0x9E3779B97F4A7C15))
        z = z + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    u01 = (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return lo + (hi - lo) * u01


def sample_queries(g: Graph, k: int, seed: int) -> np.ndarray:
    """k distinct nodes of degree >= 1, uniform, seeded (draw order kept)."""
    lib = _load()
    h = lib.kg_wrap_csr(g.n, _p32(np.ascontiguousarray(g.row_ptr, np.int32)),
                        _p32(np.ascontiguousarray(g.col, np.int32)))
    if not h:
        raise MemoryError
    try:
        out = np.empty(max(k, 1), np.int32)
        m = lib.kg_sample_queries(h, k, seed, _p32(out))
    finally:
        lib.kg_graph_free(h)
    return out[:m].copy()


# --------------------------------------------------------------- workloads
@dataclass
class Workload:
    name: str
    graph: Graph
    c: tuple            # damping fractions c = beta * lambda_max to run
    batch: int          # queries solved together
    rank: int
    tol: float          # relative residual target
    queries: np.ndarray
    precision: str = "fp64"
    notes: str = ""


def _n(full: int, scale: float) -> int:
    return max(64, int(round(full * scale)))


def workload(name: str, scale: float = 1.0, nq: Optional[int] = None) -> Workload:
    """Builds one of the named workloads (see module docstring)."""
    if name == "sbm2k":
        k = max(2, int(round(10 * scale)))
        g = sbm([200] * k, 0.05, 0.001, seed=1001, name=name)
        q = sample_queries(g, nq or 1, 2001)
        return Workload(name, g, (0.5,), 1, 32, 1e-10, q)
    if name == "cl1m":
        g = chung_lu(_n(1_000_000, scale), 2.5, 20.0, seed=1002, name=name)
        q = sample_queries(g, nq or 100, 2002)
        return Workload(name, g, (0.1, 0.5, 0.9), 1, 32, 1e-6, q)
    if name == "lnsbm4m":
        n = _n(4_000_000, scale)
        ncomm = max(2, int(round(2000 * scale)))
        sizes = lognormal_sizes(ncomm, n, 1500.0, 1.0, seed=1003)
        p_in = np.minimum(1.0, 13.6 / np.maximum(sizes - 1, 1))
        cross = n * (n - 1) / 2 - float(np.sum(sizes.astype(np.float64) * (sizes - 1) / 2))
        p_out = (2.4 * n / 2) / cross
        g = sbm(sizes, p_in, p_out, seed=1003, name=name)
        q = sample_queries(g, nq or 256, 2003)
        return Workload(name, g, (0.5, 0.9), 256, 32, 1e-6, q,
                        notes="per-community p_in = 13.6/(s_c-1); uniform p_out for 2.4 expected inter-degree")
    if name == "cl8m":
        g = chung_lu(_n(8_000_000, scale), 2.3, 12.0, seed=1004, name=name)
        q = sample_queries(g, nq or 512, 2004)
        return Workload(name, g, (0.9,), 512, 64, 1e-6, q, precision="mixed")
    if name == "dcsbm16m":
        n = _n(16_000_000, scale)
        ncomm = max(2, int(round(6470 * scale)))
        sizes = lognormal_sizes(ncomm, n, 1500.0, 1.0, seed=1005)
        g = dcsbm(sizes, 2.5, 25.0, 0.85, seed=1005, name=name)
        q = sample_queries(g, nq or 512, 2005)
        return Workload(name, g, (0.5,), 512, 64, 1e-6, q, precision="mixed")
    raise KeyError(name)
