"""Query-time Katz proximity on one MI355X: Python binding of libkatz_hip.so.

Argument marshalling only: every step of the query path runs in the HIP
library (``csrc/``), whose C ABI is ``include/katz.h``.  The module-level
functions carry the C names (``katz_index_build``, ``katz_query``,
``katz_topk_links``, ...); ``KatzIndex`` wraps them for convenience.  PyTorch
is used, when given, only for device memory and the current stream.

If the shared library has not been built, importing this package raises: there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkatz_hip.so")

KATZ_OK, KATZ_EINVAL, KATZ_ENOTSYM, KATZ_EDIVERGE, KATZ_ENOMEM = 0, -1, -2, -3, -4
KATZ_EDEVICE, KATZ_ENOCONV, KATZ_EBUSY, KATZ_EIO = -5, -6, -7, -8
KATZ_PREC_FP64, KATZ_PREC_MIXED = 0, 1
KATZ_L_AUTO, KATZ_L_CHOL, KATZ_L_IDENTITY, KATZ_L_IC0 = 0, 1, 2, 3
KATZ_METHOD_LRC, KATZ_METHOD_CG, KATZ_METHOD_PCGNR = 0, 1, 2
KATZ_PATH_LRC, KATZ_PATH_CG, KATZ_PATH_CG_FALLBACK = 0, 1, 2
KATZ_ORDER_AUTO, KATZ_ORDER_DEGREE, KATZ_ORDER_LOCALITY = 0, 1, 2

_STATUS = {0: "KATZ_OK", -1: "KATZ_EINVAL", -2: "KATZ_ENOTSYM", -3: "KATZ_EDIVERGE", -4: "KATZ_ENOMEM",
           -5: "KATZ_EDEVICE", -6: "KATZ_ENOCONV", -7: "KATZ_EBUSY", -8: "KATZ_EIO"}

EXPORTED = ["katz_build_opts_default", "katz_query_opts_default", "katz_index_build", "katz_query",
            "katz_query_noalloc", "katz_communities", "katz_index_rebuild",
            "katz_topk_links", "katz_pair_scores", "katz_sparse_katz", "katz_index_save", "katz_index_load", "katz_index_free", "katz_index_info", "katz_index_partition",
            "katz_index_lowrank", "katz_profile_enable", "katz_profile_reset", "katz_profile_read",
            "katz_server_opts_default", "katz_server_create", "katz_server_submit", "katz_server_poll",
            "katz_server_info", "katz_server_destroy", "katz_last_error"]


class katz_build_opts(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("beta_frac", ctypes.c_double), ("rank", ctypes.c_int32),
                ("max_block", ctypes.c_int32), ("labels", ctypes.POINTER(ctypes.c_int32)),
                ("l_kind", ctypes.c_int32), ("precision", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("device", ctypes.c_int32), ("lanczos_steps", ctypes.c_int32), ("order", ctypes.c_int32),
                ("u_precision", ctypes.c_int32)]


class katz_query_opts(ctypes.Structure):
    _fields_ = [("rel_tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("method", ctypes.c_int32),
                ("max_sweeps", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("force_fallback", ctypes.c_int32)]


class katz_query_stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("sweeps", ctypes.c_int32),
                ("path", ctypes.c_int32), ("rel_residual", ctypes.c_double), ("err_bound", ctypes.c_double)]


class katz_index_info_t(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("n1", ctypes.c_int32), ("n2", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("nblocks", ctypes.c_int32), ("max_block_size", ctypes.c_int32), ("rank", ctypes.c_int32),
                ("l_kind", ctypes.c_int32), ("precision", ctypes.c_int32), ("device", ctypes.c_int32),
                ("beta", ctypes.c_double), ("lambda_max", ctypes.c_double), ("c", ctypes.c_double),
                ("sigma_max", ctypes.c_double), ("sigma_next", ctypes.c_double),
                ("factor_bytes", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("build_seconds", ctypes.c_double), ("u_precision", ctypes.c_int32),
                ("build_phase_seconds", ctypes.c_double * 12)]


class katz_server_opts(ctypes.Structure):
    _fields_ = [("workers", ctypes.c_int32), ("max_batch", ctypes.c_int32), ("hbm_fraction", ctypes.c_double),
                ("k", ctypes.c_int32), ("query", katz_query_opts)]


class katz_server_info_t(ctypes.Structure):
    _fields_ = [("workers", ctypes.c_int32), ("capacity", ctypes.c_int32), ("k", ctypes.c_int32),
                ("queued_queries", ctypes.c_int64), ("live_columns", ctypes.c_int64),
                ("done_queries", ctypes.c_int64), ("done_requests", ctypes.c_int64),
                ("bytes_per_column", ctypes.c_int64)]


class katz_kernel_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("alg_bytes", ctypes.c_double)]


def _load():
    # PyTorch ships its own HIP runtime; load it first so that this library
    # binds to the same runtime instead of bringing a second one into the
    # process (two runtimes cannot share the device).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError("libkatz_hip.so is not built (run __graft_entry__.build() or "
                          "python paper_1912_06525_amd/_build.py); there is no CPU fallback")
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    pi32 = ctypes.POINTER(ctypes.c_int32)
    pdbl = ctypes.POINTER(ctypes.c_double)
    lib.katz_build_opts_default.argtypes = [ctypes.POINTER(katz_build_opts)]
    lib.katz_build_opts_default.restype = None
    lib.katz_query_opts_default.argtypes = [ctypes.POINTER(katz_query_opts)]
    lib.katz_query_opts_default.restype = None
    lib.katz_index_build.argtypes = [i32, i64, pi32, pi32, pdbl, ctypes.POINTER(katz_build_opts),
                                     ctypes.POINTER(P)]
    lib.katz_index_build.restype = ctypes.c_int
    lib.katz_index_rebuild.argtypes = [P, ctypes.POINTER(katz_build_opts), ctypes.POINTER(P)]
    lib.katz_index_rebuild.restype = ctypes.c_int
    lib.katz_communities.argtypes = [i32, i64, pi32, pi32, pdbl, i32, i32, pi32, ctypes.POINTER(i32)]
    lib.katz_communities.restype = ctypes.c_int
    lib.katz_query.argtypes = [P, pi32, i32, ctypes.POINTER(katz_query_opts), P,
                               ctypes.POINTER(katz_query_stats), P]
    lib.katz_query.restype = ctypes.c_int
    lib.katz_query_noalloc.argtypes = [P, pi32, i32, ctypes.POINTER(katz_query_opts), P,
                                       ctypes.POINTER(katz_query_stats), P]
    lib.katz_query_noalloc.restype = ctypes.c_int
    lib.katz_topk_links.argtypes = [P, pi32, i32, i32, ctypes.POINTER(katz_query_opts), P, P,
                                    ctypes.POINTER(katz_query_stats), P]
    lib.katz_topk_links.restype = ctypes.c_int
    lib.katz_sparse_katz.argtypes = [P, pi32, i32, i32, i32, ctypes.POINTER(katz_query_opts), P, P,
                                     ctypes.POINTER(katz_query_stats), P]
    lib.katz_sparse_katz.restype = ctypes.c_int
    lib.katz_pair_scores.argtypes = [P, pi32, pi32, i32, ctypes.POINTER(katz_query_opts), P,
                                     ctypes.POINTER(katz_query_stats), P]
    lib.katz_pair_scores.restype = ctypes.c_int
    lib.katz_index_save.argtypes = [P, ctypes.c_char_p]
    lib.katz_index_save.restype = ctypes.c_int
    lib.katz_index_load.argtypes = [ctypes.c_char_p, i32, ctypes.POINTER(P)]
    lib.katz_index_load.restype = ctypes.c_int
    lib.katz_index_free.argtypes = [P]
    lib.katz_index_free.restype = None
    lib.katz_index_info.argtypes = [P, ctypes.POINTER(katz_index_info_t)]
    lib.katz_index_info.restype = ctypes.c_int
    lib.katz_index_partition.argtypes = [P, pi32, pi32]
    lib.katz_index_partition.restype = ctypes.c_int
    lib.katz_index_lowrank.argtypes = [P, pdbl, pdbl]
    lib.katz_index_lowrank.restype = ctypes.c_int
    lib.katz_profile_enable.argtypes = [ctypes.c_int]
    lib.katz_profile_enable.restype = ctypes.c_int
    lib.katz_profile_reset.argtypes = []
    lib.katz_profile_reset.restype = None
    lib.katz_profile_read.argtypes = [ctypes.POINTER(katz_kernel_stat), ctypes.c_int]
    lib.katz_profile_read.restype = ctypes.c_int
    lib.katz_server_opts_default.argtypes = [ctypes.POINTER(katz_server_opts)]
    lib.katz_server_opts_default.restype = None
    lib.katz_server_create.argtypes = [P, ctypes.POINTER(katz_server_opts), ctypes.POINTER(P)]
    lib.katz_server_create.restype = ctypes.c_int
    lib.katz_server_submit.argtypes = [P, pi32, i32, ctypes.POINTER(ctypes.c_int64)]
    lib.katz_server_submit.restype = ctypes.c_int
    lib.katz_server_poll.argtypes = [P, ctypes.c_int64, pi32, pdbl, ctypes.POINTER(katz_query_stats),
                                     ctypes.POINTER(ctypes.c_double), ctypes.c_int64]
    lib.katz_server_poll.restype = ctypes.c_int
    lib.katz_server_info.argtypes = [P, ctypes.POINTER(katz_server_info_t)]
    lib.katz_server_info.restype = ctypes.c_int
    lib.katz_server_destroy.argtypes = [P]
    lib.katz_server_destroy.restype = None
    lib.katz_last_error.argtypes = []
    lib.katz_last_error.restype = ctypes.c_char_p
    return lib


_lib = _load()


class KatzError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (_STATUS.get(code, str(code)), msg))
        self.code = code


def _check(rc: int) -> int:
    if rc != KATZ_OK:
        raise KatzError(rc, (_lib.katz_last_error() or b"").decode())
    return rc


def _pi32(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if a is not None else None


def _pdbl(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _ptr(buf):
    """Device or host address of a torch tensor or numpy array."""
    if buf is None:
        return None
    if hasattr(buf, "data_ptr"):
        return ctypes.c_void_p(buf.data_ptr())
    return ctypes.c_void_p(buf.ctypes.data)


# ------------------------------------------------------- C-named wrappers
def katz_build_opts_default() -> katz_build_opts:
    o = katz_build_opts()
    _lib.katz_build_opts_default(ctypes.byref(o))
    return o


def katz_query_opts_default() -> katz_query_opts:
    o = katz_query_opts()
    _lib.katz_query_opts_default(ctypes.byref(o))
    return o


def katz_index_build(n: int, row_ptr, col_idx, val=None, opts: Optional[katz_build_opts] = None,
                     _keep=None) -> ctypes.c_void_p:
    rp = np.ascontiguousarray(row_ptr, np.int32)
    col = np.ascontiguousarray(col_idx, np.int32)
    v = None if val is None else np.ascontiguousarray(val, np.float64)
    h = ctypes.c_void_p()
    rc = _lib.katz_index_build(int(n), int(rp[-1]), _pi32(rp), _pi32(col), _pdbl(v),
                               ctypes.byref(opts) if opts is not None else None, ctypes.byref(h))
    _check(rc)
    return h


def katz_communities(n: int, row_ptr, col_idx, val=None, cap: int = 64, passes: int = 8):
    """Louvain local moving with communities capped at `cap` nodes: labels
    (int32 [n]) for KatzIndex(labels=...), and the passes made."""
    rp = np.ascontiguousarray(row_ptr, np.int32)
    col = np.ascontiguousarray(col_idx, np.int32)
    v = None if val is None else np.ascontiguousarray(val, np.float64)
    labels = np.empty(int(n), np.int32)
    done = ctypes.c_int32()
    _check(_lib.katz_communities(int(n), int(rp[-1]), _pi32(rp), _pi32(col), _pdbl(v), int(cap), int(passes),
                                 _pi32(labels), ctypes.byref(done)))
    return labels, int(done.value)


def katz_query(idx, q, opts: Optional[katz_query_opts], scores, stats=None, stream=None) -> int:
    qa = np.ascontiguousarray(q, np.int32)
    st = (katz_query_stats * len(qa))() if stats is None else stats
    rc = _lib.katz_query(idx, _pi32(qa), len(qa), ctypes.byref(opts) if opts is not None else None,
                         _ptr(scores), st, ctypes.c_void_p(stream) if stream else None)
    if rc not in (KATZ_OK, KATZ_ENOCONV):
        _check(rc)
    return rc


def katz_query_noalloc(idx, q, opts: Optional[katz_query_opts], scores, stats=None, stream=None) -> int:
    """katz_query with every solve buffer in the library's static device
    scratch (no allocation); see include/katz.h."""
    qa = np.ascontiguousarray(q, np.int32)
    st = (katz_query_stats * len(qa))() if stats is None else stats
    rc = _lib.katz_query_noalloc(idx, _pi32(qa), len(qa), ctypes.byref(opts) if opts is not None else None,
                                 _ptr(scores), st, ctypes.c_void_p(stream) if stream else None)
    if rc not in (KATZ_OK, KATZ_ENOCONV):
        _check(rc)
    return rc


def katz_topk_links(idx, q, k: int, opts: Optional[katz_query_opts], ids, scores=None, stats=None,
                    stream=None) -> int:
    qa = np.ascontiguousarray(q, np.int32)
    st = (katz_query_stats * len(qa))() if stats is None else stats
    rc = _lib.katz_topk_links(idx, _pi32(qa), len(qa), int(k), ctypes.byref(opts) if opts is not None else None,
                              _ptr(ids), _ptr(scores), st, ctypes.c_void_p(stream) if stream else None)
    if rc not in (KATZ_OK, KATZ_ENOCONV):
        _check(rc)
    return rc


def katz_pair_scores(idx, src, dst, opts: Optional[katz_query_opts], scores, stats=None, stream=None) -> int:
    s = np.ascontiguousarray(src, np.int32)
    d = np.ascontiguousarray(dst, np.int32)
    if s.shape != d.shape:
        raise ValueError("src and dst must have the same length")
    st = (katz_query_stats * len(s))() if stats is None else stats
    rc = _lib.katz_pair_scores(idx, _pi32(s), _pi32(d), len(s), ctypes.byref(opts) if opts is not None else None,
                               _ptr(scores), st, ctypes.c_void_p(stream) if stream else None)
    if rc not in (KATZ_OK, KATZ_ENOCONV):
        _check(rc)
    return rc


def katz_sparse_katz(idx, q, s: int, T: int, opts: Optional[katz_query_opts], ids, corr=None, stats=None,
                     stream=None) -> int:
    qa = np.ascontiguousarray(q, np.int32)
    st = (katz_query_stats * len(qa))() if stats is None else stats
    rc = _lib.katz_sparse_katz(idx, _pi32(qa), len(qa), int(s), int(T),
                               ctypes.byref(opts) if opts is not None else None, _ptr(ids), _ptr(corr), st,
                               ctypes.c_void_p(stream) if stream else None)
    if rc not in (KATZ_OK, KATZ_ENOCONV):
        _check(rc)
    return rc


def katz_index_save(idx, path: str) -> None:
    _check(_lib.katz_index_save(idx, os.fsencode(path)))


def katz_index_load(path: str, device: int = 0) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(_lib.katz_index_load(os.fsencode(path), int(device), ctypes.byref(h)))
    return h


def katz_index_free(idx) -> None:
    _lib.katz_index_free(idx)


def katz_index_info(idx) -> katz_index_info_t:
    info = katz_index_info_t()
    _check(_lib.katz_index_info(idx, ctypes.byref(info)))
    return info


def katz_index_partition(idx, n: int, nblocks: int):
    perm = np.empty(n, np.int32)
    bp = np.empty(nblocks + 1, np.int32)
    _check(_lib.katz_index_partition(idx, _pi32(perm), _pi32(bp)))
    return perm, bp


def katz_index_lowrank(idx, n2: int, rank: int):
    U = np.empty(max(1, n2 * rank), np.float64)
    s = np.empty(max(1, rank), np.float64)
    _check(_lib.katz_index_lowrank(idx, _pdbl(U), _pdbl(s)))
    return U[: n2 * rank].reshape(n2, rank), s[:rank]


def katz_profile_enable(on: bool) -> int:
    return _lib.katz_profile_enable(1 if on else 0)


def katz_profile_reset() -> None:
    _lib.katz_profile_reset()


def katz_profile_read() -> list:
    buf = (katz_kernel_stat * 32)()
    m = _lib.katz_profile_read(buf, 32)
    return [{"name": b.name.decode(), "launches": b.launches, "total_ms": b.total_ms, "alg_bytes": b.alg_bytes}
            for b in buf[:m]]


def katz_last_error() -> str:
    return (_lib.katz_last_error() or b"").decode()


def stats_dicts(st) -> list:
    return [{"status": s.status, "iters": s.iters, "sweeps": s.sweeps, "path": s.path,
             "rel_residual": s.rel_residual, "err_bound": s.err_bound} for s in st]


# --------------------------------------------------------------- wrapper
class KatzIndex:
    """Owns one katz_index handle."""

    def __init__(self, n: int, row_ptr, col, val=None, *, beta: float = 0.0, beta_frac: float = 0.5,
                 rank: int = 32, max_block: int = 64, labels=None, l_kind: int = KATZ_L_AUTO,
                 precision: int = KATZ_PREC_FP64, seed: int = 12345, device: int = 0,
                 lanczos_steps: int = 0, order: int = KATZ_ORDER_AUTO, u_precision: int = 0):
        o = katz_build_opts_default()
        o.beta, o.beta_frac, o.rank, o.max_block = beta, beta_frac, rank, max_block
        self._labels = None if labels is None else np.ascontiguousarray(labels, np.int32)
        o.labels = _pi32(self._labels)
        o.l_kind, o.precision, o.seed, o.device, o.lanczos_steps = l_kind, precision, seed, device, lanczos_steps
        o.order = order
        o.u_precision = u_precision
        self.n = int(n)
        self.h = katz_index_build(n, row_ptr, col, val, o)
        self.info = katz_index_info(self.h)

    @classmethod
    def from_graph(cls, g, **kw):
        return cls(g.n, g.row_ptr, g.col, **kw)

    def rebuild(self, *, beta: float = 0.0, beta_frac: float = 0.5, rank: int = 32, l_kind: int = KATZ_L_AUTO,
                precision: int = KATZ_PREC_FP64, seed: int = 12345, device: int = 0, lanczos_steps: int = 0,
                u_precision: int = 0) -> "KatzIndex":
        """katz_index_rebuild: this graph and partition, new beta-dependent
        factors for these options."""
        o = katz_build_opts_default()
        o.beta, o.beta_frac, o.rank = beta, beta_frac, rank
        o.l_kind, o.precision, o.seed, o.device, o.lanczos_steps = l_kind, precision, seed, device, lanczos_steps
        o.u_precision = u_precision
        h = ctypes.c_void_p()
        _check(_lib.katz_index_rebuild(self.h, ctypes.byref(o), ctypes.byref(h)))
        new = KatzIndex.__new__(KatzIndex)
        new._labels = None
        new.h = h
        new.info = katz_index_info(h)
        new.n = int(new.info.n)
        return new

    @classmethod
    def load(cls, path: str, device: int = 0) -> "KatzIndex":
        """An index written by save(), on `device` (< 0: host only)."""
        self = cls.__new__(cls)
        self._labels = None
        self.h = katz_index_load(path, device)
        self.info = katz_index_info(self.h)
        self.n = int(self.info.n)
        return self

    def save(self, path: str) -> None:
        katz_index_save(self.h, path)

    def close(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.katz_index_free(h)
        self.h = None

    def __del__(self):
        self.close()

    def partition(self):
        return katz_index_partition(self.h, self.n, self.info.nblocks)

    def lowrank(self):
        return katz_index_lowrank(self.h, self.info.n2, self.info.rank)

    @staticmethod
    def _opts(tol, method, max_iter, max_sweeps, check_every, force_fallback=0):
        o = katz_query_opts_default()
        o.force_fallback = int(force_fallback)
        o.rel_tol = tol
        o.method = method
        if max_iter:
            o.max_iter = max_iter
        if max_sweeps:
            o.max_sweeps = max_sweeps
        if check_every:
            o.check_every = check_every
        return o

    def query(self, q: Sequence[int], out=None, *, tol: float = 1e-6, method: int = KATZ_METHOD_LRC,
              max_iter: int = 0, max_sweeps: int = 0, check_every: int = 0, stream=None,
              force_fallback: bool = False):
        """Katz vectors of the queries: (scores [nq, n] FP64, stats list).
        `out` may be a CUDA torch tensor (device output) or None (numpy)."""
        q = np.atleast_1d(np.asarray(q, np.int32))
        if out is None:
            out = np.empty((len(q), self.n), np.float64)
        if stream is None and hasattr(out, "data_ptr") and getattr(out, "is_cuda", False):
            import torch
            stream = torch.cuda.current_stream(out.device).cuda_stream
        st = (katz_query_stats * len(q))()
        katz_query(self.h, q, self._opts(tol, method, max_iter, max_sweeps, check_every, force_fallback), out,
                   st, stream)
        return out, stats_dicts(st)

    def query_noalloc(self, q: Sequence[int], out=None, *, tol: float = 1e-6, method: int = KATZ_METHOD_LRC,
                      max_iter: int = 0, max_sweeps: int = 0, check_every: int = 0, stream=None):
        """As query(), through katz_query_noalloc (static device scratch, no
        allocation in the library)."""
        q = np.atleast_1d(np.asarray(q, np.int32))
        if out is None:
            out = np.empty((len(q), self.n), np.float64)
        if stream is None and hasattr(out, "data_ptr") and getattr(out, "is_cuda", False):
            import torch
            stream = torch.cuda.current_stream(out.device).cuda_stream
        st = (katz_query_stats * len(q))()
        katz_query_noalloc(self.h, q, self._opts(tol, method, max_iter, max_sweeps, check_every), out, st, stream)
        return out, stats_dicts(st)

    def pair_scores(self, src: Sequence[int], dst: Sequence[int], out=None, *, tol: float = 1e-6,
                    method: int = KATZ_METHOD_LRC, max_iter: int = 0, max_sweeps: int = 0, stream=None):
        """K[dst[i], src[i]] per pair: (scores [npairs] FP64, stats list)."""
        s = np.atleast_1d(np.asarray(src, np.int32))
        if out is None:
            out = np.empty(len(s), np.float64)
        st = (katz_query_stats * len(s))()
        katz_pair_scores(self.h, s, dst, self._opts(tol, method, max_iter, max_sweeps, 0), out, st, stream)
        return out, stats_dicts(st)

    def sparse_katz(self, q: Sequence[int], s: int, T: int, *, tol: float = 1e-6, method: int = KATZ_METHOD_LRC,
                    max_iter: int = 0, max_sweeps: int = 0, stream=None):
        """Sparse-Katz re-ranked links: (ids [nq, s], correlations [nq, s], stats)."""
        q = np.atleast_1d(np.asarray(q, np.int32))
        ids = np.empty((len(q), s), np.int32)
        corr = np.empty((len(q), s), np.float64)
        st = (katz_query_stats * len(q))()
        katz_sparse_katz(self.h, q, s, T, self._opts(tol, method, max_iter, max_sweeps, 0), ids, corr, st, stream)
        return ids, corr, stats_dicts(st)

    def topk(self, q: Sequence[int], k: int, ids=None, scores=None, *, tol: float = 1e-6,
             method: int = KATZ_METHOD_LRC, max_iter: int = 0, max_sweeps: int = 0, check_every: int = 0,
             stream=None):
        q = np.atleast_1d(np.asarray(q, np.int32))
        if ids is None:
            ids = np.empty((len(q), k), np.int32)
            scores = np.empty((len(q), k), np.float64) if scores is None else scores
        if stream is None and hasattr(ids, "data_ptr") and getattr(ids, "is_cuda", False):
            import torch
            stream = torch.cuda.current_stream(ids.device).cuda_stream
        st = (katz_query_stats * len(q))()
        katz_topk_links(self.h, q, k, self._opts(tol, method, max_iter, max_sweeps, check_every), ids, scores,
                        st, stream)
        return ids, scores, stats_dicts(st)


# --------------------------------------------------------------- serving
def katz_server_opts_default() -> katz_server_opts:
    o = katz_server_opts()
    _lib.katz_server_opts_default(ctypes.byref(o))
    return o


class KatzServer:
    """Continuous-batching top-K server over one KatzIndex (katz_server_*)."""

    def __init__(self, index: KatzIndex, *, workers: int = 0, max_batch: int = 64, hbm_fraction: float = 0.8,
                 k: int = 100, tol: float = 1e-6, method: int = KATZ_METHOD_LRC):
        o = katz_server_opts_default()
        o.workers, o.max_batch, o.hbm_fraction, o.k = workers, max_batch, hbm_fraction, k
        o.query.rel_tol = tol
        o.query.method = method
        self.index = index          # keeps the index alive
        self.k = k
        self.h = ctypes.c_void_p()
        _check(_lib.katz_server_create(index.h, ctypes.byref(o), ctypes.byref(self.h)))
        self._nq = {}

    def submit(self, q) -> int:
        qa = np.ascontiguousarray(np.atleast_1d(q), np.int32)
        t = ctypes.c_int64()
        _check(_lib.katz_server_submit(self.h, _pi32(qa), len(qa), ctypes.byref(t)))
        self._nq[t.value] = len(qa)
        return t.value

    def poll(self, ticket: int, timeout_us: int = -1):
        """(ids [nq, k], scores [nq, k], stats, latency_ms) or None if not done."""
        nq = self._nq[ticket]
        ids = np.empty((nq, self.k), np.int32)
        sc = np.empty((nq, self.k), np.float64)
        st = (katz_query_stats * nq)()
        lat = ctypes.c_double()
        rc = _lib.katz_server_poll(self.h, ticket, _pi32(ids), _pdbl(sc), st, ctypes.byref(lat), int(timeout_us))
        if rc == KATZ_EBUSY:
            return None
        if rc not in (KATZ_OK, KATZ_ENOCONV):
            _check(rc)
        del self._nq[ticket]
        return ids, sc, stats_dicts(st), lat.value

    def info(self) -> dict:
        i = katz_server_info_t()
        _check(_lib.katz_server_info(self.h, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in katz_server_info_t._fields_}

    def close(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.katz_server_destroy(h)
        self.h = None

    def __del__(self):
        self.close()
