"""Plain, slow, obviously-correct FP64 reference for Katz queries.

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU-baseline leg; never by the library's product path.

Paper: Coskun, Baggag, Koyuturk, "Fast Computation of Katz Index for Efficient
Processing of Link Prediction Queries" (arXiv:1912.06525).  Notation here:
``beta`` is the paper's damping factor (alpha in Section 3.1), ``A`` the
adjacency matrix (G in the paper), ``c = beta * lambda_max(A)``.

What is computed (all FP64):

* the Katz vector of query q, the q-th column of K = sum_{l>=1} beta^l A^l
  (Section 3.1, eq. KatzPath read with walks, eq. KatzMatrix);
* as the solution of (I - beta A) k = beta A e_q (eq. LinearSystem), by a
  dense Cholesky solve (small graphs) and by the truncated Neumann series
  sum_{l>=1} (beta A)^l e_q with a rigorous tail bound (all sizes);
* the top-K link-prediction list: candidates are the nodes that are neither q
  nor a neighbour of q, ordered by (score descending, node id ascending)
  (Section 3.3, the sort step of Algorithm 3);
* exact walk counts by brute-force enumeration (tiny graphs), which pin the
  walk-sum definition itself (eq. KatzPath).
"""
from __future__ import annotations

import math
from typing import Iterable, Optional, Sequence

import numpy as np
import scipy.linalg
import scipy.sparse
import scipy.sparse.linalg


class OracleError(ValueError):
    pass


# ----------------------------------------------------------------- input
def validate_csr(n: int, row_ptr, col, val=None) -> None:
    """Checks that (row_ptr, col[, val]) is the adjacency matrix of an
    undirected graph: square, int32 indices in range, strictly increasing
    column indices per row, zero diagonal, exactly symmetric, values >= 0.
    Section 3.1 takes an undirected network, so A = A^T."""
    row_ptr = np.asarray(row_ptr)
    col = np.asarray(col)
    if n < 0 or row_ptr.shape != (n + 1,):
        raise OracleError("row_ptr must have n+1 entries")
    if row_ptr[0] != 0 or np.any(np.diff(row_ptr) < 0) or row_ptr[-1] != col.shape[0]:
        raise OracleError("row_ptr must be non-decreasing from 0 to nnz")
    if col.size and (col.min() < 0 or col.max() >= n):
        raise OracleError("column index out of range")
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    if col.size:
        same_row = rows[1:] == rows[:-1]
        if np.any(same_row & (col[1:] <= col[:-1])):
            raise OracleError("columns must be strictly increasing within a row")
    if np.any(rows == col):
        raise OracleError("nonzero diagonal (self loop)")
    v = np.ones(col.shape[0]) if val is None else np.asarray(val, np.float64)
    if np.any(v < 0) or not np.all(np.isfinite(v)):
        raise OracleError("values must be finite and >= 0")
    A = scipy.sparse.csr_matrix((v, col, row_ptr), shape=(n, n))
    D = (A - A.T).tocsr()
    D.eliminate_zeros()
    if D.nnz:
        raise OracleError("matrix is not symmetric")


def csr_matrix(n: int, row_ptr, col, val=None) -> scipy.sparse.csr_matrix:
    v = np.ones(len(col)) if val is None else np.asarray(val, np.float64)
    return scipy.sparse.csr_matrix((v, np.asarray(col), np.asarray(row_ptr)), shape=(n, n))


def lambda_max(A: scipy.sparse.csr_matrix) -> float:
    """Largest eigenvalue of the symmetric nonnegative A, which equals its
    spectral norm ||A||_2 (Section 3.1 requires beta < 1/||A||_2).  Dense
    symmetric eigensolver for n <= 4000, else ARPACK to relative 1e-12."""
    n = A.shape[0]
    if A.nnz == 0:
        return 0.0
    if n <= 4000:
        return float(np.linalg.eigvalsh(A.toarray())[-1])
    vals = scipy.sparse.linalg.eigsh(A.astype(np.float64), k=1, which="LA", tol=1e-12,
                                     return_eigenvectors=False, v0=np.ones(n))
    return float(vals[-1])


def _queries(qs) -> np.ndarray:
    q = np.atleast_1d(np.asarray(qs, dtype=np.int64))
    return q


# ------------------------------------------------------------------ solve
def katz_rhs(A: scipy.sparse.csr_matrix, beta: float, qs) -> np.ndarray:
    """Right-hand side beta * A e_q of eq. LinearSystem, one column per query
    (dense n x B)."""
    q = _queries(qs)
    return beta * A[:, q].toarray()


def katz_direct(A: scipy.sparse.csr_matrix, beta: float, qs) -> np.ndarray:
    """Dense solve of (I - beta A) k = beta A e_q (eq. LinearSystem) with a
    Cholesky factorization; M = I - beta A is SPD when beta*lambda_max < 1.
    For n <= 5000 only."""
    n = A.shape[0]
    if n > 5000:
        raise OracleError("dense solve limited to n <= 5000")
    M = np.eye(n) - beta * A.toarray()
    cf = scipy.linalg.cho_factor(M, lower=True)
    return scipy.linalg.cho_solve(cf, katz_rhs(A, beta, qs))


def katz_series(A: scipy.sparse.csr_matrix, beta: float, qs, c: float,
                tol: float = 1e-13, max_terms: int = 100000):
    """Neumann series of eq. KatzMatrix applied to e_q:
    k = sum_{l>=1} (beta A)^l e_q.  Terms are added until the bound on the
    remaining tail, ||v_L|| * c / (1 - c) (because ||beta A||_2 = c), falls
    below tol * ||k||.  All terms are nonnegative for nonnegative A, so the sum
    has no cancellation.  Returns (k, terms, tail_bound) with per-column
    arrays."""
    if not (0.0 <= c < 1.0):
        raise OracleError("series diverges: beta * lambda_max must be < 1")
    v = katz_rhs(A, beta, qs)          # (beta A)^1 e_q
    s = v.copy()
    B = v.shape[1]
    terms = np.ones(B, np.int64)
    done = np.zeros(B, bool)
    tail = np.zeros(B)
    ratio = c / (1.0 - c) if c > 0 else 0.0
    for _ in range(max_terms):
        vn = np.linalg.norm(v, axis=0)
        sn = np.linalg.norm(s, axis=0)
        tb = vn * ratio
        newly = (~done) & (tb <= tol * sn)
        tail[newly] = tb[newly]
        done |= newly
        if done.all():
            break
        act = ~done
        v[:, act] = beta * (A @ v[:, act])
        s[:, act] += v[:, act]
        terms[act] += 1
    else:
        raise OracleError("series did not reach the requested tail bound")
    return s, terms, tail


def katz_residual(A: scipy.sparse.csr_matrix, beta: float, qs, k: np.ndarray) -> np.ndarray:
    """Relative residual ||b - (I - beta A) k||_2 / ||b||_2 per column, with
    b = beta A e_q; 0 where b = 0 and k = 0."""
    b = katz_rhs(A, beta, qs)
    k = np.asarray(k, np.float64).reshape(b.shape)
    r = b - (k - beta * (A @ k))
    bn = np.linalg.norm(b, axis=0)
    rn = np.linalg.norm(r, axis=0)
    with np.errstate(invalid="ignore", divide="ignore"):
        out = np.where(bn > 0, rn / np.where(bn > 0, bn, 1.0), rn)
    return out


def katz_oracle(n: int, row_ptr, col, qs, beta: Optional[float] = None,
                c: Optional[float] = None, val=None, lam: Optional[float] = None,
                tol: float = 1e-13, direct: Optional[bool] = None, validate: bool = True) -> dict:
    """Full oracle: validate, lambda_max, series (always), dense direct solve
    (n <= 5000), cross-check of the two, and the oracle's own residual.
    Exactly one of beta / c (= beta * lambda_max) is given.  Returns a dict
    with 'k' (n x B, original node order; entry q holds K_qq), 'beta', 'c',
    'lambda_max', 'terms', 'tail', 'residual' and, when run, 'k_direct'."""
    if validate:
        validate_csr(n, row_ptr, col, val)
    A = csr_matrix(n, row_ptr, col, val)
    lam = lambda_max(A) if lam is None else float(lam)
    if (beta is None) == (c is None):
        raise OracleError("give exactly one of beta and c")
    if beta is None:
        if lam <= 0:
            raise OracleError("graph has no edges: beta undefined from c")
        beta = c / lam
    cc = beta * lam
    if beta <= 0 or cc >= 1.0:
        raise OracleError("convergence needs 0 < beta < 1/lambda_max (got c = %r)" % cc)
    k, terms, tail = katz_series(A, beta, qs, cc, tol=tol)
    out = {"k": k, "beta": beta, "c": cc, "lambda_max": lam, "terms": terms, "tail": tail}
    if direct is None:
        direct = n <= 5000
    if direct:
        kd = katz_direct(A, beta, qs)
        out["k_direct"] = kd
        den = np.maximum(np.linalg.norm(kd, axis=0), np.finfo(float).tiny)
        rel = np.linalg.norm(kd - k, axis=0) / den
        out["cross_rel"] = rel
        if np.any(rel > 1e-11):
            raise OracleError("direct solve and series disagree: %r" % rel)
    out["residual"] = katz_residual(A, beta, qs, k)
    return out


# ------------------------------------------------------------------ top-K
def topk_links(n: int, row_ptr, col, scores: np.ndarray, q: int, K: int):
    """Top-K predicted links for query q (Section 3.3; Algorithm 3 sorts k_q in
    descending order): candidates are all nodes except q and its neighbours;
    full sort by (score descending, id ascending); pad with (-1, NaN).
    Returns (ids[K], scores[K], ordered candidate ids, their scores)."""
    scores = np.asarray(scores, np.float64).reshape(n)
    mask = np.ones(n, bool)
    mask[q] = False
    mask[np.asarray(col[row_ptr[q]:row_ptr[q + 1]])] = False
    cand = np.nonzero(mask)[0]
    order = np.lexsort((cand, -scores[cand]))
    sorted_ids = cand[order]
    sorted_sc = scores[sorted_ids]
    ids = np.full(K, -1, np.int64)
    sc = np.full(K, np.nan)
    m = min(K, sorted_ids.size)
    ids[:m] = sorted_ids[:m]
    sc[:m] = sorted_sc[:m]
    return ids, sc, sorted_ids, sorted_sc


def tie_classes(sorted_scores: np.ndarray, delta: float) -> np.ndarray:
    """Class label per position of a descending score list: single linkage on
    consecutive gaps <= delta (scores closer than the solver tolerance cannot
    be ordered reliably)."""
    s = np.asarray(sorted_scores, np.float64)
    if s.size == 0:
        return np.zeros(0, np.int64)
    brk = np.concatenate([[0], (s[:-1] - s[1:]) > delta]).astype(np.int64)
    return np.cumsum(brk)


def topk_accept(build_ids: Sequence[int], sorted_ids: np.ndarray, sorted_scores: np.ndarray,
                K: int, delta: float) -> tuple:
    """Acceptance of a build's top-K list against the oracle's full ordering
    under the tie rule: position-for-position equal, except that inside a tie
    class any order is accepted and the class straddling position K may
    contribute any subset of the right size.  Returns (ok, message,
    number of non-trivial classes within the first K)."""
    b = np.asarray(build_ids, np.int64)
    m = min(K, sorted_ids.size)
    if np.any(b[m:] != -1):
        return False, "padding expected after %d candidates" % m, 0
    cls = tie_classes(sorted_scores, delta)
    nontriv = 0
    pos = 0
    while pos < m:
        c = cls[pos]
        end = pos
        while end < cls.size and cls[end] == c:
            end += 1
        members = set(int(x) for x in sorted_ids[pos:end])
        if end - pos > 1:
            nontriv += 1
        hi = min(end, m)
        got = [int(x) for x in b[pos:hi]]
        if len(set(got)) != len(got) or not set(got) <= members:
            return False, "positions %d..%d: %r not within tie class" % (pos, hi, got[:8]), nontriv
        pos = end
    return True, "ok", nontriv


# ------------------------------------------------------------- brute force
def sparse_katz(n: int, row_ptr, col, q: int, s: int, T: int, beta: float, lam: Optional[float] = None) -> dict:
    """Sparse-Katz link prediction (Section 3.3, Algorithm 3), from the text:
    k_q; its candidates (all nodes but q and its neighbours) sorted by score
    (ties by id); the top-s list and the T highest-ranked candidates as the
    "modular" nodes; K_T = [k_t] for those nodes (n x T); for each listed
    candidate j, rho_j = Pearson correlation of rows q and j of K_T (NaN when
    a row is constant or T < 2); the list re-ordered by rho descending,
    undefined correlations last, ties in the Katz order.
    Returns ids (re-ranked), rho (in that order), the Katz-ordered list, its
    correlations and K_T."""
    kq = katz_oracle(n, row_ptr, col, [q], beta=beta, lam=lam, validate=False)["k"][:, 0]
    _, _, sid, _ = topk_links(n, row_ptr, col, kq, q, max(s, T))
    cand = sid[:s]
    mods = sid[:T]
    KT = None
    if len(mods) >= 2:
        KT = katz_oracle(n, row_ptr, col, mods, beta=beta, lam=lam, validate=False)["k"]
        order, rho = correlation_rerank(KT[q, :], KT[cand, :])
    else:
        order, rho = list(range(len(cand))), np.full(len(cand), np.nan)
    return {"ids": cand[order], "rho": rho[order], "katz_order": cand, "katz_rho": rho, "KT": KT,
            "modular": mods}


def pearson(x, y) -> float:
    """Pearson correlation of two equal-length vectors, written out:
    sum (x - mean x)(y - mean y) / sqrt(sum (x - mean x)^2 sum (y - mean y)^2);
    NaN when either vector is constant."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    dx = x - x.sum() / x.size
    dy = y - y.sum() / y.size
    sxx = float((dx * dx).sum())
    syy = float((dy * dy).sum())
    if not (sxx > 0 and syy > 0):
        return float("nan")
    return float((dx * dy).sum()) / math.sqrt(sxx * syy)


def correlation_rerank(xq, rows):
    """The last step of Algorithm 3: rho_j = Pearson correlation of the query's
    row xq of K_T with candidate j's row rows[j]; returns (order, rho) where
    order lists the candidates (given in Katz order) by rho descending,
    undefined correlations last, ties in the Katz order."""
    rows = np.atleast_2d(np.asarray(rows, np.float64))
    rho = np.array([pearson(xq, rows[j]) for j in range(rows.shape[0])]) if rows.size else np.zeros(0)
    key = [(0 if np.isfinite(r) else 1, -r if np.isfinite(r) else 0.0, j) for j, r in enumerate(rho)]
    return [j for _, _, j in sorted(key)], rho


def walk_counts(n: int, row_ptr, col, q: int, max_len: int) -> list:
    """Exact number of walks of each length l = 1..max_len from q to every
    node, by explicit depth-first enumeration of the walks (tiny graphs only).
    counts[l][v] is a Python int.  Pins eq. KatzPath (read with walks)."""
    adj = [list(map(int, col[row_ptr[u]:row_ptr[u + 1]])) for u in range(n)]
    counts = [[0] * n for _ in range(max_len + 1)]

    def dfs(u: int, depth: int) -> None:
        if depth:
            counts[depth][u] += 1
        if depth == max_len:
            return
        for w in adj[u]:
            dfs(w, depth + 1)

    dfs(int(q), 0)
    return counts
