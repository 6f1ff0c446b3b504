"""Pins for the CPU oracle: each check compares it with something other than
itself -- brute-force walk enumeration (plain and edge-weighted), closed
forms derived by hand for complete, star, weighted star and cycle graphs,
symmetry, reachability, relabelling and the convergence condition
(Section 3.1).  CPU only."""
import math

import numpy as np
import pytest

import katz_inputs as ki
import oracle
from oracle import reference as ko


def _graph(n, edges):
    g = ki.from_edges(n, edges)
    return g.n, g.row_ptr, g.col


def complete(n):
    return _graph(n, [(i, j) for i in range(n) for j in range(i + 1, n)])


def star(m):
    return _graph(m + 1, [(0, i) for i in range(1, m + 1)])


def cycle(n):
    return _graph(n, [(i, (i + 1) % n) for i in range(n)])


def path(n):
    return _graph(n, [(i, i + 1) for i in range(n - 1)])


# The series stops when its tail bound is below 1e-13 of ||k||; allow that
# plus rounding.  The dense solve is accurate to a few ulps times kappa(M).
SER = 3e-13


def both(n, rp, col, q, beta):
    """Series and dense solve of the oracle, for one query."""
    out = oracle.katz_oracle(n, rp, col, [q], beta=beta, direct=True)
    return out["k"][:, 0], out["k_direct"][:, 0], out


# ----------------------------------------------------------------- P2
@pytest.mark.parametrize("n,beta", [(6, 0.1), (7, 0.15), (12, 0.02)])
def test_complete_graph_closed_form(n, beta):
    # A = J - I; Sherman-Morrison on (1+beta) I - beta J gives
    # K_pq = beta / ((1+beta)(1-(n-1)beta)), K_qq = (n-1) beta^2 / (same).
    g = complete(n)
    den = (1 + beta) * (1 - (n - 1) * beta)
    for q in (0, n - 1):
        ks, kd, _ = both(*g, q, beta)
        exp = np.full(n, beta / den)
        exp[q] = (n - 1) * beta ** 2 / den
        np.testing.assert_allclose(ks, exp, rtol=SER, atol=0)
        np.testing.assert_allclose(kd, exp, rtol=1e-13, atol=0)


@pytest.mark.parametrize("m,c", [(5, 0.5), (9, 0.9), (3, 0.1)])
def test_star_closed_form(m, c):
    # lambda_max(star with m leaves) = sqrt(m); d = 1 - m beta^2.
    beta = c / math.sqrt(m)
    d = 1 - m * beta ** 2
    g = star(m)
    ks, kd, out = both(*g, 0, beta)           # centre query
    exp = np.full(m + 1, beta / d)
    exp[0] = m * beta ** 2 / d
    np.testing.assert_allclose(ks, exp, rtol=SER)
    np.testing.assert_allclose(kd, exp, rtol=1e-13)
    assert abs(out["lambda_max"] - math.sqrt(m)) < 1e-12
    ks, kd, _ = both(*g, 2, beta)             # leaf query
    exp = np.full(m + 1, beta ** 2 / d)       # other leaves and the leaf itself
    exp[0] = beta / d
    np.testing.assert_allclose(ks, exp, rtol=SER)
    np.testing.assert_allclose(kd, exp, rtol=1e-13)


@pytest.mark.parametrize("n,beta", [(9, 0.2), (8, 0.45), (5, 0.05)])
def test_cycle_closed_form(n, beta):
    # Periodic Green's function of x_j - beta (x_{j-1} + x_{j+1}) = delta_j0:
    # s = sqrt(1 - 4 beta^2), t = (1 - s) / (2 beta),
    # x_delta = (t^delta + t^(n-delta)) / (s (1 - t^n)); K = x - [delta = 0].
    s = math.sqrt(1 - 4 * beta ** 2)
    t = (1 - s) / (2 * beta)
    g = cycle(n)
    q = 3 % n
    ks, kd, _ = both(*g, q, beta)
    exp = np.empty(n)
    for v in range(n):
        dl = (v - q) % n
        exp[v] = (t ** dl + t ** (n - dl)) / (s * (1 - t ** n)) - (1.0 if dl == 0 else 0.0)
    # the series error bound is norm-wise (tail <= 1e-13 ||k||)
    np.testing.assert_allclose(ks, exp, rtol=1e-12, atol=SER * np.linalg.norm(exp))
    np.testing.assert_allclose(kd, exp, rtol=1e-12)


# ----------------------------------------------------------------- P1
def test_walk_enumeration_path3_by_hand():
    # Path 0-1-2 from node 0: odd l reaches node 1 by 2^((l-1)/2) walks, even
    # l reaches nodes 0 and 2 by 2^(l/2-1) walks each.
    n, rp, col = path(3)
    cnt = oracle.walk_counts(n, rp, col, 0, 9)
    for l in range(1, 10):
        if l % 2:
            assert cnt[l] == [0, 2 ** ((l - 1) // 2), 0]
        else:
            assert cnt[l] == [2 ** (l // 2 - 1), 0, 2 ** (l // 2 - 1)]


SMALL = {
    "tree": (7, [(0, 1), (0, 2), (1, 3), (1, 4), (2, 5), (5, 6)]),
    "tri_tail": (5, [(0, 1), (1, 2), (0, 2), (2, 3), (3, 4)]),
    "c5_chord": (5, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 0), (1, 3)]),
}


@pytest.mark.parametrize("name", sorted(SMALL))
def test_walk_sum_matches_solver(name):
    # eq. KatzPath summed over explicitly enumerated walks, plus the rigorous
    # entrywise tail bound sum_{l>L} c^l = c^(L+1)/(1-c), must contain both the
    # series and the dense solve (and lie below them: every term is >= 0).
    n, edges = SMALL[name]
    n, rp, col = _graph(n, edges)
    L = 10
    A = ko.csr_matrix(n, rp, col)
    lam = ko.lambda_max(A)
    for c in (0.05, 0.6):
        beta = c / lam
        for q in range(n):
            cnt = oracle.walk_counts(n, rp, col, q, L)
            trunc = np.array([sum(beta ** l * cnt[l][v] for l in range(1, L + 1)) for v in range(n)])
            bound = c ** (L + 1) / (1 - c)
            ks, kd, _ = both(n, rp, col, q, beta)
            for k in (ks, kd):
                assert np.all(k >= trunc - 1e-15)
                assert np.all(k - trunc <= bound + 1e-15)
            if c == 0.05:
                np.testing.assert_allclose(ks, trunc, rtol=0, atol=1e-14)


def test_walk_counts_golden():
    # Stored walk counts (tests/golden/walks_tri_tail.json, written by
    # tests/golden/make_golden.py with oracle.walk_counts) re-derived here.
    import json
    import os
    p = os.path.join(os.path.dirname(__file__), "golden", "walks_tri_tail.json")
    with open(p) as f:
        gold = json.load(f)
    n, rp, col = _graph(gold["n"], [tuple(e) for e in gold["edges"]])
    got = oracle.walk_counts(n, rp, col, gold["q"], gold["max_len"])
    assert got == gold["counts"]
    # the same counts are the entries of A^l e_q (integer matrix powers)
    A = np.zeros((n, n), dtype=object)
    for u in range(n):
        for v in col[rp[u]:rp[u + 1]]:
            A[u, v] = 1
    x = np.zeros(n, dtype=object)
    x[gold["q"]] = 1
    for l in range(1, gold["max_len"] + 1):
        x = A.dot(x)
        assert list(x) == gold["counts"][l]


# ------------------------------------------------ weighted adjacency (P1, P2)
def weighted_star(w):
    """Star whose centre 0 joins leaf i (1..m) with weight w[i-1]; the CSR
    values in entry order (row 0: leaves 1..m; row i: the centre)."""
    m = len(w)
    n, rp, col = star(m)
    val = np.concatenate([np.asarray(w, np.float64), np.asarray(w, np.float64)])
    return n, rp, col, val


def _weighted_star_expected(w, c):
    # A e_0 = w on the leaves and lambda_max = ||w||, so beta^2 sum w_i^2 = c^2.
    # Centre query: k_i = beta w_i (1 + k_0), k_0 = beta sum w_i k_i
    #   => k_0 = c^2 / (1 - c^2), k_i = beta w_i / (1 - c^2).
    # Leaf query j: k_i = beta w_i k_0, k_0 = beta w_j + beta sum w_i k_i
    #   => k_0 = beta w_j / (1 - c^2), k_i = beta^2 w_i w_j / (1 - c^2).
    w = np.asarray(w, np.float64)
    beta = c / np.linalg.norm(w)
    d = 1 - c * c
    centre = np.concatenate([[c * c / d], beta * w / d])
    j = 2
    leaf = np.concatenate([[beta * w[j - 1] / d], beta * beta * w * w[j - 1] / d])
    return beta, centre, j, leaf


@pytest.mark.parametrize("w,c", [([0.5, 1.7, 0.3, 2.0, 1.1], 0.5),
                                 ([3.0, 0.25, 0.75], 0.9),
                                 ([1.0, 1.0, 1.0, 1.0], 0.3)])
def test_weighted_star_closed_form(w, c):
    n, rp, col, val = weighted_star(w)
    beta, centre, j, leaf = _weighted_star_expected(w, c)
    out = oracle.katz_oracle(n, rp, col, [0, j], c=c, val=val, direct=True)
    assert out["lambda_max"] == pytest.approx(np.linalg.norm(w), rel=1e-13)
    assert out["beta"] == pytest.approx(beta, rel=1e-13)
    for k in (out["k"], out["k_direct"]):
        np.testing.assert_allclose(k[:, 0], centre, rtol=1e-12)
        np.testing.assert_allclose(k[:, 1], leaf, rtol=1e-12)


def _weighted_walk_sums(n, rp, col, val, q, L):
    """sums[l][v] = sum over the walks q -> v with l edges of the product of
    their edge weights, by depth-first enumeration of every walk (tiny graphs
    only; no matrix products)."""
    sums = [[0.0] * n for _ in range(L + 1)]

    def walk(u, l, prod):
        for e in range(rp[u], rp[u + 1]):
            v, p = int(col[e]), prod * float(val[e])
            sums[l + 1][v] += p
            if l + 1 < L:
                walk(v, l + 1, p)

    walk(q, 0, 1.0)
    return sums


@pytest.mark.parametrize("name", sorted(SMALL))
def test_weighted_walk_sum_matches_solver(name):
    # eq. KatzPath with each walk counted by the product of its edge weights.
    # Entrywise |(beta A)^l e_q| <= ||beta A||^l = c^l, so the terms beyond L
    # add at most c^(L+1) / (1 - c) to any entry (and nothing negative).
    n, edges = SMALL[name]
    g = ki.from_edges(n, edges)
    val = ki.edge_weights(g, seed=11)
    L = 9
    for c in (0.05, 0.5):
        for q in range(n):
            out = oracle.katz_oracle(g.n, g.row_ptr, g.col, [q], c=c, val=val, direct=True)
            beta = out["beta"]
            sums = _weighted_walk_sums(g.n, g.row_ptr, g.col, val, q, L)
            trunc = np.array([sum(beta ** l * sums[l][v] for l in range(1, L + 1)) for v in range(n)])
            bound = c ** (L + 1) / (1 - c)
            for k in (out["k"][:, 0], out["k_direct"][:, 0]):
                assert np.all(k >= trunc - 1e-14)
                assert np.all(k - trunc <= bound + 1e-14)


# ----------------------------------------------------------- P3, P4, P9
def _small_sbm():
    return ki.sbm([40, 30, 50], [0.2, 0.25, 0.15], 0.02, seed=77)


def test_symmetry_kpq_equals_kqp():
    g = _small_sbm()
    qs = ki.sample_queries(g, 6, 5)
    out = oracle.katz_oracle(g.n, g.row_ptr, g.col, qs, c=0.7)
    K = out["k"]
    for i, p in enumerate(qs):
        for j, q in enumerate(qs):
            assert abs(K[q, i] - K[p, j]) <= 1e-13 * max(abs(K[q, i]), 1e-300)


def test_reachability_and_isolated_query():
    # disjoint union: a 5-cycle (0..4), a triangle (5..7) and isolated node 8
    n, rp, col = _graph(9, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 0), (5, 6), (6, 7), (5, 7)])
    out = oracle.katz_oracle(n, rp, col, [1, 6, 8], c=0.8)
    k = out["k"]
    assert np.all(k[0:5, 0] > 0) and np.all(k[5:, 0] == 0)
    assert np.all(k[5:8, 1] > 0) and np.all(k[[0, 1, 2, 3, 4, 8], 1] == 0)
    assert np.all(k[:, 2] == 0)


def test_relabelling_permutes_scores():
    g = _small_sbm()
    rng = np.random.default_rng(3)
    perm = rng.permutation(g.n)           # new label of old node v is perm[v]
    rows = np.repeat(np.arange(g.n), g.degrees())
    h = ki.from_edges(g.n, zip(perm[rows], perm[g.col]))
    qs = ki.sample_queries(g, 3, 9)
    a = oracle.katz_oracle(g.n, g.row_ptr, g.col, qs, c=0.6)
    b = oracle.katz_oracle(h.n, h.row_ptr, h.col, perm[qs], beta=a["beta"])
    np.testing.assert_allclose(b["k"][perm, :], a["k"], rtol=1e-12, atol=1e-300)


# ----------------------------------------------------------------- P5
def test_convergence_condition():
    n, rp, col = _graph(2, [(0, 1)])
    with pytest.raises(oracle.OracleError):
        oracle.katz_oracle(n, rp, col, [0], beta=1.0)      # c = 1: M singular
    with pytest.raises(oracle.OracleError):
        oracle.katz_oracle(n, rp, col, [0], c=1.2)
    out = oracle.katz_oracle(n, rp, col, [0], c=0.999)
    b = 0.999
    # K_2: K_01 = b / (1 - b^2), K_00 = b^2 / (1 - b^2)
    np.testing.assert_allclose(out["k"][:, 0], [b * b / (1 - b * b), b / (1 - b * b)], rtol=1e-9)


@pytest.mark.parametrize("bad", ["asym", "loop", "unsorted", "range"])
def test_validation_rejects(bad):
    rp = np.array([0, 1, 2, 2], np.int32)
    col = np.array([1, 0], np.int32)
    if bad == "asym":
        rp, col = np.array([0, 1, 1, 1], np.int32), np.array([1], np.int32)
    elif bad == "loop":
        rp, col = np.array([0, 2, 3, 3], np.int32), np.array([0, 1, 0], np.int32)
    elif bad == "unsorted":
        rp, col = np.array([0, 2, 3, 4], np.int32), np.array([2, 1, 0, 0], np.int32)
    elif bad == "range":
        col = np.array([1, 5], np.int32)
    with pytest.raises(oracle.OracleError):
        oracle.validate_csr(3, rp, col)


# ------------------------------------------------------ series vs direct
@pytest.mark.parametrize("c", [0.1, 0.5, 0.9, 0.99])
def test_series_and_direct_agree_on_sbm(c):
    w = ki.workload("sbm2k", scale=0.3)
    g = w.graph
    qs = ki.sample_queries(g, 4, 11)
    out = oracle.katz_oracle(g.n, g.row_ptr, g.col, qs, c=c)
    assert np.all(out["cross_rel"] <= 1e-11)
    assert np.all(out["residual"] <= 1e-12)
    assert np.all(out["k"] >= 0)


def test_lambda_max_sparse_branch_closed_forms():
    # lambda_max above 4000 nodes runs the sparse (ARPACK) branch: K(2, 4000)
    # has sqrt(2 * 4000), its Perron vector is not the constant start vector;
    # a weighted star has ||w||; a 6000-node cycle (2-regular) has 2
    n, rp, col = _graph(4002, [(u, 2 + v) for u in range(2) for v in range(4000)])
    assert ko.lambda_max(ko.csr_matrix(n, rp, col)) == pytest.approx(math.sqrt(8000), rel=1e-11)
    w = 0.5 + (np.arange(4500) % 7) * 0.25
    n, rp, col, val = weighted_star(w)
    assert ko.lambda_max(ko.csr_matrix(n, rp, col, val)) == pytest.approx(np.linalg.norm(w), rel=1e-11)
    n, rp, col = cycle(6000)
    assert ko.lambda_max(ko.csr_matrix(n, rp, col)) == pytest.approx(2.0, rel=1e-11)


@pytest.mark.parametrize("c", [0.3, 0.8, 0.97])
def test_series_tail_bound_holds(c):
    # With a loose stopping tolerance the truncation error is far above
    # rounding, so the reported tail bound ||v_L|| c / (1 - c) is tested for
    # real against the dense solve: the dropped tail lies below it and is a
    # real fraction of it, and (every term >= 0) the truncated sum lies below
    # the exact solution entrywise.  A wrong ratio (c in place of c / (1 - c))
    # breaks the first check at every c here (error 1.3x to 33x the bound).
    g = ki.workload("sbm2k", scale=0.3).graph
    qs = ki.sample_queries(g, 3, 5)
    A = ko.csr_matrix(g.n, g.row_ptr, g.col)
    beta = c / ko.lambda_max(A)
    kd = ko.katz_direct(A, beta, qs)
    ks, terms, tail = ko.katz_series(A, beta, qs, c, tol=1e-4)
    err = np.linalg.norm(kd - ks, axis=0)
    nk = np.linalg.norm(kd, axis=0)
    assert np.all(err <= tail + 1e-12 * nk), (err, tail)
    assert np.all(err >= 0.05 * tail), (err, tail)
    assert np.all(ks <= kd + 1e-12 * np.abs(kd).max())
    assert np.all(tail <= 1e-4 * np.linalg.norm(ks, axis=0) * (1 + 1e-12))


# ------------------------------------------------------------------ top-K
def test_topk_star_leaf_query_ties_by_id():
    n, rp, col = star(6)
    out = oracle.katz_oracle(n, rp, col, [3], c=0.5)
    ids, sc, sids, ss = oracle.topk_links(n, rp, col, out["k"][:, 0], 3, 4)
    # centre 0 is the only neighbour; all other leaves tie -> ascending id
    assert list(ids) == [1, 2, 4, 5]
    assert np.all(sc == sc[0])
    ids, sc, _, _ = oracle.topk_links(n, rp, col, out["k"][:, 0], 3, 8)
    assert list(ids) == [1, 2, 4, 5, 6, -1, -1, -1] and np.isnan(sc[5:]).all()


def test_topk_path_orders_by_distance():
    n, rp, col = path(8)
    out = oracle.katz_oracle(n, rp, col, [0], c=0.5)
    ids, _, _, _ = oracle.topk_links(n, rp, col, out["k"][:, 0], 0, 6)
    assert list(ids) == [2, 3, 4, 5, 6, 7]


def test_tie_rule_acceptance():
    sids = np.array([10, 11, 12, 13, 14, 15])
    ss = np.array([5.0, 4.0, 4.0 - 1e-9, 3.0, 3.0, 1.0])
    ok = lambda b, K: oracle.topk_accept(b, sids, ss, K, 1e-6)[0]
    assert ok([10, 11, 12, 13], 4)
    assert ok([10, 12, 11, 14], 4)        # swap within class, straddle subset
    assert not ok([11, 10, 12, 13], 4)    # 10 and 11 are 1.0 apart
    assert not ok([10, 11, 12, 15], 4)
    assert ok([10, 11, 12, 13, 14, 15, -1], 7)
    assert not ok([10, 11, 12, 13, 14, 15, 99], 7)


# ------------------------------------------------- planted oracle mistakes
def test_pins_catch_planted_mistakes(monkeypatch):
    """Plants plausible mistakes in the oracle (on the CPU) and checks that the
    closed-form pins above reject each one."""
    n, rp, col = star(5)
    beta = 0.5 / math.sqrt(5)
    d = 1 - 5 * beta ** 2
    exp = np.full(6, beta / d)
    exp[0] = 5 * beta ** 2 / d

    def series_only():
        return oracle.katz_oracle(n, rp, col, [0], beta=beta, direct=False)["k"][:, 0]

    good = series_only()
    np.testing.assert_allclose(good, exp, rtol=SER)
    orig_rhs = ko.katz_rhs
    mistakes = {
        "dropped beta": lambda A, b, q: orig_rhs(A, 1.0, q),
        "e_q instead of A e_q": lambda A, b, q: b * np.eye(A.shape[0])[:, np.atleast_1d(q)],
        "transposed index": lambda A, b, q: b * A[np.atleast_1d(q), :].toarray().T[::-1],
    }
    for name, bad in mistakes.items():
        monkeypatch.setattr(ko, "katz_rhs", bad)
        got = series_only()
        assert not np.allclose(got, exp, rtol=1e-6), name
    monkeypatch.setattr(ko, "katz_rhs", orig_rhs)


def test_weighted_pins_catch_planted_mistakes(monkeypatch):
    """Plants mistakes in the oracle's handling of edge weights (on the CPU)
    and checks that the weighted star closed form rejects each one."""
    w = [0.5, 1.7, 0.3, 2.0, 1.1]
    n, rp, col, val = weighted_star(w)
    _, centre, j, leaf = _weighted_star_expected(w, 0.5)

    def run():
        out = oracle.katz_oracle(n, rp, col, [0, j], c=0.5, val=val, direct=False)
        return out["k"]

    good = run()
    np.testing.assert_allclose(good[:, 0], centre, rtol=1e-12)
    orig_csr, orig_lam = ko.csr_matrix, ko.lambda_max

    def pattern_lambda(A):
        B = A.copy()
        B.data[:] = 1.0
        return orig_lam(B)

    mistakes = {
        "weights dropped": (
            "csr_matrix", lambda n_, rp_, col_, val_=None: orig_csr(n_, rp_, col_, None)),
        "weights in reverse entry order": (
            "csr_matrix", lambda n_, rp_, col_, val_=None: orig_csr(
                n_, rp_, col_, None if val_ is None else np.asarray(val_)[::-1])),
        "lambda_max of the unweighted pattern": ("lambda_max", pattern_lambda),
    }
    for name, (attr, bad) in mistakes.items():
        monkeypatch.setattr(ko, attr, bad)
        got = run()
        assert not (np.allclose(got[:, 0], centre, rtol=1e-6)
                    and np.allclose(got[:, 1], leaf, rtol=1e-6)), name
        monkeypatch.setattr(ko, "csr_matrix", orig_csr)
        monkeypatch.setattr(ko, "lambda_max", orig_lam)


# ------------------------------------------------ residual (P8 support)
@pytest.mark.parametrize("n,beta", [(6, 0.1), (9, 0.05)])
def test_residual_closed_forms_complete_graph(n, beta):
    """||b - (I - beta A) k|| / ||b|| on K_n, q = 0, b = beta A e_q (eq.
    LinearSystem), for three k with hand-derived values: k = 0 gives 1;
    k = b gives ||beta A b|| / ||b|| with A b = (n-2) on v != q and (n-1) at
    q; the closed-form Katz vector gives 0 (to rounding)."""
    nn, rp, col = complete(n)
    A = ko.csr_matrix(nn, rp, col)
    b = ko.katz_rhs(A, beta, [0])
    assert ko.katz_residual(A, beta, [0], np.zeros((n, 1)))[0] == pytest.approx(1.0, abs=1e-15)
    want = beta * math.sqrt((n - 1) * (n - 2) ** 2 + (n - 1) ** 2) / math.sqrt(n - 1)
    assert ko.katz_residual(A, beta, [0], b)[0] == pytest.approx(want, rel=1e-14)
    d = (1 + beta) * (1 - (n - 1) * beta)
    k = np.full((n, 1), beta / d)
    k[0, 0] = (n - 1) * beta ** 2 / d
    assert ko.katz_residual(A, beta, [0], k)[0] < 1e-14


# ------------------------------------------------- Sparse-Katz (Algorithm 3)
def test_sparse_katz_cycle_closed_form():
    """On the cycle C_n every Katz score is a closed form of the distance, so
    the candidate list, the modular nodes, K_T and the correlations all follow
    from it (no solve): the oracle's re-ranked list must match."""
    n, q, s, T = 23, 0, 8, 6
    nn, rp, col = cycle(n)
    beta = 0.3
    sq = math.sqrt(1 - 4 * beta ** 2)
    t = (1 - sq) / (2 * beta)

    def K(d):
        d = np.minimum(d % n, (-d) % n)
        return (t ** d + t ** (n - d)) / (sq * (1 - t ** n)) - (d == 0)

    cand = [v for v in range(n) if v not in (q, 1, n - 1)]
    cand.sort(key=lambda v: (-K(v - q), v))
    mods = cand[:T]
    KT = np.array([[K(v - m) for m in mods] for v in range(n)])
    rho = []
    for v in cand[:s]:
        x, y = KT[q], KT[v]
        rho.append(np.corrcoef(x, y)[0, 1] if np.ptp(y) > 0 else np.nan)
    want = [v for _, v in sorted(zip([-r for r in rho], cand[:s]), key=lambda p: (p[0], cand.index(p[1])))]
    want_rho = sorted(rho, reverse=True)
    got = oracle.sparse_katz(nn, rp, col, q, s, T, beta)
    assert list(got["katz_order"]) == cand[:s]
    assert list(got["modular"]) == mods
    np.testing.assert_allclose(got["katz_rho"], rho, rtol=0, atol=1e-9)
    # mirror-image nodes have exactly equal correlations: any order inside a
    # tie class is right (the same rule as for the top-K list)
    ok, msg, ntie = oracle.topk_accept(got["ids"], np.array(want), np.array(want_rho), s, 1e-9)
    assert ok, msg
    assert ntie >= 1
    assert sorted(got["ids"].tolist()) == sorted(cand[:s])          # a permutation of the top-s list
    assert np.all(np.abs(got["rho"]) <= 1 + 1e-12)


def test_sparse_katz_correlation_step_by_hand():
    """The oracle's correlation and re-rank step (Algorithm 3, last step) on
    rows whose correlations are worked out by hand: x = (1, 2, 3, 4) has
    deviations (-1.5, -0.5, 0.5, 1.5), sum of squares 5.
      (2, 4, 6, 8): rho = 1;   (4, 3, 2, 1): rho = -1;
      (1, 3, 2, 4): deviations (-1.5, 0.5, -0.5, 1.5), cross sum 4, rho = 0.8;
      (2, 1, 4, 3): deviations (-0.5, -1.5, 1.5, 0.5), cross sum 3, rho = 0.6;
      (5, 5, 5, 5): constant, undefined (last);  (3, 6, 9, 12): rho = 1 (tie,
      keeps the Katz order after (2, 4, 6, 8))."""
    x = [1.0, 2.0, 3.0, 4.0]
    rows = [[5, 5, 5, 5], [4, 3, 2, 1], [2, 1, 4, 3], [2, 4, 6, 8], [1, 3, 2, 4], [3, 6, 9, 12]]
    order, rho = oracle.correlation_rerank(x, rows)
    want = [float("nan"), -1.0, 0.6, 1.0, 0.8, 1.0]
    assert np.isnan(rho[0])
    np.testing.assert_allclose(rho[1:], want[1:], rtol=0, atol=1e-15)
    assert order == [3, 5, 4, 2, 1, 0]
    assert np.isnan(oracle.pearson([1.0, 2.0], [7.0, 7.0]))
    assert oracle.pearson([0.0, 1.0, 0.0], [0.0, 0.0, 1.0]) == pytest.approx(-0.5, abs=1e-15)
