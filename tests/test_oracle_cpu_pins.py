"""Pins for the multi-core CPU tools (oracle/katz_cpu.c): the truncated
Neumann series that serves as the oracle at benchmark sizes, and the plain
CPU CG baseline.  Each check compares them with something other than
themselves: closed forms for complete, star, weighted star and cycle graphs,
walk counts enumerated by hand or stored in tests/golden, the tail bound
against a closed form at a loose stop, reachability, and thread-count
independence (Section 3.1, eqs. KatzPath, KatzMatrix, LinearSystem).  CPU
only."""
import json
import math
import os

import numpy as np
import pytest

import katz_inputs as ki
from oracle import cpu


def _graph(n, edges):
    g = ki.from_edges(n, edges)
    return g.n, g.row_ptr, g.col


def complete(n):
    return _graph(n, [(i, j) for i in range(n) for j in range(i + 1, n)])


def star(m):
    return _graph(m + 1, [(0, i) for i in range(1, m + 1)])


def cycle(n):
    return _graph(n, [(i, (i + 1) % n) for i in range(n)])


def complete_expected(n, beta, q):
    # A = J - I; (I - beta A)^{-1} by Sherman-Morrison: K_pq = beta / d,
    # K_qq = (n - 1) beta^2 / d with d = (1 + beta)(1 - (n - 1) beta)
    d = (1 + beta) * (1 - (n - 1) * beta)
    e = np.full(n, beta / d)
    e[q] = (n - 1) * beta ** 2 / d
    return e


def cycle_expected(n, beta, q):
    # periodic Green's function of x_j - beta (x_{j-1} + x_{j+1}) = delta_j0
    s = math.sqrt(1 - 4 * beta ** 2)
    t = (1 - s) / (2 * beta)
    e = np.empty(n)
    for v in range(n):
        dl = (v - q) % n
        e[v] = (t ** dl + t ** (n - dl)) / (s * (1 - t ** n)) - (1.0 if dl == 0 else 0.0)
    return e


@pytest.mark.parametrize("n,beta", [(6, 0.1), (12, 0.02), (40, 0.02)])
def test_series_complete_graph_closed_form(n, beta):
    nn, rp, col = complete(n)
    c = beta * (n - 1)                      # lambda_max(K_n) = n - 1
    qs = [0, n - 1, 3, 0]                   # a repeated query gives the same column
    r = cpu.katz_series_mt(nn, rp, col, qs, beta, c)
    for j, q in enumerate(qs):
        np.testing.assert_allclose(r["k"][:, j], complete_expected(n, beta, q), rtol=3e-13, atol=0)
    assert np.array_equal(r["k"][:, 0], r["k"][:, 3])
    assert np.all(r["tail"] <= 1e-13 * np.linalg.norm(r["k"], axis=0))


@pytest.mark.parametrize("m,c", [(5, 0.5), (9, 0.9), (3, 0.1)])
def test_series_star_closed_form(m, c):
    # lambda_max = sqrt(m); d = 1 - m beta^2: K_cc = m beta^2 / d,
    # K_c,leaf = beta / d, K_leaf,leaf' = K_leaf,leaf = beta^2 / d
    beta = c / math.sqrt(m)
    d = 1 - m * beta ** 2
    n, rp, col = star(m)
    r = cpu.katz_series_mt(n, rp, col, [0, 2], beta, c)
    centre = np.full(m + 1, beta / d)
    centre[0] = m * beta ** 2 / d
    leaf = np.full(m + 1, beta ** 2 / d)
    leaf[0] = beta / d
    np.testing.assert_allclose(r["k"][:, 0], centre, rtol=3e-13)
    np.testing.assert_allclose(r["k"][:, 1], leaf, rtol=3e-13)


@pytest.mark.parametrize("n,beta", [(9, 0.2), (8, 0.45), (301, 0.3)])
def test_series_cycle_closed_form(n, beta):
    nn, rp, col = cycle(n)
    q = 3 % n
    r = cpu.katz_series_mt(nn, rp, col, [q], beta, 2 * beta)   # lambda_max(C_n) = 2
    e = cycle_expected(n, beta, q)
    np.testing.assert_allclose(r["k"][:, 0], e, rtol=1e-12, atol=3e-13 * np.linalg.norm(e))


@pytest.mark.parametrize("w,c", [([0.5, 1.7, 0.3, 2.0, 1.1], 0.5), ([3.0, 0.25, 0.75], 0.9)])
def test_series_weighted_star_closed_form(w, c):
    # centre 0 joins leaf i with weight w_i; lambda_max = ||w||, beta ||w|| = c.
    # Centre query: k_0 = c^2 / (1 - c^2), k_i = beta w_i / (1 - c^2).
    # Leaf query j: k_0 = beta w_j / (1 - c^2), k_i = beta^2 w_i w_j / (1 - c^2).
    w = np.asarray(w, np.float64)
    m = len(w)
    n, rp, col = star(m)
    val = np.concatenate([w, w])            # row 0: leaves 1..m; row i: the centre
    beta = c / np.linalg.norm(w)
    d = 1 - c * c
    j = 2
    r = cpu.katz_series_mt(n, rp, col, [0, j], beta, c, val=val)
    np.testing.assert_allclose(r["k"][:, 0], np.concatenate([[c * c / d], beta * w / d]), rtol=1e-12)
    np.testing.assert_allclose(r["k"][:, 1], np.concatenate([[beta * w[j - 1] / d], beta ** 2 * w * w[j - 1] / d]),
                               rtol=1e-12)


def _walk_counts_by_hand(n, rp, col, q, L):
    """counts[l][v]: walks q -> v with l edges, by depth-first enumeration."""
    counts = [[0] * n for _ in range(L + 1)]

    def dfs(u, depth):
        if depth:
            counts[depth][u] += 1
        if depth == L:
            return
        for e in range(rp[u], rp[u + 1]):
            dfs(int(col[e]), depth + 1)

    dfs(q, 0)
    return counts


def test_series_walk_sums_golden_and_enumerated():
    # eq. KatzPath with walks: sum_{l <= L} beta^l count_l(v) lies below k_v
    # and within the entrywise tail c^(L+1) / (1 - c) of it (|(beta A)^l e_q|
    # <= c^l entrywise).  Counts from the stored fixture and from enumeration.
    with open(os.path.join(os.path.dirname(__file__), "golden", "walks_tri_tail.json")) as f:
        gold = json.load(f)
    n, rp, col = _graph(gold["n"], [tuple(e) for e in gold["edges"]])
    A = np.zeros((n, n))
    for u in range(n):
        A[u, col[rp[u]:rp[u + 1]]] = 1.0
    lam = float(np.linalg.eigvalsh(A)[-1])
    L = gold["max_len"]
    assert _walk_counts_by_hand(n, rp, col, gold["q"], L) == gold["counts"]
    for c in (0.05, 0.6):
        beta = c / lam
        r = cpu.katz_series_mt(n, rp, col, [gold["q"]], beta, c)
        trunc = np.array([sum(beta ** l * gold["counts"][l][v] for l in range(1, L + 1)) for v in range(n)])
        bound = c ** (L + 1) / (1 - c)
        k = r["k"][:, 0]
        assert np.all(k >= trunc - 1e-15)
        assert np.all(k - trunc <= bound + 1e-15)
    # a second graph, every query node, counts enumerated here
    n, rp, col = _graph(7, [(0, 1), (0, 2), (1, 3), (1, 4), (2, 5), (5, 6), (3, 4)])
    A = np.zeros((n, n))
    for u in range(n):
        A[u, col[rp[u]:rp[u + 1]]] = 1.0
    lam = float(np.linalg.eigvalsh(A)[-1])
    L, c = 10, 0.4
    beta = c / lam
    r = cpu.katz_series_mt(n, rp, col, list(range(n)), beta, c)
    for q in range(n):
        cnt = _walk_counts_by_hand(n, rp, col, q, L)
        trunc = np.array([sum(beta ** l * cnt[l][v] for l in range(1, L + 1)) for v in range(n)])
        k = r["k"][:, q]
        assert np.all(k >= trunc - 1e-15)
        assert np.all(k - trunc <= c ** (L + 1) / (1 - c) + 1e-15)


@pytest.mark.parametrize("beta", [0.15, 0.4, 0.485])
def test_series_tail_bound_at_loose_stop(beta):
    # With a loose stop the truncation error is real: it lies below the
    # reported bound ||v_L|| c / (1 - c), is a real fraction of it, and every
    # entry of the partial sum lies below the closed form (terms >= 0).
    n = 64
    nn, rp, col = cycle(n)
    c = 2 * beta
    r = cpu.katz_series_mt(nn, rp, col, [5], beta, c, tol=1e-4)
    e = cycle_expected(n, beta, 5)
    err = np.linalg.norm(e - r["k"][:, 0])
    assert err <= r["tail"][0] * (1 + 1e-9)
    assert err >= 0.05 * r["tail"][0]
    assert np.all(r["k"][:, 0] <= e + 1e-14)
    assert r["tail"][0] <= 1e-4 * np.linalg.norm(r["k"][:, 0]) * (1 + 1e-12)


def test_series_reachability_isolated_and_threads():
    # disjoint union of K_5 and C_7 plus an isolated node: scores across
    # components are exactly 0, an isolated query has k = 0; the result does
    # not depend on the thread count
    edges = [(i, j) for i in range(5) for j in range(i + 1, 5)]
    edges += [(5 + i, 5 + (i + 1) % 7) for i in range(7)]
    n, rp, col = _graph(13, edges)
    beta = 0.2
    c = 4 * beta
    qs = [1, 8, 12]
    r1 = cpu.katz_series_mt(n, rp, col, qs, beta, c, threads=1)
    r3 = cpu.katz_series_mt(n, rp, col, qs, beta, c, threads=3)
    assert np.array_equal(r1["k"], r3["k"]) and r3["threads"] == 3
    k = r1["k"]
    assert np.all(k[5:, 0] == 0) and np.all(k[:5, 0] > 0)
    assert np.all(k[:5, 1] == 0) and np.all(k[12:, 1] == 0) and np.all(k[5:12, 1] > 0)
    assert np.all(k[:, 2] == 0)
    np.testing.assert_allclose(k[:5, 0], complete_expected(5, beta, 1), rtol=3e-13)


def test_series_rejects_divergent_and_bad_ids():
    n, rp, col = cycle(6)
    with pytest.raises(ValueError):
        cpu.katz_series_mt(n, rp, col, [0], 0.5, 1.0)
    with pytest.raises(ValueError):
        cpu.katz_series_mt(n, rp, col, [6], 0.1, 0.2)


@pytest.mark.parametrize("tol", [1e-6, 1e-11])
def test_cg_closed_forms(tol):
    # plain CG reaches the requested true residual; its error is then within
    # tol (1 + c) / (1 - c) of the closed form
    cases = []
    n, rp, col = complete(30)
    cases.append((n, rp, col, 0.02, 29 * 0.02, [0, 7], lambda q: complete_expected(30, 0.02, q)))
    n, rp, col = cycle(101)
    cases.append((n, rp, col, 0.45, 0.9, [3, 50], lambda q: cycle_expected(101, 0.45, q)))
    for n, rp, col, beta, c, qs, exp in cases:
        r = cpu.cg_mt(n, rp, col, qs, beta, tol=tol)
        assert r["converged"]
        assert np.all(r["rel_residual"] <= tol)
        for j, q in enumerate(qs):
            e = exp(q)
            assert np.linalg.norm(r["k"][:, j] - e) <= tol * (1 + c) / (1 - c) * np.linalg.norm(e) * 1.01


def test_cg_isolated_query_and_star():
    n, rp, col = _graph(6, [(0, 1), (0, 2), (0, 3)])   # star on 0..3, nodes 4 and 5 isolated
    beta = 0.5 / math.sqrt(3)
    r = cpu.cg_mt(n, rp, col, [4, 0], beta, tol=1e-12)
    assert np.all(r["k"][:, 0] == 0) and r["rel_residual"][0] == 0 and r["iters"][0] == 0
    d = 1 - 3 * beta ** 2
    want = np.array([3 * beta ** 2 / d, beta / d, beta / d, beta / d, 0, 0])
    np.testing.assert_allclose(r["k"][:, 1], want, rtol=1e-11, atol=1e-15)


# ---------------------------------------------------------------- lambda_max
def _path(n):
    return _graph(n, [(i, i + 1) for i in range(n - 1)])


def _bipartite(a, b):
    return _graph(a + b, [(i, a + j) for i in range(a) for j in range(b)])


def _petersen():
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    return _graph(10, outer + spokes + inner)


@pytest.mark.parametrize("name,gr,expected", [
    ("K6", lambda: complete(6), 5.0),
    ("K40", lambda: complete(40), 39.0),
    ("star50", lambda: star(50), math.sqrt(50)),
    ("star4000", lambda: star(4000), math.sqrt(4000)),
    ("K(2,4000)", lambda: _bipartite(2, 4000), math.sqrt(8000)),
    ("cycle6000", lambda: cycle(6000), 2.0),
    ("cycle7", lambda: cycle(7), 2.0),
    ("path50", lambda: _path(50), 2 * math.cos(math.pi / 51)),
    ("petersen", _petersen, 3.0),
])
def test_lambda_max_closed_forms(name, gr, expected):
    """lambda_max of graphs whose spectrum is known: K_n (n - 1), a star and
    K(a, b) (sqrt(m), sqrt(ab)), regular graphs (the degree), a path
    (2 cos(pi / (n + 1)))."""
    n, rp, col = gr()
    r = cpu.lambda_max_mt(n, rp, col)
    assert abs(r["lambda"] - expected) <= 1e-11 * expected, (name, r, expected)


def test_lambda_max_weighted_star_and_union():
    """A weighted star has lambda_max = ||w||; a disjoint union takes the
    larger component's value (star of 9 leaves: 3, beside K_5: 4)."""
    m = 7
    w = np.array([0.5, 1.5, 2.0, 0.25, 3.0, 1.0, 0.75])
    g = ki.from_edges(m + 1, [(0, i) for i in range(1, m + 1)])
    val = np.empty(g.row_ptr[-1])
    for i in range(g.n):
        for e in range(g.row_ptr[i], g.row_ptr[i + 1]):
            j = g.col[e]
            val[e] = w[max(i, j) - 1]
    r = cpu.lambda_max_mt(g.n, g.row_ptr, g.col, val=val)
    assert abs(r["lambda"] - np.linalg.norm(w)) <= 1e-12 * np.linalg.norm(w)
    edges = [(0, i) for i in range(1, 10)] + [(10 + i, 10 + j) for i in range(5) for j in range(i + 1, 5)]
    n, rp, col = _graph(15, edges)
    r = cpu.lambda_max_mt(n, rp, col)
    assert abs(r["lambda"] - 4.0) <= 1e-11 * 4
    # no edges: 0
    r = cpu.lambda_max_mt(5, np.zeros(6, np.int64), np.zeros(0, np.int32))
    assert r["lambda"] == 0.0


def test_lambda_max_random_graphs_vs_dense_and_threads():
    """Random community graphs: equal to the dense eigensolve of A, and
    bit-identical for 1 and 4 threads (fixed-order reductions)."""
    for seed in (1, 2, 3):
        g = ki.sbm([40, 60, 25], 0.2, 0.02, seed=seed)
        A = np.zeros((g.n, g.n))
        for i in range(g.n):
            A[i, g.col[g.row_ptr[i]:g.row_ptr[i + 1]]] = 1.0
        ev = np.linalg.eigvalsh(A)[-1]
        r1 = cpu.lambda_max_mt(g.n, g.row_ptr, g.col, threads=1)
        r4 = cpu.lambda_max_mt(g.n, g.row_ptr, g.col, threads=4)
        assert abs(r1["lambda"] - ev) <= 1e-11 * ev, (seed, r1, ev)
        assert r1["lambda"] == r4["lambda"]
