"""Parity of the HIP query path (through the C ABI) against the CPU FP64
oracle.  GPU only.

Tolerances: a returned k with true relative residual rho satisfies
||k - k*|| / ||k*|| <= rho (1 + c) / (1 - c) (kappa(M) <= (1+c)/(1-c),
Sec. 3.1).  Tests request rho = tau (1 - c) / (1 + c) so that the error is
below tau (norm-wise and entrywise against ||k||), with tau = 1e-6 for the
FP64 path and 1e-9 for the small 2,000-node SBM solved to 1e-10 residual.
"""
import math

import numpy as np
import pytest
from conftest import oracle_beta

import katz_inputs as ki
import oracle

pytestmark = pytest.mark.gpu

K = pytest.importorskip("paper_1912_06525_amd")


def _accept(kh, k, tau, what=""):
    nk = np.linalg.norm(k)
    err = np.linalg.norm(kh - k)
    assert err <= tau * max(nk, 1e-300), "%s: rel err %.3e > %.1e" % (what, err / max(nk, 1e-300), tau)
    assert np.max(np.abs(kh - k)) <= tau * max(nk, 1e-300), what


def _check(g, idx, beta, qs, tau, method=K.KATZ_METHOD_LRC, **kw):
    # beta: the test's own value, given to the index build and to the oracle
    c = idx.info.c
    tol = tau * (1 - c) / (1 + c)
    sc, st = idx.query(qs, tol=tol, method=method, **kw)
    ref = oracle.katz_oracle(g.n, g.row_ptr, g.col, qs, beta=beta, validate=False)
    A = oracle.csr_matrix(g.n, g.row_ptr, g.col)
    res = oracle.katz_residual(A, beta, qs, sc.T)
    for j, q in enumerate(qs):
        assert st[j]["status"] == 0, st[j]
        _accept(sc[j], ref["k"][:, j], tau, "q=%d" % q)
        assert res[j] <= 1.05 * tol + 1e-15, (res[j], tol)
        assert abs(st[j]["rel_residual"] - res[j]) <= 1e-3 * tol + 1e-15
    return sc, st


@pytest.fixture(scope="module")
def sbm2k():
    w = ki.workload("sbm2k")
    return w


@pytest.mark.parametrize("method", [K.KATZ_METHOD_LRC, K.KATZ_METHOD_CG])
@pytest.mark.parametrize("rank,uprec", [(0, 0), (5, 1), (32, 2), (32, 3)])
def test_sbm2k_fp64_1e10(sbm2k, method, rank, uprec):
    g = sbm2k.graph
    beta = oracle_beta(g, 0.5)
    idx = K.KatzIndex.from_graph(g, beta=beta, rank=rank, labels=g.labels, max_block=200, u_precision=uprec)
    sc, st = idx.query(sbm2k.queries, tol=1e-10, method=method)
    ref = oracle.katz_oracle(g.n, g.row_ptr, g.col, sbm2k.queries, beta=beta)
    assert st[0]["status"] == 0 and st[0]["rel_residual"] <= 1e-10
    _accept(sc[0], ref["k_direct"][:, 0], 3.1e-10, "sbm2k")
    assert st[0]["path"] == (K.KATZ_PATH_CG if method == K.KATZ_METHOD_CG else K.KATZ_PATH_LRC)


def test_full_rank_converges_in_one_iteration(sbm2k):
    # Theorem 1 with r = n2 and exact eigenvectors: S S~^{-1} = I.
    g = ki.sbm([30, 30, 30], [0.3, 0.3, 0.3], 0.05, seed=8)
    beta = oracle_beta(g, 0.8)
    idx0 = K.KatzIndex.from_graph(g, beta=beta, rank=0, labels=g.labels, max_block=12, device=-1)
    n2 = idx0.info.n2
    idx = K.KatzIndex.from_graph(g, beta=beta, rank=n2, labels=g.labels, max_block=12,
                                 l_kind=K.KATZ_L_CHOL, lanczos_steps=10 ** 6, u_precision=1)
    qs = ki.sample_queries(g, 3, 4)
    sc, st = _check(g, idx, beta, qs, 1e-9)
    assert all(s["iters"] <= 2 for s in st), st


@pytest.mark.parametrize("order", [K.KATZ_ORDER_DEGREE, K.KATZ_ORDER_LOCALITY])
@pytest.mark.parametrize("lk", [K.KATZ_L_CHOL, K.KATZ_L_IDENTITY])
@pytest.mark.parametrize("c", [0.1, 0.5, 0.9, 0.99])
def test_small_sbm_both_factors(lk, c, order):
    # dense chol(M22) is for small separators: a smaller graph for CHOL
    g = ki.workload("lnsbm4m", scale=0.0006 if lk == K.KATZ_L_CHOL else 0.002).graph
    beta = oracle_beta(g, c)
    idx = K.KatzIndex.from_graph(g, beta=beta, rank=16, labels=g.labels, max_block=32, l_kind=lk, order=order)
    qs = ki.sample_queries(g, 5, 31)
    _check(g, idx, beta, qs, 1e-6)


@pytest.mark.parametrize("prec", [K.KATZ_PREC_FP64, K.KATZ_PREC_MIXED])
@pytest.mark.parametrize("lk", [K.KATZ_L_CHOL, K.KATZ_L_IDENTITY])
@pytest.mark.parametrize("B", [2, 3])
def test_narrow_batches_match_oracle(B, lk, prec):
    # 2 and 3 columns through the narrow low-rank kernels: 128 row groups per
    # workgroup (2 columns) and a column lane past the batch (3 of 4), with the
    # unfused (CHOL) and fused (identity) preconditioner in both precisions
    g = ki.workload("lnsbm4m", scale=0.0006 if lk == K.KATZ_L_CHOL else 0.002).graph
    beta = oracle_beta(g, 0.9)
    idx = K.KatzIndex.from_graph(g, beta=beta, rank=16, labels=g.labels, max_block=32, l_kind=lk,
                                 precision=prec)
    qs = ki.sample_queries(g, B, 41)
    _check(g, idx, beta, qs, 1e-6)


def test_closed_forms_through_gpu():
    import math
    # star with m leaves: K_c,leaf = beta/d, K_leaf,leaf' = beta^2/d, d = 1 - m beta^2
    m = 40
    g = ki.from_edges(m + 1, [(0, i) for i in range(1, m + 1)])
    beta = 0.9 / math.sqrt(m)  # lambda_max of the star is sqrt(m)
    idx = K.KatzIndex.from_graph(g, beta=beta, rank=1)
    d = 1 - m * beta ** 2
    sc, st = idx.query([0, 5], tol=1e-12)
    exp0 = np.full(m + 1, beta / d)
    exp0[0] = m * beta ** 2 / d
    exp5 = np.full(m + 1, beta ** 2 / d)
    exp5[0] = beta / d
    np.testing.assert_allclose(sc[0], exp0, rtol=1e-10)
    np.testing.assert_allclose(sc[1], exp5, rtol=1e-10)
    assert abs(idx.info.lambda_max - math.sqrt(m)) < 1e-10
    # complete graph K_n: K_pq = beta / ((1+beta)(1-(n-1)beta))
    n = 30
    g = ki.from_edges(n, [(i, j) for i in range(n) for j in range(i + 1, n)])
    beta = 0.7 / (n - 1)  # lambda_max of K_n is n - 1
    idx = K.KatzIndex.from_graph(g, beta=beta, rank=2, max_block=8)
    den = (1 + beta) * (1 - (n - 1) * beta)
    sc, _ = idx.query([3], tol=1e-12)
    exp = np.full(n, beta / den)
    exp[3] = (n - 1) * beta ** 2 / den
    np.testing.assert_allclose(sc[0], exp, rtol=1e-10)
    # cycle C_n
    n, q = 101, 7
    g = ki.from_edges(n, [(i, (i + 1) % n) for i in range(n)])
    beta = 0.8 / 2  # lambda_max of a cycle is 2
    idx = K.KatzIndex.from_graph(g, beta=beta, rank=4, max_block=10)
    s = math.sqrt(1 - 4 * beta ** 2)
    t = (1 - s) / (2 * beta)
    sc, _ = idx.query([q], tol=1e-12)
    dl = (np.arange(n) - q) % n
    exp = (t ** dl + t ** (n - dl)) / (s * (1 - t ** n)) - (dl == 0)
    np.testing.assert_allclose(sc[0], exp, rtol=1e-9, atol=1e-12 * np.linalg.norm(exp))


def test_isolated_and_disconnected():
    g = ki.from_edges(12, [(0, 1), (1, 2), (2, 0), (2, 3), (5, 6), (6, 7), (7, 8), (8, 5)])
    idx = K.KatzIndex.from_graph(g, beta_frac=0.6, rank=2, max_block=3)
    sc, st = idx.query([4, 1, 6], tol=1e-12)
    assert np.all(sc[0] == 0) and st[0]["status"] == 0          # isolated node 4
    # exact zeros across components in exact arithmetic; the rank-r
    # preconditioner's Ritz vectors span components, so PCG leaves rounding-level
    # values there
    tiny = lambda x, k: np.all(np.abs(x) <= 1e-13 * np.linalg.norm(k))
    assert tiny(sc[1][4:], sc[1]) and np.all(sc[1][:4] > 0)
    assert tiny(sc[2][:5], sc[2]) and tiny(sc[2][9:], sc[2]) and np.all(sc[2][5:9] > 0)
    cg, _ = idx.query([1, 6], tol=1e-12, method=K.KATZ_METHOD_CG)
    assert np.all(cg[0][4:] == 0) and np.all(cg[1][:5] == 0) and np.all(cg[1][9:] == 0)


def test_batch_columns_match_single_solves():
    g = ki.workload("lnsbm4m", scale=0.003).graph
    idx = K.KatzIndex.from_graph(g, beta_frac=0.7, rank=8, labels=g.labels, max_block=32)
    qs = ki.sample_queries(g, 7, 3)
    tol = 1e-9
    sb, _ = idx.query(qs, tol=tol)
    for j, q in enumerate(qs):
        s1, _ = idx.query([q], tol=tol)
        _accept(sb[j], s1[0], 1e-7, "batch col %d" % j)


def test_forced_fallback_to_cg():
    g = ki.workload("lnsbm4m", scale=0.002).graph
    beta = oracle_beta(g, 0.9)
    idx = K.KatzIndex.from_graph(g, beta=beta, rank=4, labels=g.labels, max_block=32)
    qs = ki.sample_queries(g, 3, 5)
    # fault injection from the host: the first (LRC) sweep is declared broken
    # down, the refinement sweeps then run plain CG on the residual
    sc, st = idx.query(qs, tol=1e-8, force_fallback=True)
    assert all(s["path"] == K.KATZ_PATH_CG_FALLBACK for s in st)
    assert all(s["sweeps"] >= 1 and s["status"] == 0 for s in st)
    ref = oracle.katz_oracle(g.n, g.row_ptr, g.col, qs, beta=beta)
    for j in range(len(qs)):
        _accept(sc[j], ref["k"][:, j], 1e-8 * 19 * 1.05, "fallback")
    # an iteration cap on every path ends in KATZ_ENOCONV with the best iterate
    sc, st = idx.query(qs, tol=1e-12, max_iter=2, max_sweeps=2)
    assert all(s["status"] == K.KATZ_ENOCONV for s in st)


def test_device_output_buffer():
    import torch
    g = ki.workload("sbm2k").graph
    idx = K.KatzIndex.from_graph(g, beta_frac=0.5, rank=8, labels=g.labels)
    qs = ki.sample_queries(g, 3, 99)
    out = torch.empty((3, g.n), dtype=torch.float64, device="cuda")
    idx.query(qs, out=out, tol=1e-10)
    torch.cuda.synchronize()
    host, _ = idx.query(qs, tol=1e-10)
    assert np.array_equal(out.cpu().numpy(), host)


@pytest.mark.parametrize("K_", [1, 10, 100])
def test_topk_matches_oracle(K_):
    g = ki.workload("lnsbm4m", scale=0.003).graph
    beta = oracle_beta(g, 0.5)
    idx = K.KatzIndex.from_graph(g, beta=beta, rank=8, labels=g.labels, max_block=32)
    qs = ki.sample_queries(g, 4, 123)
    tau = 1e-9
    tol = tau * (1 - 0.5) / (1 + 0.5)
    ids, scs, st = idx.topk(qs, K_, tol=tol)
    ref = oracle.katz_oracle(g.n, g.row_ptr, g.col, qs, beta=beta)
    for j, q in enumerate(qs):
        k = ref["k"][:, j]
        oid, osc, sid, ssc = oracle.topk_links(g.n, g.row_ptr, g.col, k, q, K_)
        ok, msg, _ = oracle.topk_accept(ids[j], sid, ssc, K_, 2 * tau * np.linalg.norm(k))
        assert ok, msg
        m = ids[j] >= 0
        np.testing.assert_allclose(scs[j][m], k[ids[j][m]], rtol=0, atol=tau * np.linalg.norm(k))


def test_topk_ties_and_padding():
    # star: leaf query -> every other leaf ties exactly (K_leaf,leaf' = beta^2/d);
    # fewer candidates than k -> padding with (-1, NaN)
    m = 9
    g = ki.from_edges(m + 1, [(0, i) for i in range(1, m + 1)])
    beta = 0.5 / math.sqrt(m)  # lambda_max of the star is sqrt(m)
    idx = K.KatzIndex.from_graph(g, beta=beta, rank=1)
    ids, scs, _ = idx.topk([4], 12, tol=1e-12)
    ref = oracle.katz_oracle(g.n, g.row_ptr, g.col, [4], beta=beta)
    k = ref["k"][:, 0]
    _, _, sid, ssc = oracle.topk_links(g.n, g.row_ptr, g.col, k, 4, 12)
    ok, msg, ntie = oracle.topk_accept(ids[0], sid, ssc, 12, 2e-10 * np.linalg.norm(k))
    assert ok, msg
    assert sorted(ids[0][:8].tolist()) == [1, 2, 3, 5, 6, 7, 8, 9] and ids[0][8:].tolist() == [-1] * 4
    assert np.isnan(scs[0][8:]).all() and ntie == 1


def test_loaded_index_answers_identically(tmp_path):
    # an index written by save() and loaded on the device gives the same bits
    g = ki.workload("lnsbm4m", scale=0.002).graph
    beta = oracle_beta(g, 0.7)
    a = K.KatzIndex.from_graph(g, beta=beta, rank=8, labels=g.labels, max_block=32)
    p = str(tmp_path / "idx.katz")
    a.save(p)
    b = K.KatzIndex.load(p, device=0)
    qs = ki.sample_queries(g, 5, 77)
    sa, sta = a.query(qs, tol=1e-9)
    sb, stb = b.query(qs, tol=1e-9)
    assert np.array_equal(sa, sb)
    assert [s["iters"] for s in sta] == [s["iters"] for s in stb]
    ia, xa, _ = a.topk(qs, 20, tol=1e-9)
    ib, xb, _ = b.topk(qs, 20, tol=1e-9)
    assert np.array_equal(ia, ib) and np.array_equal(xa, xb)


def test_pair_scores_match_oracle():
    # pairwise Katz K[dst, src]: repeated sources, src == dst (K_qq), an
    # isolated source and more distinct sources than one batch holds
    g = ki.workload("lnsbm4m", scale=0.002).graph
    beta = oracle_beta(g, 0.6)
    idx = K.KatzIndex.from_graph(g, beta=beta, rank=8, labels=g.labels, max_block=32)
    rng = np.random.default_rng(5)
    deg = np.diff(g.row_ptr)
    srcs = ki.sample_queries(g, 600, 41)               # > 512 distinct: two batches
    src = np.concatenate([srcs, srcs[:50], [srcs[3]]])
    dst = rng.integers(0, g.n, size=len(src)).astype(np.int32)
    dst[-1] = srcs[3]                                  # K_qq
    iso = np.nonzero(deg == 0)[0]
    if len(iso):
        src = np.append(src, iso[0])
        dst = np.append(dst, srcs[0])
    tau = 1e-8
    tol = tau * (1 - 0.6) / (1 + 0.6)
    sc, st = idx.pair_scores(src, dst, tol=tol)
    assert all(s["status"] == 0 for s in st)
    uq = np.unique(src)
    ref = oracle.katz_oracle(g.n, g.row_ptr, g.col, uq, beta=beta, validate=False)["k"]
    col = {int(q): j for j, q in enumerate(uq)}
    for t in range(len(src)):
        k = ref[:, col[int(src[t])]]
        assert abs(sc[t] - k[dst[t]]) <= tau * max(np.linalg.norm(k), 1e-300), t
    # device output buffer gives the same values
    import torch
    out = torch.empty(len(src), dtype=torch.float64, device="cuda")
    idx.pair_scores(src, dst, out=out, tol=tol)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), sc)


def test_device_lanczos_matches_host(monkeypatch):
    # the index build's Lanczos on R run on the device (forced) reproduces
    # the host run: same Ritz values, Ritz vectors up to sign, same answers
    g = ki.workload("lnsbm4m", scale=0.004).graph
    beta = oracle_beta(g, 0.9)
    monkeypatch.setenv("KATZ_LANCZOS", "1")
    a = K.KatzIndex.from_graph(g, beta=beta, rank=12, labels=g.labels, max_block=32)
    monkeypatch.setenv("KATZ_LANCZOS", "2")
    b = K.KatzIndex.from_graph(g, beta=beta, rank=12, labels=g.labels, max_block=32)
    assert a.info.l_kind == K.KATZ_L_IDENTITY and b.info.rank == a.info.rank == 12
    ua, sa = a.lowrank()
    ub, sb = b.lowrank()
    np.testing.assert_allclose(sb, sa, rtol=0, atol=1e-10)
    for t in range(len(sa) - 1):
        if sa[t] - sa[t + 1] > 1e-6 and (t == 0 or sa[t - 1] - sa[t] > 1e-6):  # simple, separated pairs
            assert abs(abs(ua[:, t] @ ub[:, t]) - 1.0) < 1e-6, t
    qs = ki.sample_queries(g, 4, 9)
    tol = 1e-9
    ka, sta = a.query(qs, tol=tol)
    kb, stb = b.query(qs, tol=tol)
    for j in range(len(qs)):
        assert np.linalg.norm(ka[j] - kb[j]) <= 20 * tol * np.linalg.norm(ka[j])


def test_device_lanczos_full_spectrum(monkeypatch):
    # Theorem 1 on the device path: with m = n2 steps the device Lanczos
    # returns the top eigenvalues of the dense R = I - S
    g = ki.sbm([40, 35, 45, 30], [0.3, 0.3, 0.3, 0.3], 0.04, seed=13)
    beta = oracle_beta(g, 0.8)
    monkeypatch.setenv("KATZ_LANCZOS", "2")
    idx = K.KatzIndex.from_graph(g, beta=beta, rank=6, labels=g.labels, max_block=8, l_kind=K.KATZ_L_IDENTITY,
                                 lanczos_steps=10 ** 6)
    info = idx.info
    perm, _ = idx.partition()
    A = oracle.csr_matrix(g.n, g.row_ptr, g.col).toarray()
    P = np.zeros((g.n, g.n))
    P[perm, np.arange(g.n)] = 1.0
    M = np.eye(g.n) - beta * (P @ A @ P.T)
    n1 = info.n1
    M11, M12, M22 = M[:n1, :n1], M[:n1, n1:], M[n1:, n1:]
    S = M22 - M12.T @ np.linalg.solve(M11, M12)
    sig = np.sort(np.linalg.eigvalsh(np.eye(info.n2) - S))[::-1]
    U, s = idx.lowrank()
    np.testing.assert_allclose(s, sig[:6], rtol=0, atol=1e-10)
    np.testing.assert_allclose(U.T @ U, np.eye(6), atol=1e-10)


@pytest.mark.parametrize("s,T", [(20, 8), (300, 5)])
def test_sparse_katz_matches_oracle(s, T):
    # Sparse-Katz (Algorithm 3): the re-ranked top-s list and its
    # correlations (computed and sorted on the device) against the oracle,
    # tie classes of correlation width 1e-7; a list longer than a workgroup
    # (300) takes several sort elements per thread
    g = ki.workload("lnsbm4m", scale=0.002).graph
    beta = oracle_beta(g, 0.7)
    idx = K.KatzIndex.from_graph(g, beta=beta, rank=8, labels=g.labels, max_block=32)
    qs = ki.sample_queries(g, 3, 61)
    ids, corr, st = idx.sparse_katz(qs, s, T, tol=1e-11)
    assert all(x["status"] == 0 for x in st)
    for i, q in enumerate(qs):
        ref = oracle.sparse_katz(g.n, g.row_ptr, g.col, int(q), s, T, beta)
        m = len(ref["ids"])
        assert np.all(ids[i][m:] == -1)
        fin = np.isfinite(ref["rho"])
        np.testing.assert_allclose(corr[i][:m][fin], ref["rho"][fin], rtol=0, atol=1e-7)
        # finite part: same order up to ties; undefined ones last, in Katz order
        nf = int(fin.sum())
        ok, msg, _ = oracle.topk_accept(ids[i][:nf], ref["ids"][:nf], ref["rho"][:nf], nf, 1e-7)
        assert ok, msg
        assert np.array_equal(ids[i][nf:m], ref["ids"][nf:m])


@pytest.mark.parametrize("own_streams", [True, False])
def test_concurrent_queries_from_threads(own_streams):
    # independent one-query solves from several host threads on a fresh index:
    # workspace creation overlaps the HIP-graph capture of other threads'
    # iteration chunks (>= 8 iterations per solve); results equal the
    # sequential ones bit for bit
    import threading
    import torch
    g = ki.workload("lnsbm4m", scale=0.002).graph
    beta = oracle_beta(g, 0.9)
    qs = ki.sample_queries(g, 24, 88)
    ref_idx = K.KatzIndex.from_graph(g, beta=beta, rank=8, labels=g.labels, max_block=32)
    ref = {int(q): ref_idx.query([q], tol=1e-11)[0][0] for q in qs}
    assert all(s["iters"] >= 8 for s in ref_idx.query(qs[:4], tol=1e-11)[1])
    idx = K.KatzIndex.from_graph(g, beta=beta, rank=8, labels=g.labels, max_block=32)
    got, errs = {}, []

    def worker(t):
        try:
            st = torch.cuda.Stream() if own_streams else None
            for q in qs[t::6]:
                out = torch.empty((1, g.n), dtype=torch.float64, device="cuda")
                idx.query([q], out=out, tol=1e-11, stream=st.cuda_stream if st else None)
                (st or torch.cuda.current_stream()).synchronize()
                got[int(q)] = out.cpu().numpy()[0]
        except Exception as e:
            errs.append(repr(e))
    ths = [threading.Thread(target=worker, args=(t,)) for t in range(6)]
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    assert not errs, errs[:2]
    for q in qs:
        assert np.array_equal(got[int(q)], ref[int(q)]), q


@pytest.mark.parametrize("prec", [K.KATZ_PREC_FP64, K.KATZ_PREC_MIXED])
@pytest.mark.parametrize("B", [1, 8, 40, 130])
def test_weighted_graph_matches_oracle(prec, B):
    # weighted adjacency (every kernel's weighted variant): one column, the
    # narrow and the 64-wide SpMM layouts, and blocks larger than the batched
    # block solve keeps in registers (tile kernel beside it)
    g = ki.workload("lnsbm4m", scale=0.002).graph
    val = ki.edge_weights(g, seed=3)
    A = oracle.csr_matrix(g.n, g.row_ptr, g.col, val)
    beta = 0.7 / oracle.lambda_max(A)
    idx = K.KatzIndex.from_graph(g, val=val, beta=beta, rank=8, labels=g.labels, max_block=32, precision=prec)
    _, bp = idx.partition()
    assert np.diff(bp).max() > 4
    qs = ki.sample_queries(g, B, 17)
    tau = 1e-6
    c = idx.info.c
    tol = tau * (1 - c) / (1 + c)
    ref = oracle.katz_oracle(g.n, g.row_ptr, g.col, qs, beta=beta, val=val, validate=False)["k"]
    for method in (K.KATZ_METHOD_LRC, K.KATZ_METHOD_CG):
        sc, st = idx.query(qs, tol=tol, method=method)
        res = oracle.katz_residual(A, beta, qs, sc.T)
        for j, q in enumerate(qs):
            assert st[j]["status"] == 0, st[j]
            _accept(sc[j], ref[:, j], tau, "method %d q=%d" % (method, q))
            assert res[j] <= 1.05 * tol + 1e-15, (res[j], tol)


@pytest.mark.parametrize("prec", [K.KATZ_PREC_FP64, K.KATZ_PREC_MIXED])
@pytest.mark.parametrize("B", [1, 7, 40])
def test_rank0_identity_preconditioner(prec, B):
    # L = I without a low-rank part: S~^{-1} = I, so <r, z> = <r, r> and the
    # search direction is p = r + bcg p (no preconditioner pass)
    g = ki.workload("lnsbm4m", scale=0.002).graph
    beta = oracle_beta(g, 0.8)
    idx = K.KatzIndex.from_graph(g, beta=beta, rank=0, labels=g.labels, max_block=32, precision=prec,
                                 l_kind=K.KATZ_L_IDENTITY)
    assert idx.info.rank == 0 and idx.info.l_kind == K.KATZ_L_IDENTITY
    qs = ki.sample_queries(g, B, 23)
    _check(g, idx, beta, qs, 1e-6)


@pytest.mark.parametrize("method", [K.KATZ_METHOD_LRC, K.KATZ_METHOD_CG])
def test_poll_schedule_does_not_change_results(method):
    # iterations after convergence change nothing, so every polling schedule
    # (adaptive with and without a hint, fixed intervals) gives the same bits
    g = ki.workload("lnsbm4m", scale=0.002).graph
    beta = oracle_beta(g, 0.8)
    idx = K.KatzIndex.from_graph(g, beta=beta, rank=8, labels=g.labels, max_block=32)
    qs = ki.sample_queries(g, 3, 29)
    ref, st_ref = idx.query(qs, tol=1e-9, method=method, check_every=1)
    for ce in (0, 0, 3, 8):   # the first adaptive call polls from a hint left by the previous one
        sc, st = idx.query(qs, tol=1e-9, method=method, check_every=ce)
        assert np.array_equal(sc, ref), ce
        assert [s["iters"] for s in st] == [s["iters"] for s in st_ref], ce


def test_query_wider_than_one_launch():
    # 530 queries: one launch of 512 columns (8 column groups per lane) and
    # one of 18, both against the oracle
    g = ki.workload("sbm2k").graph
    beta = oracle_beta(g, 0.5)
    idx = K.KatzIndex.from_graph(g, beta=beta, rank=8, labels=g.labels, max_block=64)
    qs = ki.sample_queries(g, 530, 31)
    assert len(qs) == 530
    _check(g, idx, beta, qs, 1e-6)


@pytest.mark.parametrize("c", [0.5, 0.9, 0.99])
@pytest.mark.parametrize("B", [1, 4, 40])
def test_ic0_factor_matches_oracle(c, B):
    """L = the zero-fill incomplete Cholesky factor of M22 (the preconditioner
    ablation, any SPD L serves Theorem 1): results equal the oracle's at 1,
    4 and 40 columns (the dense G apply with the unfused low-rank kernels)."""
    g = ki.workload("lnsbm4m", scale=0.0006).graph
    beta = oracle_beta(g, c)
    idx = K.KatzIndex.from_graph(g, beta=beta, rank=16, labels=g.labels, max_block=32, l_kind=K.KATZ_L_IC0)
    assert idx.info.l_kind == K.KATZ_L_IC0
    qs = ki.sample_queries(g, B, 61)
    _check(g, idx, beta, qs, 1e-6)


@pytest.mark.parametrize("prec", [K.KATZ_PREC_FP64, K.KATZ_PREC_MIXED])
@pytest.mark.parametrize("lk", [K.KATZ_L_CHOL, K.KATZ_L_IDENTITY, K.KATZ_L_IC0])
@pytest.mark.parametrize("B", [1, 6])
def test_pcgnr_ablation_matches_oracle(lk, B, prec):
    """The PCGNR ablation (Algorithm 2's recurrence with gamma = s^T S~^{-1} s)
    reaches the same Katz vectors as the oracle, with every L, both
    precisions, one and several columns; it needs at least as many
    iterations as PCG on these graphs."""
    g = ki.workload("lnsbm4m", scale=0.0006 if lk != K.KATZ_L_IDENTITY else 0.002).graph
    beta = oracle_beta(g, 0.9)
    idx = K.KatzIndex.from_graph(g, beta=beta, rank=16, labels=g.labels, max_block=32, l_kind=lk, precision=prec)
    qs = ki.sample_queries(g, B, 71)
    _, st = _check(g, idx, beta, qs, 1e-6, method=K.KATZ_METHOD_PCGNR)
    _, st2 = _check(g, idx, beta, qs, 1e-6, method=K.KATZ_METHOD_LRC)
    assert all(s["path"] == K.KATZ_PATH_LRC for s in st)
    assert sum(s["iters"] for s in st) >= sum(s["iters"] for s in st2)


def test_bad_method_rejected():
    g = ki.workload("sbm2k").graph
    idx = K.KatzIndex.from_graph(g, beta_frac=0.5, rank=4, labels=g.labels, max_block=200)
    with pytest.raises(K.KatzError) as e:
        idx.query([3], method=7)
    assert e.value.code == K.KATZ_EINVAL


_WALK_SCRIPT = r"""
import sys, numpy as np
sys.path.insert(0, sys.argv[2])
import katz_inputs as ki, paper_1912_06525_amd as K
g = ki.workload("lnsbm4m", scale=0.004).graph
out = {}
for prec in (K.KATZ_PREC_FP64, K.KATZ_PREC_MIXED):
    idx = K.KatzIndex.from_graph(g, beta_frac=0.9, rank=16, labels=g.labels, max_block=32, precision=prec)
    for B in (1, 40, 130):
        qs = ki.sample_queries(g, B, 90 + B)
        for m in (K.KATZ_METHOD_LRC, K.KATZ_METHOD_CG):
            sc, st = idx.query(qs, tol=1e-8, method=m)
            out["p%d_b%d_m%d" % (prec, B, m)] = sc
            out["p%d_b%d_m%d_it" % (prec, B, m)] = np.array([x["iters"] for x in st])
    idx.close()
np.savez(sys.argv[1], **out)
"""


def test_results_independent_of_chunk_walk(tmp_path):
    """The SpMM chunk walk (contiguous or XCD slabs, any workgroup count) is
    a timing choice: scores and iteration counts must be bit-identical under
    every walk, since each chunk's reduction terms have a fixed slot.  Each
    walk runs in a child process (the walk is pinned by the environment)."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    walks = [{}, {"KATZ_XCD_SLAB": "1"}, {"KATZ_SPMM_NWG": "1000"},
             {"KATZ_XCD_SLAB": "1", "KATZ_SPMM_NWG": "3000"}]
    res = []
    for t, extra in enumerate(walks):
        env = dict(os.environ)
        for k in ("KATZ_XCD_SLAB", "KATZ_SPMM_NWG"):
            env.pop(k, None)
        env.update(extra)
        f = str(tmp_path / ("walk%d.npz" % t))
        print("walk", extra, flush=True)
        subprocess.run([sys.executable, "-c", _WALK_SCRIPT, f, root], env=env, check=True, timeout=300)
        res.append(np.load(f))
    for t in range(1, len(walks)):
        for k in res[0].files:
            assert np.array_equal(res[0][k], res[t][k]), (walks[t], k)


_VROW_SCRIPT = r"""
import sys, numpy as np
sys.path.insert(0, sys.argv[2])
import katz_inputs as ki, paper_1912_06525_amd as K
g = ki.workload("lnsbm4m", scale=0.004).graph
out = {}
for prec, up, rank in ((K.KATZ_PREC_FP64, 3, 16), (K.KATZ_PREC_FP64, 3, 32), (K.KATZ_PREC_MIXED, 0, 8),
                       (K.KATZ_PREC_FP64, 3, 20)):
    idx = K.KatzIndex.from_graph(g, beta_frac=0.9, rank=rank, labels=g.labels, max_block=32, precision=prec,
                                 u_precision=up)
    qs = ki.sample_queries(g, 8, 7 + rank)
    for j, q in enumerate(qs[:6]):
        sc, st = idx.query([q], tol=1e-8)
        out["p%d_r%d_q%d" % (prec, rank, j)] = sc
        out["p%d_r%d_q%d_it" % (prec, rank, j)] = np.array([st[0]["iters"], st[0]["sweeps"]])
    for nb in (2, 3, 8):
        sc, st = idx.query(qs[:nb], tol=1e-8)
        out["p%d_r%d_b%d" % (prec, rank, nb)] = sc
        out["p%d_r%d_b%d_it" % (prec, rank, nb)] = np.array([[x["iters"], x["sweeps"]] for x in st])
    idx.close()
np.savez(sys.argv[1], **out)
"""


def test_row_major_factor_gives_identical_results(tmp_path):
    """Solves of one to eight columns read the BF16 low-rank factor from a
    row-major copy (16-byte row loads) when the rank is 8, 16, 32 or 64; the
    column-major reads (KATZ_VROW=0) take the same values in the same order,
    so scores and iteration counts must be bit-identical.  Rank 20 has no
    row-major copy and checks the fallback.  Each setting runs in a child
    process."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    res = []
    for t, vrow in enumerate(("1", "0")):
        env = dict(os.environ)
        env["KATZ_VROW"] = vrow
        f = str(tmp_path / ("vrow%d.npz" % t))
        print("KATZ_VROW", vrow, flush=True)
        subprocess.run([sys.executable, "-c", _VROW_SCRIPT, f, root], env=env, check=True, timeout=300)
        res.append(np.load(f))
    assert res[0].files == res[1].files
    for k in res[0].files:
        assert np.array_equal(res[0][k], res[1][k]), k


_SPRHS_SCRIPT = r"""
import sys, numpy as np
sys.path.insert(0, sys.argv[2])
import katz_inputs as ki, paper_1912_06525_amd as K
out = {}
cases = []
g = ki.workload("lnsbm4m", scale=0.004).graph
cases.append(("sbm", g, None, g.labels))
cases.append(("sbmw", g, ki.edge_weights(g, seed=3), g.labels))
h = ki.chung_lu(200_000, 2.5, 10, seed=11)
cases.append(("cl", h, None, None))
for name, gr, val, lab in cases:
    deg = np.diff(gr.row_ptr)
    qs = list(ki.sample_queries(gr, 5, 21)) + [int(np.argmax(deg)), int(np.argmin(deg))]
    for prec in (K.KATZ_PREC_FP64, K.KATZ_PREC_MIXED):
        idx = K.KatzIndex.from_graph(gr, val=val, beta_frac=0.9, rank=16, labels=lab, max_block=32, precision=prec)
        for j, q in enumerate(qs):
            sc, st = idx.query([q], tol=1e-9)
            out["%s_p%d_q%d" % (name, prec, j)] = sc[0]
            out["%s_p%d_q%d_st" % (name, prec, j)] = np.array([st[0]["status"], st[0]["iters"], st[0]["sweeps"]])
        idx.close()
np.savez(sys.argv[1], **out)
"""


@pytest.mark.parametrize("switch", ["KATZ_SPARSE_RHS", "KATZ_FUSE"])
def test_one_column_forms_match(tmp_path, switch):
    """Two one-column forms against their plain versions, on community and
    Chung-Lu graphs, unweighted and weighted, FP64 and the precision form,
    including the largest- and smallest-degree nodes.  KATZ_SPARSE_RHS: the
    first sweep's Schur right-hand side from the rows b = beta A e_q reaches
    instead of a block solve and an SpMM over every row.  KATZ_FUSE: the
    residual update, V^T r and the PCG step in one pass and one finalize
    instead of separate passes.  The same status and number of sweeps (a
    wrong right-hand side would be caught by the residual check and cost a
    sweep), iterations within one, scores within rounding of each other."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    res = []
    for t, flag in enumerate(("1", "0")):
        env = dict(os.environ)
        env[switch] = flag
        f = str(tmp_path / ("sw%d.npz" % t))
        print(switch, flag, flush=True)
        subprocess.run([sys.executable, "-c", _SPRHS_SCRIPT, f, root], env=env, check=True, timeout=300)
        res.append(np.load(f))
    assert res[0].files == res[1].files
    for k in res[0].files:
        a, b = res[0][k], res[1][k]
        if k.endswith("_st"):
            assert a[0] == 0 and b[0] == 0 and a[2] == b[2] and abs(int(a[1]) - int(b[1])) <= 1, (k, a, b)
        else:
            tol = 1e-7 if "_p%d_" % K.KATZ_PREC_FP64 in k else 1e-5
            assert np.linalg.norm(a - b) <= tol * np.linalg.norm(b), k



@pytest.mark.parametrize("B", [16, 40, 130])
def test_precision_form_reported_residual_is_true_residual(B):
    """From 16 columns the precision form updates each sweep's FP64 residual
    as r -= M d for the sweep's FP32 correction d instead of forming b - M K
    again.  The relative residual each column reports must be the true one
    of the returned scores (the oracle's b - (I - beta A) k in FP64) up to
    rounding, over two or more sweeps, and the scores must match the
    oracle."""
    g = ki.workload("lnsbm4m", scale=0.004).graph
    A = oracle.csr_matrix(g.n, g.row_ptr, g.col)
    beta = 0.9 / oracle.lambda_max(A)
    idx = K.KatzIndex.from_graph(g, beta=beta, rank=16, labels=g.labels, max_block=32,
                                 precision=K.KATZ_PREC_MIXED)
    qs = ki.sample_queries(g, B, 29 + B)
    tol = 1e-10
    ref = oracle.katz_oracle(g.n, g.row_ptr, g.col, qs, beta=beta, validate=False)["k"]
    for method in (K.KATZ_METHOD_LRC, K.KATZ_METHOD_CG):
        sc, st = idx.query(qs, tol=tol, method=method)
        true = oracle.katz_residual(A, beta, qs, sc.T)
        assert max(x["sweeps"] for x in st) >= 2
        for j in range(B):
            assert st[j]["status"] == 0, st[j]
            assert abs(st[j]["rel_residual"] - true[j]) <= 1e-12 + 1e-3 * true[j], (j, st[j], true[j])
            assert true[j] <= tol * 1.01, (j, true[j])
            c = ref[:, j]
            assert np.linalg.norm(sc[j] - c) <= 1e-8 * np.linalg.norm(c), j
    idx.close()



def test_deferred_x_update_gives_identical_results(tmp_path):
    """From two columns the LRC solve adds alpha p to the solution in the
    search-direction update instead of the residual update (KATZ_DEFER_X);
    the same values are added in the same precision, so scores and
    iteration counts must be bit-identical both ways, in FP64 and in the
    precision form.  Each setting runs in a child process."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    res = []
    for t, flag in enumerate(("1", "0")):
        env = dict(os.environ)
        env["KATZ_DEFER_X"] = flag
        f = str(tmp_path / ("defer%d.npz" % t))
        print("KATZ_DEFER_X", flag, flush=True)
        subprocess.run([sys.executable, "-c", _WALK_SCRIPT, f, root], env=env, check=True, timeout=300)
        res.append(np.load(f))
    for k in res[0].files:
        assert np.array_equal(res[0][k], res[1][k]), k


_CHUNK_SCRIPT = r"""
import sys, numpy as np
sys.path.insert(0, sys.argv[2])
import katz_inputs as ki, paper_1912_06525_amd as K
g = ki.workload("lnsbm4m", scale=0.004).graph
deg = np.diff(g.row_ptr)
qs = list(ki.sample_queries(g, 12, 31)) + [int(np.argmax(deg)), int(np.argmin(deg))]
out = {}
for prec in (K.KATZ_PREC_FP64, K.KATZ_PREC_MIXED):
    idx = K.KatzIndex.from_graph(g, beta_frac=0.9, rank=16, labels=g.labels, max_block=32, precision=prec)
    for m in (K.KATZ_METHOD_LRC, K.KATZ_METHOD_CG):
        for ti, tol in enumerate((1e-6, 1e-9)):
            for j, q in enumerate(qs):
                sc, st = idx.query([q], tol=tol, method=m)
                key = "p%d_m%d_t%d_q%d" % (prec, m, ti, j)
                out[key] = sc[0]
                out[key + "_it"] = np.array([st[0]["status"], st[0]["iters"], st[0]["sweeps"]])
    idx.close()
np.savez(sys.argv[1], **out)
"""


def test_iteration_graphs_give_identical_results(tmp_path):
    """Iteration chunks replayed from captured HIP graphs (one column: every
    chunk length up to 8 captured at a solve kind's first capture) launch the
    same kernels with the same arguments as the eager loop (KATZ_GRAPHS=0):
    one-column scores, statuses, iteration and sweep counts must be
    bit-identical, over consecutive queries whose iteration counts differ (so
    that the adaptive schedule's first chunk changes length), at two
    tolerances, in FP64 and in the precision form.  Each setting runs in a
    child process."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    res = []
    for t, flag in enumerate(("1", "0")):
        env = dict(os.environ)
        env["KATZ_GRAPHS"] = flag
        f = str(tmp_path / ("graphs%d.npz" % t))
        print("KATZ_GRAPHS", flag, flush=True)
        subprocess.run([sys.executable, "-c", _CHUNK_SCRIPT, f, root], env=env, check=True, timeout=300)
        res.append(np.load(f))
    assert res[0].files == res[1].files
    its = set()
    for k in res[0].files:
        assert np.array_equal(res[0][k], res[1][k]), k
        if k.endswith("_it"):
            assert res[0][k][0] == 0, (k, res[0][k])
            its.add(int(res[0][k][1]))
    assert len(its) >= 3, its  # the first chunk's length really varied


@pytest.mark.parametrize("prec", [K.KATZ_PREC_FP64, K.KATZ_PREC_MIXED])
@pytest.mark.parametrize("B", [1, 20])
def test_louvain_partition_matches_oracle(prec, B):
    """An index whose initial parts are katz_communities (Louvain local
    moving capped at max_block) instead of one part cut into BFS chunks:
    blocks with internal edges on a Chung-Lu graph, the same oracle
    parity."""
    g = ki.chung_lu(20_000, 2.5, 10, seed=17)
    beta = oracle_beta(g, 0.9)
    lab, _ = K.katz_communities(g.n, g.row_ptr, g.col, cap=32, passes=8)
    idx = K.KatzIndex.from_graph(g, beta=beta, rank=16, max_block=32, labels=lab, precision=prec)
    assert idx.info.max_block_size > 1
    deg = np.diff(g.row_ptr)
    qs = list(ki.sample_queries(g, B - 1, 5)) + [int(np.argmax(deg))] if B > 1 else [int(np.argmax(deg))]
    _check(g, idx, beta, qs, 1e-8)
    idx.close()


def test_growing_pair_and_topk_requests_on_one_index():
    """Pair and top-K calls of growing and shrinking size on one index: the
    workspace's pair and selection buffers are regrown (the old ones freed)
    between calls, and every call still matches the oracle."""
    g = ki.workload("lnsbm4m", scale=0.002).graph
    beta = oracle_beta(g, 0.6)
    idx = K.KatzIndex.from_graph(g, beta=beta, rank=8, labels=g.labels, max_block=32)
    qs = ki.sample_queries(g, 8, 61)
    ref = oracle.katz_oracle(g.n, g.row_ptr, g.col, qs, beta=beta, validate=False)["k"]
    tau = 1e-8
    tol = tau * (1 - 0.6) / (1 + 0.6)
    rng = np.random.default_rng(9)
    for npairs in (3, 40, 10, 700, 90):
        j = rng.integers(0, len(qs), size=npairs)
        dst = rng.integers(0, g.n, size=npairs).astype(np.int32)
        sc, st = idx.pair_scores(qs[j], dst, tol=tol)
        assert all(s["status"] == 0 for s in st)
        for t in range(npairs):
            k = ref[:, j[t]]
            assert abs(sc[t] - k[dst[t]]) <= tau * np.linalg.norm(k), (npairs, t)
    for K_ in (5, 60, 7, 150, 20):
        ids, scs, st = idx.topk(qs, K_, tol=tol)
        for jj, q in enumerate(qs):
            k = ref[:, jj]
            _, _, sid, ssc = oracle.topk_links(g.n, g.row_ptr, g.col, k, q, K_)
            ok, msg, _ = oracle.topk_accept(ids[jj], sid, ssc, K_, 2 * tau * np.linalg.norm(k))
            assert ok, (K_, msg)
            m = ids[jj] >= 0
            np.testing.assert_allclose(scs[jj][m], k[ids[jj][m]], rtol=0, atol=tau * np.linalg.norm(k))
    idx.close()
