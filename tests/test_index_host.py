"""Host-side index logic through the C ABI with a host-only index (device=-1):
partition validity, Lemma 1 (block elimination is exact), Theorem 1 (spectrum
of S S~^{-1}), lambda_max, error codes, and the exported symbol set.  CPU only:
no GPU compute is called."""
import os
import re

import numpy as np
import pytest
import scipy.linalg as sl

import katz_inputs as ki
import oracle
import paper_1912_06525_amd as K
from conftest import oracle_beta

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_header_symbols_exported():
    src = open(os.path.join(ROOT, "include", "katz.h")).read()
    names = set(re.findall(r"^\s*(?:int|void|const char\*)\s+(katz_\w+)\s*\(", src, re.M))
    assert {"katz_index_build", "katz_query", "katz_topk_links"} <= names
    for nm in names:
        assert hasattr(K._lib, nm), nm
    assert names == set(K.EXPORTED)


def _dense_parts(g, idx, beta, val=None):
    info = idx.info
    perm, bp = idx.partition()
    n, n1 = g.n, info.n1
    A = oracle.csr_matrix(g.n, g.row_ptr, g.col, val).toarray()
    P = np.zeros((n, n))
    P[perm, np.arange(n)] = 1.0          # P @ x puts node v at position perm[v]
    Ap = P @ A @ P.T
    M = np.eye(n) - beta * Ap
    return M, Ap, perm, bp, n1


@pytest.mark.parametrize("labels", [True, False])
def test_partition_is_block_diagonal(labels):
    g = ki.workload("sbm2k").graph
    idx = K.KatzIndex.from_graph(g, beta_frac=0.5, rank=0, device=-1, max_block=48,
                                 labels=g.labels if labels else None)
    info = idx.info
    perm, bp = idx.partition()
    assert sorted(perm.tolist()) == list(range(g.n))
    assert bp[0] == 0 and bp[-1] == info.n1 and np.all(np.diff(bp) >= 1)
    assert np.diff(bp).max() <= 48
    blk = np.full(g.n, -1)
    for b in range(len(bp) - 1):
        blk[bp[b]:bp[b + 1]] = b
    rows = np.repeat(np.arange(g.n), g.degrees())
    pu, pv = perm[rows], perm[g.col]
    interior = (pu < info.n1) & (pv < info.n1)
    assert np.all(blk[pu[interior]] == blk[pv[interior]])   # no edges between blocks
    assert info.n1 + info.n2 == g.n


@pytest.mark.parametrize("weighted", [False, True])
def test_lemma1_block_elimination_exact(weighted):
    g = ki.workload("sbm2k", scale=0.4).graph
    val = ki.edge_weights(g, seed=13) if weighted else None
    beta = 0.7 / oracle.lambda_max(oracle.csr_matrix(g.n, g.row_ptr, g.col, val))
    idx = K.KatzIndex.from_graph(g, val=val, beta=beta, rank=0, device=-1, labels=g.labels, max_block=64)
    M, Ap, perm, bp, n1 = _dense_parts(g, idx, beta, val)
    qs = ki.sample_queries(g, 3, 17)
    ref = oracle.katz_oracle(g.n, g.row_ptr, g.col, qs, beta=beta, val=val)["k_direct"]
    M11, M12, M22 = M[:n1, :n1], M[:n1, n1:], M[n1:, n1:]
    for i, q in enumerate(qs):
        b = beta * Ap[:, perm[q]]
        b1, b2 = b[:n1], b[n1:]
        S = M22 - M12.T @ np.linalg.solve(M11, M12)
        k2 = np.linalg.solve(S, b2 - M12.T @ np.linalg.solve(M11, b1))      # eq. (5)
        k1 = np.linalg.solve(M11, b1 - M12 @ k2)                             # eq. (6)
        k = np.concatenate([k1, k2])[perm]
        np.testing.assert_allclose(k, ref[:, i], rtol=1e-11, atol=1e-14)


def test_star_centre_is_the_separator():
    m = 7
    g = ki.from_edges(m + 1, [(0, i) for i in range(1, m + 1)])
    labels = np.arange(m + 1, dtype=np.int32)
    beta = 0.6 / np.sqrt(m)  # lambda_max of the star is sqrt(m)
    idx = K.KatzIndex.from_graph(g, beta=beta, rank=1, device=-1, labels=labels, l_kind=K.KATZ_L_CHOL)
    info = idx.info
    assert info.n2 == 1 and info.n1 == m
    perm, _ = idx.partition()
    assert perm[0] == m                     # centre placed last
    # S = 1 - m beta^2 (scalar); with L = chol(M22) = 1, R = m beta^2
    U, s = idx.lowrank()
    assert abs(s[0] - m * beta ** 2) < 1e-14


def _ic0(A):
    """Zero-fill incomplete Cholesky of the dense SPD M-matrix A, written out
    for the test: L keeps the pattern of A's lower triangle and L L^T equals
    A on that pattern and the diagonal (the defining property, asserted)."""
    n = len(A)
    pat = np.tril(A, -1) != 0
    L = np.zeros_like(A)
    for i in range(n):
        for k in range(i):
            if pat[i, k]:
                L[i, k] = (A[i, k] - L[i, :k] @ L[k, :k]) / L[k, k]
        L[i, i] = np.sqrt(A[i, i] - L[i, :i] @ L[i, :i])
    P = L @ L.T
    on = pat | pat.T | np.eye(n, dtype=bool)
    np.testing.assert_allclose(P[on], A[on], rtol=0, atol=1e-13)
    assert np.all(L[np.triu(np.ones((n, n), bool), 1)] == 0) and np.all(L[np.tril(~pat, -1)] == 0)
    return L


def _factor(lkind, M22):
    if lkind == K.KATZ_L_CHOL:
        return np.linalg.cholesky(M22)
    if lkind == K.KATZ_L_IC0:
        return _ic0(M22)
    return np.eye(len(M22))


@pytest.mark.parametrize("lkind", [K.KATZ_L_CHOL, K.KATZ_L_IDENTITY, K.KATZ_L_IC0])
def test_theorem1_spectrum(lkind):
    g = ki.sbm([12, 10, 14], [0.5, 0.5, 0.5], 0.08, seed=5)
    r = 3
    beta = oracle_beta(g, 0.8)
    idx = K.KatzIndex.from_graph(g, beta=beta, rank=r, device=-1, labels=g.labels, max_block=8,
                                 l_kind=lkind, lanczos_steps=10 ** 6)
    M, Ap, perm, bp, n1 = _dense_parts(g, idx, beta)
    n2 = idx.info.n2
    assert n2 >= r + 2
    M11, M12, M22 = M[:n1, :n1], M[:n1, n1:], M[n1:, n1:]
    S = M22 - M12.T @ np.linalg.solve(M11, M12)
    L = _factor(lkind, M22)
    Li = np.linalg.inv(L)
    R = np.eye(n2) - Li @ S @ Li.T
    sig_all = np.sort(np.linalg.eigvalsh(R))[::-1]
    U, s = idx.lowrank()
    np.testing.assert_allclose(s, sig_all[:r], rtol=0, atol=1e-10)
    assert np.all(sig_all < 1)                              # S is SPD
    if lkind == K.KATZ_L_CHOL:
        assert np.all(sig_all > -1e-12)                     # R is PSD for L = chol(M22)
    Dg = np.diag(s / (1 - s))
    St_inv = Li.T @ (np.eye(n2) + U @ Dg @ U.T) @ Li       # eq. inverseTildeS
    ev = np.sort(np.linalg.eigvals(S @ St_inv).real)
    expect = np.sort(np.concatenate([np.ones(r), 1 - sig_all[r:]]))
    np.testing.assert_allclose(ev, expect, atol=1e-9)


@pytest.mark.parametrize("lkind", [K.KATZ_L_CHOL, K.KATZ_L_IDENTITY, K.KATZ_L_IC0])
def test_theorem1_spectrum_weighted(lkind):
    # Theorem 1 on a weighted adjacency: the index's Ritz values are the top of
    # the dense spectrum of R, and the preconditioned Schur complement has
    # eigenvalues 1 (r times) and 1 - sigma_i for the rest
    g = ki.sbm([12, 10, 14], [0.5, 0.5, 0.5], 0.08, seed=6)
    val = ki.edge_weights(g, seed=21)
    r = 3
    beta = 0.8 / oracle.lambda_max(oracle.csr_matrix(g.n, g.row_ptr, g.col, val))
    idx = K.KatzIndex.from_graph(g, val=val, beta=beta, rank=r, device=-1, labels=g.labels, max_block=8,
                                 l_kind=lkind, lanczos_steps=10 ** 6)
    M, Ap, perm, bp, n1 = _dense_parts(g, idx, beta, val)
    n2 = idx.info.n2
    assert n2 >= r + 2
    M11, M12, M22 = M[:n1, :n1], M[:n1, n1:], M[n1:, n1:]
    S = M22 - M12.T @ np.linalg.solve(M11, M12)
    L = _factor(lkind, M22)
    Li = np.linalg.inv(L)
    R = np.eye(n2) - Li @ S @ Li.T
    sig_all = np.sort(np.linalg.eigvalsh(R))[::-1]
    U, s = idx.lowrank()
    np.testing.assert_allclose(s, sig_all[:r], rtol=0, atol=1e-10)
    Dg = np.diag(s / (1 - s))
    ev = np.sort(np.linalg.eigvals(S @ (Li.T @ (np.eye(n2) + U @ Dg @ U.T) @ Li)).real)
    expect = np.sort(np.concatenate([np.ones(r), 1 - sig_all[r:]]))
    np.testing.assert_allclose(ev, expect, atol=1e-9)


def test_lambda_and_beta():
    g = ki.chung_lu(3000, 2.5, 8.0, seed=2)
    idx = K.KatzIndex.from_graph(g, beta_frac=0.9, rank=0, device=-1)
    lam = oracle.lambda_max(oracle.csr_matrix(g.n, g.row_ptr, g.col))
    assert abs(idx.info.lambda_max - lam) <= 1e-10 * lam
    assert abs(idx.info.c - 0.9) < 1e-12


def test_error_codes():
    g = ki.from_edges(3, [(0, 1), (1, 2)])
    with pytest.raises(K.KatzError) as e:
        K.KatzIndex.from_graph(g, beta_frac=1.0, device=-1)
    assert e.value.code == K.KATZ_EDIVERGE
    with pytest.raises(K.KatzError) as e:
        K.KatzIndex(2, [0, 1, 1], [1], beta=0.1, device=-1)
    assert e.value.code == K.KATZ_ENOTSYM
    # an entry below the diagonal only, a triangle with one direction missing,
    # and a weighted pair whose two values differ
    for n_, rp_, col_, val_ in ((2, [0, 0, 1], [0], None),
                                (3, [0, 2, 3, 4], [1, 2, 0, 1], None),
                                (2, [0, 1, 2], [1, 0], [1.0, 2.0])):
        with pytest.raises(K.KatzError) as e:
            K.KatzIndex(n_, rp_, col_, val_, beta=0.1, device=-1)
        assert e.value.code == K.KATZ_ENOTSYM, (rp_, col_)
    with pytest.raises(K.KatzError) as e:
        K.KatzIndex(2, [0, 2, 2], [0, 1], beta=0.1, device=-1)
    assert e.value.code == K.KATZ_EINVAL
    with pytest.raises(K.KatzError) as e:
        K.KatzIndex(3, [0, 2, 3, 4], [2, 1, 0, 0], beta=0.1, device=-1)
    assert e.value.code == K.KATZ_EINVAL
    # a row pointer past the entries with a smaller one after it: rejected by
    # the row-pointer pass before any row (or symmetric partner) is read
    with pytest.raises(K.KatzError) as e:
        K.KatzIndex(8, [0, 1, 2, 3, 4, 5, 6, 14, 12], [6, 6, 6, 6, 6, 6, 0, 1, 2, 3, 4, 5], beta=0.1,
                    device=-1)
    assert e.value.code == K.KATZ_EINVAL
    idx = K.KatzIndex.from_graph(g, beta_frac=0.5, device=-1, rank=0)
    with pytest.raises(K.KatzError) as e:
        idx.query([0])
    assert e.value.code == K.KATZ_EDEVICE
    with pytest.raises(K.KatzError) as e:
        idx.query([7])
    assert e.value.code == K.KATZ_EINVAL


# ------------------------------------------------------------ index files
def _info_tuple(info):
    return (info.n, info.n1, info.n2, info.nnz, info.nblocks, info.max_block_size, info.rank, info.l_kind,
            info.precision, info.beta, info.lambda_max, info.c, info.sigma_max, info.sigma_next, info.u_precision)


@pytest.mark.parametrize("c,req", [(0.5, 0), (0.995, 0), (0.5, 2), (0.995, 3), (0.5, 1)])
def test_lowrank_storage_resolution(c, req):
    # auto (0): BF16 (3) when every weight sigma / (1 - sigma) <= 16, else
    # FP32 (2); an explicit request is kept as given
    g = ki.chung_lu(3000, 2.5, 8.0, seed=4)
    idx = K.KatzIndex.from_graph(g, beta=oracle_beta(g, c), rank=6, device=-1, u_precision=req)
    _, s = idx.lowrank()
    dmax = np.max(np.abs(s / (1 - s)))
    if req:
        assert idx.info.u_precision == req
    else:
        assert idx.info.u_precision == (3 if dmax <= 16 else 2), (dmax, idx.info.u_precision)
    if c > 0.99:
        assert dmax > 16   # the case exercises the FP32 branch


def test_index_file_round_trip(tmp_path):
    g = ki.workload("sbm2k", scale=0.5).graph
    for lk in (K.KATZ_L_CHOL, K.KATZ_L_IDENTITY):
        a = K.KatzIndex.from_graph(g, beta=oracle_beta(g, 0.6), rank=6, device=-1, labels=g.labels,
                                   max_block=40, l_kind=lk)
        p = str(tmp_path / ("idx%d.katz" % lk))
        a.save(p)
        b = K.KatzIndex.load(p, device=-1)
        assert _info_tuple(a.info) == _info_tuple(b.info)
        pa, ba = a.partition()
        pb, bb = b.partition()
        assert np.array_equal(pa, pb) and np.array_equal(ba, bb)
        ua, sa = a.lowrank()
        ub, sb = b.lowrank()
        assert np.array_equal(ua, ub) and np.array_equal(sa, sb)


@pytest.mark.parametrize("prec,uprec", [(K.KATZ_PREC_FP64, 1), (K.KATZ_PREC_FP64, 2), (K.KATZ_PREC_MIXED, 0)])
def test_weighted_index_file_round_trip(tmp_path, prec, uprec):
    # weighted adjacency, both precisions and explicit storage of V: the file
    # keeps the weights and every option; one weight changed in the file
    # breaks symmetry and is rejected
    g = ki.workload("sbm2k", scale=0.4).graph
    val = ki.edge_weights(g, seed=9)
    A = oracle.csr_matrix(g.n, g.row_ptr, g.col, val)
    beta = 0.6 / oracle.lambda_max(A)
    a = K.KatzIndex.from_graph(g, val=val, beta=beta, rank=5, device=-1, max_block=32, precision=prec,
                               u_precision=uprec)
    p = tmp_path / "w.katz"
    a.save(str(p))
    b = K.KatzIndex.load(str(p), device=-1)
    assert _info_tuple(a.info) == _info_tuple(b.info)
    assert b.info.precision == prec and (uprec == 0 or b.info.u_precision == uprec)
    raw = bytearray(p.read_bytes())
    at, cnt = _index_arrays(raw)["val"]
    assert cnt == len(val)
    # the stored weights are the caller's, in the permuted CSR order
    stored = np.frombuffer(bytes(raw[at:at + 8 * cnt]), dtype="<f8")
    assert np.array_equal(np.sort(stored), np.sort(val))
    bad = bytearray(raw)
    w0 = np.frombuffer(bytes(bad[at:at + 8]), dtype="<f8")[0]
    bad[at:at + 8] = np.array([w0 * 1.5], dtype="<f8").tobytes()
    q = tmp_path / "w_bad.katz"
    q.write_bytes(bytes(bad))
    with pytest.raises(K.KatzError) as e:
        K.KatzIndex.load(str(q), device=-1)
    assert e.value.code == K.KATZ_EINVAL


def test_index_file_rejects_damage(tmp_path):
    g = ki.workload("sbm2k", scale=0.3).graph
    a = K.KatzIndex.from_graph(g, beta=oracle_beta(g, 0.5), rank=2, device=-1, max_block=32)
    p = tmp_path / "good.katz"
    a.save(str(p))
    raw = bytearray(p.read_bytes())
    n = a.info.n

    def load_code(data, name):
        q = tmp_path / name
        q.write_bytes(bytes(data))
        with pytest.raises(K.KatzError) as e:
            K.KatzIndex.load(str(q), device=-1)
        return e.value.code

    with pytest.raises(K.KatzError) as e:
        K.KatzIndex.load(str(tmp_path / "missing.katz"), device=-1)
    assert e.value.code == K.KATZ_EIO
    bad = bytearray(raw)
    bad[0] = ord("X")
    assert load_code(bad, "magic.katz") == K.KATZ_EINVAL
    assert load_code(raw[: len(raw) // 2], "short.katz") == K.KATZ_EIO
    # header: magic 8, version 4, tag 4, then 84 bytes of scalars; perm's
    # element count (u64) at 100, its elements from 108
    perm0 = int.from_bytes(raw[108:112], "little")
    bad = bytearray(raw)
    bad[108:112] = raw[112:116]                       # perm[0] = perm[1]: not a permutation
    assert perm0 != int.from_bytes(raw[112:116], "little")
    assert load_code(bad, "perm.katz") == K.KATZ_EINVAL
    # the first column index: after perm, iperm (n each), rp (n + 1), col's count
    off = 108 + 4 * n + 8 + 4 * n + 8 + 4 * (n + 1) + 8
    bad = bytearray(raw)
    bad[off:off + 4] = (n + 5).to_bytes(4, "little")  # column out of range
    assert load_code(bad, "col.katz") == K.KATZ_EINVAL
    # row pointers out of order: one past the entries with the last in place
    # (must be rejected before any row is read through it)
    arr = _index_arrays(raw)
    rp_at, nb1 = arr["rp"][0], arr["blk_start"][1]
    bad = bytearray(raw)
    nnz = int.from_bytes(raw[rp_at + 4 * n:rp_at + 4 * n + 4], "little")
    bad[rp_at + 4 * (n - 1):rp_at + 4 * n] = (nnz + 5).to_bytes(4, "little")
    assert load_code(bad, "rowptr.katz") == K.KATZ_EINVAL
    # a block start past the last block's end (block sizes must be checked
    # before any block's rows are read)
    bs_at = arr["blk_start"][0]
    n1 = int.from_bytes(raw[bs_at + 4 * (nb1 - 1):bs_at + 4 * nb1], "little")
    bad = bytearray(raw)
    bad[bs_at + 4 * (nb1 - 2):bs_at + 4 * (nb1 - 1)] = (n1 + 3).to_bytes(4, "little")
    assert load_code(bad, "blkstart.katz") == K.KATZ_EINVAL
    # a good file still loads after all this
    b = K.KatzIndex.load(str(p), device=-1)
    assert b.info.n == n


def _index_arrays(raw):
    """name -> (offset of the first element, element count) of every array of
    an index file: 100 header bytes, then each array as a u64 count and its
    elements, in the order the writer puts them."""
    order = [("perm", 4), ("iperm", 4), ("rp", 4), ("col", 4), ("split", 4), ("val", 8),
             ("blk_start", 4), ("blk_off", 8), ("minv", 8), ("ginv", 8), ("lchol", 8),
             ("U", 8), ("V", 8), ("sigma", 8), ("D", 8)]
    out, at = {}, 100
    for name, esz in order:
        cnt = int.from_bytes(raw[at:at + 8], "little")
        out[name] = (at + 8, cnt)
        at += 8 + esz * cnt
    assert at == len(raw)
    return out


def test_query_option_defaults():
    # documented defaults of katz_query_opts (the adaptive polling schedule
    # is check_every = 0)
    o = K.katz_query_opts_default()
    assert o.rel_tol == 1e-6 and o.max_iter == 1000 and o.max_sweeps == 6
    assert o.check_every == 0 and o.force_fallback == 0


def test_build_phase_times():
    """katz_index_info_t reports the build's wall time per phase: every phase
    is nonnegative, a host-only build has no upload, and the phases account
    for the build time."""
    g = ki.workload("lnsbm4m", scale=0.01).graph
    idx = K.KatzIndex.from_graph(g, beta_frac=0.5, rank=8, max_block=32, device=-1, labels=g.labels)
    ph = list(idx.info.build_phase_seconds)
    assert len(ph) == 12 and all(x >= 0 for x in ph)
    assert ph[11] == 0.0
    assert ph[2] > 0 and ph[10] > 0            # partition and the host Lanczos ran
    assert sum(ph) <= idx.info.build_seconds * 1.01 + 1e-3
    assert sum(ph) >= 0.5 * idx.info.build_seconds


# ------------------------------------------------------------ communities
def _modularity(n, rp, col, lab, val=None):
    """Newman-Girvan modularity of the labelling, from its definition:
    sum over C of [w_in(C) / 2m - (tot(C) / 2m)^2], w_in counting both
    directions of every edge inside C."""
    rp = np.asarray(rp)
    col = np.asarray(col)
    w = np.ones(len(col)) if val is None else np.asarray(val, float)
    row = np.repeat(np.arange(n), np.diff(rp))
    k = np.bincount(row, weights=w, minlength=n)
    m2 = k.sum()
    inside = w[lab[row] == lab[col]].sum()
    tot = np.bincount(lab, weights=k)
    return inside / m2 - (tot ** 2).sum() / m2 ** 2


def _random_graph(n, p, seed, weighted):
    rng = np.random.default_rng(seed)
    edges = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p]
    g = ki.from_edges(n, edges)
    val = None
    if weighted:
        # one edge in eight of weight zero (allowed: weights are nonnegative)
        wt = {e: float(rng.uniform(0.2, 3.0)) if rng.random() < 0.875 else 0.0 for e in edges}
        rows = np.repeat(np.arange(n), g.degrees())
        val = np.array([wt[(min(a, b), max(a, b))] for a, b in zip(rows, g.col)])
    return g, val


def test_communities_recover_planted_sbm():
    """40 planted communities of 30 nodes (p_in 0.5, p_out 0.002): local
    moving finds them (adjusted Rand index above 0.95) and their modularity
    to within 0.02."""
    from sklearn.metrics import adjusted_rand_score
    g = ki.sbm([30] * 40, 0.5, 0.002, seed=3)
    lab, passes = K.katz_communities(g.n, g.row_ptr, g.col, cap=64, passes=20)
    assert adjusted_rand_score(g.labels, lab) > 0.95
    assert 1 <= passes < 20
    q_found = _modularity(g.n, g.row_ptr, g.col, lab)
    q_planted = _modularity(g.n, g.row_ptr, g.col, np.asarray(g.labels))
    assert q_found > q_planted - 0.02


def test_communities_closed_cases():
    """Two disjoint 10-cliques: two communities (cap 10); cap 5 splits each
    clique into parts of at most 5; passes = 0 leaves every node alone;
    isolated nodes stay alone."""
    edges = [(i, j) for base in (0, 10) for i in range(base, base + 10) for j in range(i + 1, base + 10)]
    g = ki.from_edges(22, edges)  # nodes 20 and 21 isolated
    lab, _ = K.katz_communities(g.n, g.row_ptr, g.col, cap=10, passes=10)
    assert lab.tolist() == [0] * 10 + [1] * 10 + [2, 3]
    lab5, _ = K.katz_communities(g.n, g.row_ptr, g.col, cap=5, passes=10)
    assert np.bincount(lab5).max() <= 5
    for c in np.unique(lab5):  # no community spans the two cliques
        members = np.flatnonzero(lab5 == c)
        assert len({int(v) // 10 for v in members if v < 20}) <= 1
    lab0, p0 = K.katz_communities(g.n, g.row_ptr, g.col, cap=10, passes=0)
    assert lab0.tolist() == list(range(22)) and p0 == 0


def test_communities_numbered_in_breadth_first_order():
    """Community ids follow the order in which a breadth-first search (from
    node 0, neighbours in row order, restarting at the smallest unreached
    node) first reaches each community; the ids are 0 .. ncomm - 1."""
    from collections import deque
    g = ki.chung_lu(3000, 2.5, 4, seed=9)  # several components
    lab, _ = K.katz_communities(g.n, g.row_ptr, g.col, cap=16, passes=6)
    seen = np.zeros(g.n, bool)
    order = []
    for s0 in range(g.n):
        if seen[s0]:
            continue
        seen[s0] = True
        dq = deque([s0])
        while dq:
            u = dq.popleft()
            order.append(u)
            for v in g.col[g.row_ptr[u]:g.row_ptr[u + 1]]:
                if not seen[v]:
                    seen[v] = True
                    dq.append(v)
    firsts = []
    for u in order:
        if lab[u] not in firsts:
            firsts.append(int(lab[u]))
    assert firsts == list(range(int(lab.max()) + 1))


@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("cap", [4, 1000])
def test_communities_local_optimum_by_brute_force(weighted, cap):
    """Run to convergence, the labelling is a local optimum of the true
    modularity (computed from its definition): no single node moves to a
    neighbouring community with room for a gain above rounding.  Modularity never falls from one pass to the next, and two
    calls give the same labels."""
    g, val = _random_graph(60, 0.12, seed=5 + cap, weighted=weighted)
    lab, passes = K.katz_communities(g.n, g.row_ptr, g.col, val, cap=cap, passes=100)
    assert passes < 100
    lab2, _ = K.katz_communities(g.n, g.row_ptr, g.col, val, cap=cap, passes=100)
    assert np.array_equal(lab, lab2)
    assert np.bincount(lab).max() <= cap
    q = _modularity(g.n, g.row_ptr, g.col, lab, val)
    for v in range(g.n):
        nb = g.col[g.row_ptr[v]:g.row_ptr[v + 1]]
        for c in set(lab[nb].tolist()):
            if c == lab[v] or np.sum(lab == c) >= cap:
                continue
            t = lab.copy()
            t[v] = c
            assert _modularity(g.n, g.row_ptr, g.col, t, val) <= q + 1e-12, (v, c)
    qs = [_modularity(g.n, g.row_ptr, g.col, K.katz_communities(g.n, g.row_ptr, g.col, val, cap=cap,
                                                                 passes=p)[0], val) for p in range(passes + 1)]
    assert all(b >= a - 1e-12 for a, b in zip(qs, qs[1:])), qs
    assert qs[-1] > qs[0]


def test_communities_as_partition_labels():
    """Communities feed the build as labels: the partition stays block
    diagonal with blocks within max_block."""
    g = ki.chung_lu(5000, 2.5, 10, seed=4)
    lab, _ = K.katz_communities(g.n, g.row_ptr, g.col, cap=32, passes=8)
    idx = K.KatzIndex.from_graph(g, beta_frac=0.5, rank=0, device=-1, max_block=32, labels=lab)
    info = idx.info
    perm, bp = idx.partition()
    assert np.diff(bp).max() <= 32 and info.n1 + info.n2 == g.n
    blk = np.full(g.n, -1)
    for b in range(len(bp) - 1):
        blk[bp[b]:bp[b + 1]] = b
    rows = np.repeat(np.arange(g.n), g.degrees())
    pu, pv = perm[rows], perm[g.col]
    interior = (pu < info.n1) & (pv < info.n1)
    assert np.all(blk[pu[interior]] == blk[pv[interior]])
    idx.close()


def test_communities_errors():
    g = ki.from_edges(3, [(0, 1), (1, 2)])
    for cap, passes in ((0, 4), (4, -1)):
        with pytest.raises(K.KatzError) as e:
            K.katz_communities(g.n, g.row_ptr, g.col, cap=cap, passes=passes)
        assert e.value.code == K.KATZ_EINVAL
    with pytest.raises(K.KatzError) as e:
        K.katz_communities(2, [0, 1, 1], [1])
    assert e.value.code == K.KATZ_ENOTSYM


# ------------------------------------------------------------ rebuild for other options
def _file_bytes(idx, path):
    """The index file without its build-time field (bytes 92..100)."""
    idx.save(path)
    b = bytearray(open(path, "rb").read())
    b[92:100] = b"\0" * 8
    return bytes(b)


_REBUILD_CASES = [
    # (graph, weighted, partition options, source options, target options)
    ("sbm2k", False, dict(labels=True, max_block=200), dict(beta_frac=0.3, rank=4),
     dict(beta_frac=0.8, rank=8, l_kind=K.KATZ_L_CHOL)),
    ("sbm2k", False, dict(labels=True, max_block=200), dict(beta_frac=0.5, rank=8, l_kind=K.KATZ_L_CHOL),
     dict(beta_frac=0.95, rank=8, l_kind=K.KATZ_L_IC0)),
    ("cl", False, dict(), dict(beta_frac=0.5, rank=16), dict(beta_frac=0.9, rank=24)),
    ("cl", True, dict(order=K.KATZ_ORDER_DEGREE), dict(beta_frac=0.5, rank=16),
     dict(beta_frac=0.7, rank=32, precision=K.KATZ_PREC_MIXED)),
    ("cl", False, dict(), dict(beta_frac=0.2, rank=0), dict(beta=0.005, rank=5, u_precision=1, lanczos_steps=40)),
]


@pytest.mark.parametrize("case", range(len(_REBUILD_CASES)))
def test_rebuild_equals_a_fresh_build(case, tmp_path):
    """katz_index_rebuild reuses the graph's checks, lambda_max, partition and
    order and recomputes the beta-dependent factors: its index file equals a
    fresh build's with the target options byte for byte (build time aside),
    also from a loaded source, and the source is left unchanged."""
    gname, weighted, popt, sopt, topt = _REBUILD_CASES[case]
    g = ki.workload("sbm2k").graph if gname == "sbm2k" else ki.chung_lu(20000, 2.5, 8, seed=7)
    val = ki.edge_weights(g, seed=2) if weighted else None
    part = dict(popt)
    if part.pop("labels", False):
        part["labels"] = g.labels
    src = K.KatzIndex(g.n, g.row_ptr, g.col, val, device=-1, **part, **sopt)
    before = _file_bytes(src, str(tmp_path / "src.katz"))
    fresh = K.KatzIndex(g.n, g.row_ptr, g.col, val, device=-1, **part, **topt)
    want = _file_bytes(fresh, str(tmp_path / "fresh.katz"))
    re = src.rebuild(device=-1, **topt)
    assert _file_bytes(re, str(tmp_path / "re.katz")) == want
    assert _file_bytes(src, str(tmp_path / "src2.katz")) == before
    ph = list(re.info.build_phase_seconds)
    assert ph[:8] == [0.0] * 8 and ph[8] >= 0.0
    loaded = K.KatzIndex.load(str(tmp_path / "src.katz"), device=-1)
    re2 = loaded.rebuild(device=-1, **topt)
    assert _file_bytes(re2, str(tmp_path / "re2.katz")) == want
    for x in (src, fresh, re, loaded, re2):
        x.close()


def test_rebuild_errors():
    g = ki.workload("sbm2k").graph
    src = K.KatzIndex.from_graph(g, beta_frac=0.5, rank=4, device=-1, labels=g.labels, max_block=200)
    for kw, code in ((dict(beta_frac=1.0), K.KATZ_EDIVERGE), (dict(beta=1.0), K.KATZ_EDIVERGE),
                     (dict(rank=-1), K.KATZ_EINVAL), (dict(u_precision=5), K.KATZ_EINVAL),
                     (dict(l_kind=9), K.KATZ_EINVAL), (dict(precision=4), K.KATZ_EINVAL)):
        with pytest.raises(K.KatzError) as e:
            src.rebuild(device=-1, **kw)
        assert e.value.code == code, kw
    import ctypes
    h = ctypes.c_void_p()
    assert K._lib.katz_index_rebuild(None, None, ctypes.byref(h)) == K.KATZ_EINVAL
    assert K._lib.katz_index_rebuild(src.h, None, None) == K.KATZ_EINVAL
    # the source still answers host-side calls
    assert src.info.rank == 4
    src.close()
