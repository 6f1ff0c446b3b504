"""Precision form (FP32 inner solves, BF16 low-rank factor, FP64 dots and FP64
residual refinement) against the CPU FP64 oracle.  GPU only.

The refinement sweeps make the returned k meet the requested FP64 residual
whatever the inner precision, so the acceptance is the FP64 path's:
||k^ - k|| <= tau ||k|| with the residual requested as tau (1-c)/(1+c)."""
import numpy as np
import pytest

import katz_inputs as ki
import oracle
from conftest import oracle_beta

pytestmark = pytest.mark.gpu
K = pytest.importorskip("paper_1912_06525_amd")


def _run(g, idx, beta, qs, tau, method=K.KATZ_METHOD_LRC):
    # beta: the test's own value, given to the index build and to the oracle
    c = idx.info.c
    tol = tau * (1 - c) / (1 + c)
    sc, st = idx.query(qs, tol=tol, method=method)
    ref = oracle.katz_oracle(g.n, g.row_ptr, g.col, qs, beta=beta, validate=False)
    for j in range(len(qs)):
        k = ref["k"][:, j]
        assert st[j]["status"] == 0 and st[j]["rel_residual"] <= tol, st[j]
        err = np.linalg.norm(sc[j] - k)
        assert err <= tau * np.linalg.norm(k), err / np.linalg.norm(k)
    return st


@pytest.mark.parametrize("c", [0.5, 0.9])
@pytest.mark.parametrize("method", [K.KATZ_METHOD_LRC, K.KATZ_METHOD_CG])
def test_mixed_small_sbm(c, method):
    g = ki.workload("lnsbm4m", scale=0.002).graph
    beta = oracle_beta(g, c)
    idx = K.KatzIndex.from_graph(g, beta=beta, rank=16, labels=g.labels, max_block=32,
                                 precision=K.KATZ_PREC_MIXED)
    qs = ki.sample_queries(g, 6, 71)
    st = _run(g, idx, beta, qs, 1e-6, method)
    assert all(s["sweeps"] >= 2 for s in st)          # FP32 inner solve, FP64 refinement


def test_mixed_chung_lu_batch():
    g = ki.chung_lu(30000, 2.3, 12.0, seed=1004)
    beta = oracle_beta(g, 0.9)
    idx = K.KatzIndex.from_graph(g, beta=beta, rank=32, precision=K.KATZ_PREC_MIXED)
    qs = ki.sample_queries(g, 20, 5)
    _run(g, idx, beta, qs, 1e-6)


def test_mixed_matches_fp64_path():
    g = ki.workload("sbm2k").graph
    qs = ki.sample_queries(g, 5, 9)
    a = K.KatzIndex.from_graph(g, beta_frac=0.5, rank=8, labels=g.labels, precision=K.KATZ_PREC_MIXED)
    b = K.KatzIndex.from_graph(g, beta_frac=0.5, rank=8, labels=g.labels)
    sa, _ = a.query(qs, tol=1e-10)
    sb, _ = b.query(qs, tol=1e-10)
    for j in range(len(qs)):
        assert np.linalg.norm(sa[j] - sb[j]) <= 1e-9 * np.linalg.norm(sb[j])


@pytest.mark.parametrize("B,rank", [(16, 32), (100, 70), (64, 8)])
def test_mixed_batched_mfma_preconditioner(B, rank):
    # B >= 16 FP32 panels take the bf16 MFMA low-rank kernels (ragged B and rank)
    g = ki.chung_lu(20000, 2.3, 12.0, seed=11)
    beta = oracle_beta(g, 0.9)
    idx = K.KatzIndex.from_graph(g, beta=beta, rank=rank, precision=K.KATZ_PREC_MIXED)
    qs = ki.sample_queries(g, B, 3)
    st = _run(g, idx, beta, qs, 1e-6)
    # same queries one at a time (scalar kernels) agree within the tolerance
    one, _ = idx.query(qs[:2], tol=1e-8)
    ref = oracle.katz_oracle(g.n, g.row_ptr, g.col, qs[:2], beta=beta)
    for j in range(2):
        assert np.linalg.norm(one[j] - ref["k"][:, j]) <= 1e-6 * np.linalg.norm(ref["k"][:, j])


def test_mixed_preconditioner_effective():
    # the MFMA preconditioner must actually precondition: fewer inner
    # iterations than with rank 0 on a graph whose top eigenvalues dominate
    g = ki.chung_lu(20000, 2.3, 12.0, seed=12)
    qs = ki.sample_queries(g, 32, 7)
    its = {}
    for rank in (0, 32):
        idx = K.KatzIndex.from_graph(g, beta_frac=0.99, rank=rank, precision=K.KATZ_PREC_MIXED)
        _, st = idx.query(qs, tol=1e-6)
        assert all(s["status"] == 0 for s in st)
        its[rank] = np.mean([s["iters"] for s in st])
    assert its[32] < its[0], its
