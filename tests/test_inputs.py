"""Seeded input generators: structure, determinism and expected sizes. CPU only."""
import numpy as np
import pytest

import katz_inputs as ki
import oracle


def _check_simple(g):
    oracle.validate_csr(g.n, g.row_ptr, g.col)


def test_sbm_small_shape_and_determinism():
    w = ki.workload("sbm2k")
    g = w.graph
    _check_simple(g)
    assert g.n == 2000
    # E[edges] = 10 * C(200,2) * 0.05 + (C(2000,2) - 10 C(200,2)) * 0.001 = 11750
    m = g.nnz // 2
    assert abs(m - 11750) < 5 * np.sqrt(11750)
    h = ki.workload("sbm2k").graph
    assert np.array_equal(g.col, h.col) and np.array_equal(g.row_ptr, h.row_ptr)
    assert np.array_equal(w.queries, ki.workload("sbm2k").queries)
    assert np.bincount(g.labels).tolist() == [200] * 10


def test_sbm_intra_fraction():
    g = ki.workload("lnsbm4m", scale=0.02).graph
    _check_simple(g)
    rows = np.repeat(np.arange(g.n), g.degrees())
    frac = np.mean(g.labels[rows] == g.labels[g.col])
    assert 0.80 < frac < 0.90
    assert abs(g.degrees().mean() - 16) < 1.0


def test_chung_lu_mean_degree():
    g = ki.chung_lu(20000, 2.5, 20.0, seed=3)
    _check_simple(g)
    d = g.degrees()
    assert abs(d.mean() - 20) < 1.5
    assert d.max() > 5 * d.mean()          # heavy tail


def test_dcsbm_hybrid():
    g = ki.workload("dcsbm16m", scale=0.002).graph
    _check_simple(g)
    rows = np.repeat(np.arange(g.n), g.degrees())
    frac = np.mean(g.labels[rows] == g.labels[g.col])
    assert 0.75 < frac < 0.92


def test_lognormal_sizes_sum():
    s = ki.lognormal_sizes(100, 50000, 400.0, 1.0, seed=9)
    assert s.sum() == 50000 and s.min() >= 2


def test_queries_distinct_nonisolated():
    g = ki.chung_lu(5000, 2.3, 4.0, seed=4)
    q = ki.sample_queries(g, 50, 1)
    assert len(set(q.tolist())) == 50
    assert np.all(g.degrees()[q] >= 1)
