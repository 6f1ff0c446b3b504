"""Serving form: continuous batching of top-K requests over worker slots.
GPU only.  Checks every request against the oracle's ranking (tie rule), a
request's result alone vs inside a mix of concurrent requests, request
splitting across workers, and admission by the HBM budget."""
import threading
import time

import numpy as np
import pytest

import katz_inputs as ki
import oracle
from conftest import oracle_beta

pytestmark = pytest.mark.gpu
K = pytest.importorskip("paper_1912_06525_amd")

TAU = 1e-8


@pytest.fixture(scope="module")
def setup():
    g = ki.workload("dcsbm16m", scale=0.002).graph
    beta = oracle_beta(g, 0.5)
    idx = K.KatzIndex.from_graph(g, beta=beta, rank=16, labels=g.labels)
    return g, idx, beta


def _tol(idx):
    return TAU * (1 - idx.info.c) / (1 + idx.info.c)


def _check_against_oracle(g, beta, qs, ids, k):
    ref = oracle.katz_oracle(g.n, g.row_ptr, g.col, qs, beta=beta, validate=False)
    for j, q in enumerate(qs):
        kv = ref["k"][:, j]
        _, _, sid, ssc = oracle.topk_links(g.n, g.row_ptr, g.col, kv, q, k)
        ok, msg, _ = oracle.topk_accept(ids[j], sid, ssc, k, 2 * TAU * np.linalg.norm(kv))
        assert ok, msg


def test_server_alone_vs_mix(setup):
    g, idx, beta = setup
    k = 20
    srv = K.KatzServer(idx, workers=3, max_batch=16, k=k, tol=_tol(idx))
    try:
        R = ki.sample_queries(g, 8, 77)
        t = srv.submit(R)
        ids_a, sc_a, st_a, _ = srv.poll(t)
        _check_against_oracle(g, beta, R, ids_a, k)
        # a mix: several requests of mixed sizes submitted from two threads,
        # with R again in the middle
        rng = np.random.default_rng(5)
        others = [ki.sample_queries(g, int(s), int(seed)) for s, seed in
                  zip(rng.integers(1, 40, size=10), rng.integers(0, 10 ** 6, size=10))]
        tickets = []
        lock = threading.Lock()

        def sub(reqs):
            for r in reqs:
                tk = srv.submit(r)
                with lock:
                    tickets.append((tk, r))
                time.sleep(0.001)

        th = [threading.Thread(target=sub, args=(others[i::2],)) for i in range(2)]
        for x in th:
            x.start()
        tR = srv.submit(R)
        for x in th:
            x.join()
        ids_b, sc_b, st_b, _ = srv.poll(tR)
        # same request alone and in the mix: same ranking (tie rule), scores within tolerance
        for j in range(len(R)):
            assert np.all(np.abs(sc_a[j] - sc_b[j]) <= 2 * TAU * np.abs(sc_a[j]).max())
        _check_against_oracle(g, beta, R, ids_b, k)
        for tk, r in tickets:
            ids, sc, st, lat = srv.poll(tk)
            assert ids.shape == (len(r), k) and lat > 0
            assert all(s["status"] == 0 for s in st)
        _check_against_oracle(g, beta, others[3], srv_result(srv, others[3]), k)
    finally:
        srv.close()


def srv_result(srv, q):
    t = srv.submit(q)
    return srv.poll(t)[0]


def test_server_splits_large_request(setup):
    g, idx, beta = setup
    k = 10
    srv = K.KatzServer(idx, workers=2, max_batch=8, k=k, tol=_tol(idx))
    try:
        qs = ki.sample_queries(g, 29, 901)           # more than one worker batch
        t = srv.submit(qs)
        ids, sc, st, _ = srv.poll(t)
        assert ids.shape == (29, k)
        _check_against_oracle(g, beta, qs, ids, k)
        info = srv.info()
        assert info["done_queries"] >= 29 and info["queued_queries"] == 0
    finally:
        srv.close()


def test_server_admission_by_hbm(setup):
    g, idx, beta = setup
    srv = K.KatzServer(idx, workers=4, max_batch=512, k=5, hbm_fraction=0.8)
    try:
        info = srv.info()
        free = 288e9
        assert info["workers"] * info["capacity"] * info["bytes_per_column"] <= 0.8 * free * 1.05
        assert 1 <= info["capacity"] <= 512
    finally:
        srv.close()
    with pytest.raises(K.KatzError) as e:
        K.KatzServer(idx, workers=1, max_batch=1, k=5, hbm_fraction=1e-12)
    assert e.value.code == K.KATZ_ENOMEM
