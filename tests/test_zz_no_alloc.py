"""katz_query_noalloc (every solve buffer in the library's static device
scratch, no allocation) against katz_query on the same index and inputs,
through the C ABI: two calls in a row, the second with a smaller input, on
two indexes of different sizes (so the scratch layout changes between
calls), device and host output, both methods, and the rejection of an index
too large for the scratch and of the PCGNR ablation.  GPU only."""
import numpy as np
import pytest

import katz_inputs as ki
import oracle
from conftest import oracle_beta

pytestmark = pytest.mark.gpu
K = pytest.importorskip("paper_1912_06525_amd")


def _close(a, b, tau):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) <= tau * nb and np.max(np.abs(a - b)) <= tau * nb


def _two_calls(g, idx, c, tau, sizes, seed, method=K.KATZ_METHOD_LRC, host=False):
    import torch
    tol = tau * (1 - c) / (1 + c)
    for t, nq in enumerate(sizes):
        qs = ki.sample_queries(g, nq, seed + t)
        print("noalloc: n=%d nq=%d method=%d host=%s" % (g.n, nq, method, host), flush=True)
        ref, st0 = idx.query(qs, tol=tol, method=method)
        if host:
            out = np.full((nq, g.n), np.nan)
            got, st1 = idx.query_noalloc(qs, out=out, tol=tol, method=method)
        else:
            out = torch.full((nq, g.n), float("nan"), dtype=torch.float64, device="cuda")
            _, st1 = idx.query_noalloc(qs, out=out, tol=tol, method=method)
            torch.cuda.synchronize()
            got = out.cpu().numpy()
        for j in range(nq):
            assert st1[j]["status"] == 0 and st1[j]["rel_residual"] <= tol, st1[j]
            # both within tau of the exact vector, so within 2 tau of each other
            assert _close(got[j], ref[j], 2 * tau), (nq, j)
    return qs, got


def test_noalloc_matches_query_sbm2k():
    g = ki.workload("sbm2k").graph
    c, tau = 0.5, 1e-9
    beta = oracle_beta(g, c)
    idx = K.KatzIndex.from_graph(g, beta=beta, rank=32, labels=g.labels, max_block=200)
    qs, got = _two_calls(g, idx, c, tau, (8, 3), 31)
    # the last call against the oracle's dense solve as well
    ref = oracle.katz_oracle(g.n, g.row_ptr, g.col, qs, beta=beta, validate=False)
    for j in range(len(qs)):
        assert _close(got[j], ref["k_direct"][:, j], tau)
    _two_calls(g, idx, c, tau, (5, 2), 41, method=K.KATZ_METHOD_CG, host=True)
    # the PCGNR ablation needs buffers beyond the scratch layout: refused
    with pytest.raises(K.KatzError) as e:
        idx.query_noalloc(qs, out=np.empty((len(qs), g.n)), method=K.KATZ_METHOD_PCGNR)
    assert e.value.code == K.KATZ_EINVAL and "PCGNR" in str(e.value)
    idx.close()


def test_noalloc_matches_query_larger_index_mixed():
    """A 40k-node community graph in the precision form, 40 then 5 columns
    (the tiled output transpose, then the narrow kernels), after the small
    index above has used the scratch."""
    g = ki.workload("lnsbm4m", scale=0.01).graph
    c, tau = 0.5, 1e-7
    beta = oracle_beta(g, c)
    idx = K.KatzIndex.from_graph(g, beta=beta, rank=16, labels=g.labels, max_block=64,
                                 precision=K.KATZ_PREC_MIXED)
    _two_calls(g, idx, c, tau, (40, 5), 51)
    idx.close()


def test_noalloc_rejects_index_beyond_scratch():
    """One query column of a 6M-node index needs more than the 256 MiB scratch:
    KATZ_EINVAL with both sizes in the message; katz_query still serves it."""
    g = ki.chung_lu(6_000_000, 2.5, 1.5, seed=5)
    idx = K.KatzIndex.from_graph(g, beta_frac=0.5, rank=0, max_block=64)
    q = ki.sample_queries(g, 1, 9)
    with pytest.raises(K.KatzError) as e:
        idx.query_noalloc(q, out=np.empty((1, g.n)))
    assert e.value.code == K.KATZ_EINVAL and "scratch" in str(e.value)
    sc, st = idx.query(q, tol=1e-6)
    assert st[0]["status"] == 0
    idx.close()
