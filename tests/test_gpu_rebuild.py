"""GPU check of katz_index_rebuild: an index rebuilt on the device for
another damping factor answers bit-identically to a fresh build with those
options, in both precisions, one column and a batch, with the Lanczos on R on
the host and on the device."""
import numpy as np
import pytest

import katz_inputs as ki

pytestmark = pytest.mark.gpu
K = pytest.importorskip("paper_1912_06525_amd")


@pytest.mark.parametrize("lanczos", ["1", "2"])
@pytest.mark.parametrize("prec", [0, 1])
def test_rebuilt_index_answers_like_a_fresh_build(monkeypatch, lanczos, prec):
    monkeypatch.setenv("KATZ_LANCZOS", lanczos)
    g = ki.chung_lu(20000, 2.5, 8, seed=7)
    src = K.KatzIndex.from_graph(g, beta_frac=0.5, rank=16, precision=prec)
    re = src.rebuild(beta_frac=0.9, rank=24, precision=prec)
    fresh = K.KatzIndex.from_graph(g, beta_frac=0.9, rank=24, precision=prec)
    qs = ki.sample_queries(g, 40, 3)
    for q in ([int(qs[0])], qs):
        a, sa = re.query(q, tol=1e-9)
        b, sb = fresh.query(q, tol=1e-9)
        assert np.array_equal(a, b)
        assert [s["iters"] for s in sa] == [s["iters"] for s in sb]
    a0, _ = src.query([int(qs[0])], tol=1e-9)  # the source still answers for its own beta
    assert np.all(np.isfinite(a0))
    for x in (src, re, fresh):
        x.close()
