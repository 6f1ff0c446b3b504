"""CPU FP64 oracle for query-time Katz scores -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The library's product path never calls it, and it
shares no code with the HIP library (no kernels, headers, helpers or tables).

It computes the plain definition of the Katz index of a query node (Section 3.1,
eqs. KatzPath, KatzMatrix, LinearSystem): k_q = sum_{l>=1} beta^l A^l e_q =
((I - beta A)^{-1} - I) e_q = (I - beta A)^{-1} beta A e_q, two independent
ways (a dense Cholesky solve and a truncated Neumann series with a rigorous
tail bound), plus the top-K link-prediction ranking (Section 3.3, Algorithm 3's
sort step) and the Sparse-Katz re-ranking (Algorithm 3).
"""
from .reference import (  # noqa: F401
    OracleError,
    validate_csr,
    csr_matrix,
    lambda_max,
    katz_rhs,
    katz_direct,
    katz_series,
    katz_oracle,
    katz_residual,
    topk_links,
    topk_accept,
    tie_classes,
    walk_counts,
    sparse_katz,
    pearson,
    correlation_rerank,
)
from .cpu import katz_series_mt, cg_mt, lambda_max_mt  # noqa: F401,E402
