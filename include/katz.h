/*
 * katz.h -- query-time Katz proximity on one MI355X (gfx950).
 *
 * Method: Coskun, Baggag, Koyuturk, "Fast Computation of Katz Index for
 * Efficient Processing of Link Prediction Queries" (arXiv:1912.06525).
 *
 * For a query node q of an undirected graph with adjacency matrix A the
 * library returns the Katz vector k_q, the q-th column of
 *     K = sum_{l>=1} beta^l A^l = (I - beta A)^{-1} - I          (Sec. 3.1,
 * eqs. KatzPath/KatzMatrix), obtained by solving
 *     M k_q = beta A e_q,   M = I - beta A                      (eq. LinearSystem).
 * It needs 0 < beta < 1/lambda_max(A) (Sec. 3.1), so that M is SPD.
 *
 * Index (Algorithm 1, Sec. 3.2 steps 1-4): nodes are reordered into
 * independent blocks plus a vertex separator, so that
 *     M = [[M11, M12], [M12^T, M22]]
 * with M11 block diagonal (Lemma 1).  Each M11 block is factorised and its
 * inverse stored; the Schur complement S = M22 - M12^T M11^{-1} M12 is never
 * formed.  A rank-r preconditioner (eqs. RMatrix, inverseTildeS)
 *     S~^{-1} = L^{-T} (I + U~ D U~^T) L^{-1},  D = diag(sigma_i / (1 - sigma_i)),
 * uses the top r eigenpairs (sigma_i, u_i) of R = I - L^{-1} S L^{-T}.
 *
 * Query (Algorithm 2, Sec. 3.2 steps 5-6; Lemma 1 eqs. 5-6): build
 * b = beta A e_q in the permuted order, f = b2 - M12^T M11^{-1} b1, solve
 * S k2 = f by preconditioned conjugate gradients, then
 * k1 = M11^{-1} (b1 - M12 k2), merge and unpermute.  Plain CG on M (the
 * paper's comparison method) is available as a method and is the fallback.
 * Every result is checked by its true FP64 residual ||b - M k||_2 / ||b||_2
 * and refined in FP64 until it meets the requested tolerance.
 *
 * Threading: an index is immutable after build; katz_query and
 * katz_topk_links may run concurrently on one index from several host threads
 * (each call takes its own device workspace).  Errors are returned as status
 * codes; katz_last_error() returns the calling thread's last message.
 */
#ifndef KATZ_H
#define KATZ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct katz_index katz_index; /* opaque; immutable after build */

enum katz_status {
  KATZ_OK = 0,
  KATZ_EINVAL = -1,   /* bad argument (null pointer, out-of-range id, bad CSR) */
  KATZ_ENOTSYM = -2,  /* adjacency matrix is not symmetric */
  KATZ_EDIVERGE = -3, /* beta * lambda_max(A) >= 1: series diverges, M not SPD */
  KATZ_ENOMEM = -4,   /* host or device allocation failed */
  KATZ_EDEVICE = -5,  /* HIP error, or index built without a device */
  KATZ_ENOCONV = -6,  /* some query missed the tolerance (see stats) */
  KATZ_EBUSY = -7,    /* server: request still running (poll), server stopping (submit) */
  KATZ_EIO = -8       /* file error or corrupt index file */
};

enum katz_precision {
  KATZ_PREC_FP64 = 0, /* every panel, factor and reduction in FP64 */
  KATZ_PREC_MIXED = 1 /* FP32 SpMM/block solves, BF16 low-rank factor with
                         FP32 accumulation, FP64 dots, FP64 residual refinement */
};

enum katz_l_kind {
  KATZ_L_AUTO = 0,    /* CHOL when the separator is small (<= 1024), else IDENTITY */
  KATZ_L_CHOL = 1,    /* L = dense Cholesky factor of M22 (eq. RMatrix as printed); n2 <= 4096 */
  KATZ_L_IDENTITY = 2, /* L = I: R = I - S, preconditioner I + U~ D U~^T */
  KATZ_L_IC0 = 3      /* L = incomplete Cholesky factor of M22 with zero fill (an SPD L of
                         M22's own sparsity; the preconditioner ablation); n2 <= 4096 */
};

enum katz_method {
  KATZ_METHOD_LRC = 0,   /* PCG on the Schur complement S, preconditioned by S~ (Sec. 3.2 step 5) */
  KATZ_METHOD_CG = 1,    /* plain CG on M, the comparison method and the fallback */
  KATZ_METHOD_PCGNR = 2  /* ablation: Algorithm 2's recurrence with the step gamma = s^T S~^{-1} s
                            for s = S r, i.e. preconditioned CG on the normal equations of S
                            (two S-applies per iteration); results as LRC */
};

enum katz_order {
  KATZ_ORDER_AUTO = 0,     /* LOCALITY */
  KATZ_ORDER_DEGREE = 1,   /* blocks largest first; separator by degree (hubs first) */
  KATZ_ORDER_LOCALITY = 2  /* blocks and separator in BFS visit order */
};

enum katz_path {
  KATZ_PATH_LRC = 0,        /* Schur-complement PCG with the rank-r preconditioner */
  KATZ_PATH_CG = 1,         /* plain CG on M (requested) */
  KATZ_PATH_CG_FALLBACK = 2 /* LRC broke down or stalled; CG finished the query */
};

typedef struct {
  double beta;            /* damping factor beta; used when > 0 */
  double beta_frac;       /* else c in (0,1): beta = c / lambda_max(A) */
  int32_t rank;           /* r, low-rank correction dimension (>= 0) */
  int32_t max_block;      /* cap on the size of an M11 block (0: 64) */
  const int32_t* labels;  /* optional initial partition, n entries, or NULL */
  int32_t l_kind;         /* enum katz_l_kind */
  int32_t precision;      /* enum katz_precision */
  uint64_t seed;          /* Lanczos start vector seed */
  int32_t device;         /* HIP device ordinal; -1 builds a host-only index
                             (inspectable, not queryable) */
  int32_t lanczos_steps;  /* 0: max(2r, r + 20) */
  int32_t order;          /* enum katz_order: node order inside the two parts */
  int32_t u_precision;    /* storage of the low-rank factor V on the device:
                             0 auto, 1 FP64, 2 FP32, 3 BF16 (FP64 path; the
                             mixed path always stores BF16).  Auto takes BF16
                             when every weight D_i = sigma_i / (1 - sigma_i) of
                             the correction is at most 16, else FP32: the
                             preconditioner's error from rounding V grows like
                             D_max times the storage precision.  The
                             preconditioner is a fixed symmetric operator either
                             way, so the solution's accuracy does not depend on
                             it, only the iteration count. */
} katz_build_opts;

typedef struct {
  double rel_tol;      /* target true FP64 ||b - M k||_2 / ||b||_2 (default 1e-6) */
  int32_t max_iter;    /* inner iterations per refinement sweep (default 1000) */
  int32_t method;      /* enum katz_method (default LRC) */
  int32_t max_sweeps;  /* FP64 refinement sweeps (default 6) */
  int32_t check_every; /* inner iterations between host convergence polls;
                          0 (default): adaptive, the first poll after as many
                          iterations as the previous solve of the same kind on
                          this index needed (8 if none), then after 1, 1, 2, 2,
                          4, 4, 8, 8, ... more.  Iterations after convergence
                          change nothing, so results do not depend on it. */
  int32_t force_fallback; /* fault injection for tests: every LRC solve stops after
                             one iteration and counts as broken down, so the
                             refinement sweeps run plain CG (default 0) */
} katz_query_opts;

typedef struct {
  int32_t status;      /* KATZ_OK, or KATZ_ENOCONV if the tolerance was missed */
  int32_t iters;       /* inner (P)CG iterations, summed over sweeps */
  int32_t sweeps;      /* FP64 residual/refinement sweeps */
  int32_t path;        /* enum katz_path */
  double rel_residual; /* true FP64 ||b - M k||_2 / ||b||_2 of the returned k */
  double err_bound;    /* bound on ||k - k*||_2 / ||k*||_2:
                          rel_residual * (1 + c) / (1 - c) */
} katz_query_stats;

typedef struct {
  int32_t n, n1, n2;       /* nodes; block-interior nodes; separator nodes */
  int64_t nnz;             /* stored adjacency entries (2 |E|) */
  int32_t nblocks;         /* M11 blocks */
  int32_t max_block_size;  /* largest M11 block */
  int32_t rank;            /* r actually kept */
  int32_t l_kind;          /* resolved katz_l_kind (CHOL, IDENTITY or IC0) */
  int32_t precision;
  int32_t device;          /* -1 for a host-only index */
  double beta, lambda_max, c;
  double sigma_max;        /* largest kept eigenvalue of R (0 if r = 0) */
  double sigma_next;       /* Ritz value r+1 of the Lanczos run: a lower bound
                              of sigma_{r+1} (interlacing), tight only when the
                              run has converged that far (0 if unknown) */
  int64_t factor_bytes;    /* M11 block inverses as stored on the device */
  int64_t device_bytes;    /* total resident index bytes on the device */
  double build_seconds;
  int32_t u_precision;     /* storage of V as resolved (1 FP64, 2 FP32, 3 BF16) */
  /* wall seconds of the build's phases (0 for an index loaded from a file):
     [0] validation, [1] lambda_max, [2]-[6] partition (BFS chunking, vertex
     cover, minimality, components, node order), [7] permuted CSR, [8] M11
     block inverses, [9] M22 factor, [10] Lanczos on R (host or device),
     [11] upload to the device */
  double build_phase_seconds[12];
} katz_index_info_t;

/* Sets the documented defaults. */
void katz_build_opts_default(katz_build_opts* o);
void katz_query_opts_default(katz_query_opts* o);

/*
 * Builds the index (Algorithm 1): validates the CSR, computes lambda_max(A)
 * by Lanczos, partitions the graph into blocks of at most max_block nodes
 * plus a vertex separator (Sec. 3.2 steps 2-3), inverts every M11 block
 * through its Cholesky factor (step 4), factors M22 when l_kind is CHOL (or
 * takes its zero-fill incomplete factor for IC0), and
 * runs Lanczos on R for the top `rank` eigenpairs (eq. RMatrix).  Then the
 * index is copied to the device once.  With a device (opts->device >= 0), the
 * Lanczos on R runs there for large separators, and so does the Lanczos for
 * lambda_max from 2M nodes (a temporary device copy of the CSR, freed before
 * the call returns; the same iteration and stop rule as on the host, so beta
 * agrees with a host-only build to rounding).
 *   n, nnz, row_ptr[n+1], col_idx[nnz]: host CSR, int32, strictly increasing
 *     columns per row, no diagonal, symmetric.
 *   val: host FP64 nonnegative weights [nnz], or NULL for an unweighted graph.
 *   opts: may be NULL (defaults with beta_frac 0.5).
 * The inputs are copied; the caller keeps ownership.  *out receives the index
 * (free with katz_index_free).  Errors: KATZ_EINVAL (malformed CSR, bad
 * options), KATZ_ENOTSYM, KATZ_EDIVERGE (beta * lambda_max >= 1),
 * KATZ_ENOMEM, KATZ_EDEVICE.
 */
int katz_index_build(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                     const double* val, const katz_build_opts* opts, katz_index** out);

/*
 * Another index of src's graph for other options, without repeating the
 * steps that do not depend on beta (Algorithm 1; Sec. 3.2 steps 1-3: the
 * CSR checks, lambda_max, the partition, the node order and the permuted
 * adjacency are src's).  The M11 block inverses, the separator factor and
 * the Lanczos on R (step 4 and eq. RMatrix) are computed afresh from opts
 * exactly as katz_index_build computes them: beta or beta_frac, rank, l_kind,
 * precision, u_precision, seed, lanczos_steps and device apply;
 * max_block, labels and order are ignored (the partition is src's).  With
 * the same graph, partition options and seed, the result equals a fresh
 * build's.  For a new damping factor (per-beta reindexing) this skips the
 * partition, most of a build's time on large graphs.
 *   src: any index (built, loaded, or host-only); it is not modified and
 *     stays valid.  opts: may be NULL (defaults).
 *   *out receives the new index (free with katz_index_free).
 * Errors: KATZ_EINVAL (null src or out, bad options), KATZ_EDIVERGE
 * (beta * lambda_max >= 1, or a factor not positive definite), KATZ_ENOMEM,
 * KATZ_EDEVICE.
 */
int katz_index_rebuild(const katz_index* src, const katz_build_opts* opts, katz_index** out);

/*
 * Communities to pass as katz_build_opts.labels for a graph without planted
 * labels (Sec. 3.2 step 2 partitions with METIS; this library offers this
 * instead, or the build's default of one part cut into BFS chunks).  It is
 * the local-moving phase of the Louvain method on the modularity of the
 * weighted graph, every community capped at `cap` nodes (the build's
 * max_block suits): each node starts alone; a pass visits the nodes in id
 * order and moves each to the neighbouring community of the largest
 * modularity gain (its own wins ties, then the first reached in its row);
 * a community at the cap takes no one; passes stop when one moves no node or
 * after `passes`.  Serial, deterministic, O(nnz) per pass, host only.
 *   n, nnz, row_ptr, col_idx, val: the CSR as for katz_index_build (checked
 *     the same way; val NULL: unweighted).
 *   cap >= 1; passes >= 0 (0: every node alone).
 *   labels[n] (caller-owned, written): community ids 0, 1, ... in the
 *     order a breadth-first search first reaches each community (from node
 *     0, neighbours in row order, restarting at the smallest unreached
 *     node).  The build lays the parts out in label order, so this keeps
 *     neighbouring communities at nearby positions.
 *   passes_run (nullable): the passes made.
 * Errors: KATZ_EINVAL (malformed CSR, bad cap or passes, null labels),
 * KATZ_ENOTSYM, KATZ_ENOMEM.
 */
int katz_communities(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx, const double* val,
                     int32_t cap, int32_t passes, int32_t* labels, int32_t* passes_run);

/*
 * Katz vectors of nq query nodes (Algorithm 2; Lemma 1 eqs. 5-6).
 *   q[nq]: host array of node ids in [0, n), original numbering.
 *   scores: nq * n FP64, query-major: scores[i*n + v] = K[v, q[i]]
 *     (entry v = q[i] holds K_qq, the weighted closed walks).  Host or
 *     device pointer (detected); caller-allocated.
 *   st: nullable, nq entries.
 *   stream: hipStream_t to run on, or NULL for the null stream.  The call
 *     returns after the results are complete.
 * Queries run together as the columns of one batched solve.  Returns KATZ_OK,
 * or KATZ_ENOCONV if some query missed opts->rel_tol (its stats say which;
 * its scores are still the best iterate), KATZ_EINVAL, KATZ_EDEVICE,
 * KATZ_ENOMEM.
 */
int katz_query(const katz_index* idx, const int32_t* q, int32_t nq, const katz_query_opts* opts,
               double* scores, katz_query_stats* st, void* stream);

/*
 * katz_query without allocation, for callers that cannot allocate device
 * memory (code running under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and errors as
 * katz_query, with these differences:
 *   - every buffer of the solve (panels, partial sums, per-column state) lies
 *     in a static device array of the library, 256 MiB, one per GPU the
 *     library runs on, held until the process ends; the call makes no
 *     hipMalloc, hipFree, pinned-host or graph allocation (its first call on
 *     a device only looks up that array's address);
 *   - KATZ_EINVAL when one query column of this index needs more scratch
 *     than 256 MiB (the message gives both sizes; about 60 bytes per node
 *     and column in FP64, so graphs of up to about 4 million nodes fit);
 *     larger nq runs in chunks of the columns that fit;
 *   - it runs on `stream` itself (not on a workspace stream), without HIP
 *     graphs, kernel profiling or the SpMM launch-shape autotuner (it uses
 *     the shape an earlier katz_query chose, or the default; results do not
 *     depend on that shape);
 *   - the KATZ_METHOD_PCGNR ablation is not offered (KATZ_EINVAL);
 *   - every call on one GPU shares that GPU's scratch, which keeps the last
 *     call's contents (the state that must start at zero is cleared by each
 *     call): calls that overlap on one GPU, from several threads or streams,
 *     race and must be serialised by the caller.
 */
int katz_query_noalloc(const katz_index* idx, const int32_t* q, int32_t nq, const katz_query_opts* opts,
                       double* scores, katz_query_stats* st, void* stream);

/*
 * Top-k predicted links per query (Sec. 3.3; the descending sort of
 * Algorithm 3): candidates are all nodes except q and its neighbours, ranked
 * by (Katz score descending, node id ascending).
 *   ids: nq * k int32 (query-major), padded with -1 when fewer than k
 *     candidates exist; scores: nq * k FP64 (NaN padding) or NULL.  Host or
 *     device pointers.  Other arguments as katz_query.
 */
int katz_topk_links(const katz_index* idx, const int32_t* q, int32_t nq, int32_t k,
                    const katz_query_opts* opts, int32_t* ids, double* scores,
                    katz_query_stats* st, void* stream);

/*
 * Writes the index to a file, so that the offline part of the method
 * (Sec. 3.2 steps 1-4, Algorithm 1) is done once and later processes only
 * run queries (Algorithm 2).  The file holds the reordering, the permuted
 * CSR, the M11 block inverses, the M22 factor and the low-rank factors, in
 * this host's byte order.  path: a file name; an existing file is replaced.
 * Errors: KATZ_EINVAL (null argument), KATZ_EIO (cannot open or write).
 */
int katz_index_save(const katz_index* idx, const char* path);

/*
 * Reads an index written by katz_index_save and, when device >= 0, copies
 * it to that device (device < 0: host-only, for the inspection calls).  The
 * file is validated in full before use (sizes, CSR structure, symmetry,
 * permutation, block structure, factor shapes).  *out receives the index
 * (free with katz_index_free).  Errors: KATZ_EINVAL (null argument, not an
 * index file, other version or byte order, or failed validation), KATZ_EIO
 * (cannot open, truncated), KATZ_ENOMEM, KATZ_EDEVICE.
 */
int katz_index_load(const char* path, int32_t device, katz_index** out);

/*
 * Katz scores of node pairs (the pairwise query of Sec. 3.1): scores[i] =
 * K[dst[i], src[i]] = ((I - beta A)^{-1} - I)[dst[i], src[i]] (K is
 * symmetric, so the roles may be swapped).  Pairs sharing a source share one
 * solve: the distinct sources run as the columns of batched solves, and only
 * the requested entries leave the device.
 *   src[npairs], dst[npairs]: host arrays of node ids in [0, n).
 *   scores: npairs FP64, host or device pointer (detected), caller-allocated.
 *   st: nullable, npairs entries (each pair gets its source's solve stats).
 * Errors as katz_query.
 */
int katz_pair_scores(const katz_index* idx, const int32_t* src, const int32_t* dst, int32_t npairs,
                     const katz_query_opts* opts, double* scores, katz_query_stats* st, void* stream);

/*
 * Sparse-Katz link prediction (Sec. 3.3, Algorithm 3).  For each query q:
 * the top-s candidates of k_q (q and its neighbours excluded, as in
 * katz_topk_links) are re-ranked by the Pearson correlation of their row
 * with q's row in K_T = [k_t1 ... k_tT], the Katz vectors of the T
 * highest-ranked candidates ("modular" nodes).  Rows are T-vectors K[v, t].
 * Correlation descending; undefined correlations (a constant row, or fewer
 * than 2 modular nodes) last; ties keep the Katz order.
 *   s in [0, 4096], T in [2, 4096].
 *   ids: nq * s int32 (padded with -1); corr: nq * s FP64 correlations (NaN
 *     when undefined or padded) or NULL.  Host or device pointers.
 *   st: nullable, nq entries (the stats of the k_q solves).
 * Errors as katz_query.
 */
int katz_sparse_katz(const katz_index* idx, const int32_t* q, int32_t nq, int32_t s, int32_t T,
                     const katz_query_opts* opts, int32_t* ids, double* corr, katz_query_stats* st,
                     void* stream);

/* Frees host and device memory of the index.  NULL is a no-op. */
void katz_index_free(katz_index* idx);

/* Sizes and parameters of an index. */
int katz_index_info(const katz_index* idx, katz_index_info_t* info);

/*
 * Host copies of the index's reordering (Sec. 3.2 step 3), for inspection:
 *   perm[n]: new position of original node v (NULL to skip);
 *   block_ptr[nblocks + 1]: first new position of each M11 block, ending at
 *   n1 (NULL to skip).  Separator nodes occupy positions [n1, n).
 */
int katz_index_partition(const katz_index* idx, int32_t* perm, int32_t* block_ptr);

/*
 * Host copy of the low-rank factors (eqs. RMatrix, inverseTildeS):
 *   U[n2 * rank]: Ritz vectors of R, row-major (row = separator position);
 *   sigma[rank]: their Ritz values, descending.  Either may be NULL.
 */
int katz_index_lowrank(const katz_index* idx, double* U, double* sigma);

/* ------------------------------------------------------------- serving
 * Continuous batching of top-K link-prediction requests (Sec. 3.3) on one
 * index: `workers` worker slots, each with a device workspace of `max_batch`
 * query columns and its own stream, take columns from the request queue
 * (merging small requests, splitting large ones) whenever they are free, so
 * requests arriving while others run are admitted as slots free up and their
 * batches overlap on the device.  Requests are served in arrival order,
 * each free worker taking up to max_batch columns.  Workers x max_batch is admitted
 * against hbm_fraction of the free HBM at creation (reduced to fit; KATZ_ENOMEM
 * if not even one column fits).  All calls are thread-safe. */
typedef struct katz_server katz_server;

typedef struct {
  int32_t workers;       /* worker slots (0: 4), reduced to fit the HBM budget */
  int32_t max_batch;     /* query columns per worker batch, 1..512 (default 64) */
  double hbm_fraction;   /* share of free HBM for the workspaces (default 0.8) */
  int32_t k;             /* links returned per query node (default 100) */
  katz_query_opts query; /* solve options for every batch */
} katz_server_opts;

typedef struct {
  int32_t workers, capacity, k;   /* as admitted */
  int64_t queued_queries;         /* query nodes waiting for a worker */
  int64_t live_columns;           /* query columns being solved now */
  int64_t done_queries, done_requests;
  int64_t bytes_per_column;       /* device workspace bytes per resident column */
} katz_server_info_t;

void katz_server_opts_default(katz_server_opts* o);
/* Starts the workers.  idx must outlive the server.  Errors: KATZ_EINVAL,
 * KATZ_EDEVICE (host-only index), KATZ_ENOMEM. */
int katz_server_create(const katz_index* idx, const katz_server_opts* opts, katz_server** out);
/* Queues a request of nq query nodes (copied); returns at once with a ticket.
 * Errors: KATZ_EINVAL (bad ids), KATZ_EBUSY (server stopping), KATZ_ENOMEM
 * (host memory for the request's nq x k result slots). */
int katz_server_submit(katz_server* s, const int32_t* q, int32_t nq, int64_t* ticket);
/* Waits up to timeout_us (0: do not wait, < 0: forever) for a request; when it
 * is complete copies ids[nq*k], scores[nq*k], st[nq] (each nullable) and the
 * submit-to-completion latency, releases the ticket and returns its status
 * (KATZ_OK, KATZ_ENOCONV, or the error of a batch that failed, e.g.
 * KATZ_EDEVICE).  KATZ_EBUSY if still running, KATZ_EINVAL for an unknown
 * ticket. */
int katz_server_poll(katz_server* s, int64_t ticket, int32_t* ids, double* scores, katz_query_stats* st,
                     double* latency_ms, int64_t timeout_us);
int katz_server_info(katz_server* s, katz_server_info_t* info);
/* Finishes the queued requests, stops the workers and frees the workspaces
 * and the server.  No other call on s may be in progress or follow (a thread
 * still waiting in katz_server_poll must have returned first). */
void katz_server_destroy(katz_server* s);

/* Per-kernel timing of the query path (tracing aid): with profiling on, every
 * launch of the hot kernels is bracketed by HIP events on the solve stream and
 * the algorithmic bytes it moves are booked to its kind. */
typedef struct {
  char name[32];      /* kernel kind */
  int64_t launches;   /* timed launches */
  double total_ms;    /* summed event time */
  double alg_bytes;   /* summed algorithmic bytes (each operand counted once) */
} katz_kernel_stat;

/* Turns profiling on (1) or off (0); returns the previous setting. */
int katz_profile_enable(int on);
/* Clears the accumulated statistics. */
void katz_profile_reset(void);
/* Copies up to max kinds into out; returns the number written. */
int katz_profile_read(katz_kernel_stat* out, int max);

/* Thread-local message describing the last error on this thread. */
const char* katz_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* KATZ_H */
