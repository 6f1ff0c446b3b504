/*
 * Multi-core FP64 CPU tools for query-time Katz -- TEST INFRASTRUCTURE ONLY.
 *
 * Called (through oracle/cpu.py) by the test suite and by the benchmark's CPU
 * leg, never by the library's product path.  Shares no code, header, table or
 * helper with the HIP library; it reads the same CSR arrays the generators
 * produce.
 *
 * Paper: Coskun, Baggag, Koyuturk, "Fast Computation of Katz Index for
 * Efficient Processing of Link Prediction Queries" (arXiv:1912.06525).
 * Notation: beta is the damping factor (alpha in Sec. 3.1), A the symmetric
 * nonnegative adjacency matrix, c = beta * lambda_max(A) < 1.
 *
 * ko_series -- the oracle at benchmark sizes: the Katz vector of query q,
 *   k_q = sum_{l >= 1} (beta A)^l e_q                     (Sec. 3.1, eq. KatzMatrix
 *   applied to e_q; the walk sum of eq. KatzPath), as a truncated Neumann
 *   series.  Term l is v_l = beta A v_{l-1}, v_0 = e_q, a plain CSR product in
 *   a fixed entry order.  Column j stops after term L when the rigorous tail
 *   bound ||sum_{l > L} v_l|| <= ||v_L|| c / (1 - c) (||beta A||_2 = c) is at
 *   most tol * ||s_L||.  Every term is >= 0, so the sum has no cancellation.
 *
 * ko_cg -- the CPU baseline: plain conjugate gradients (the paper's
 *   comparison method, Sec. 4) on M k = beta A e_q with M = I - beta A
 *   (eq. LinearSystem), several right-hand sides at once, each with its own
 *   step lengths and stop test, OpenMP over rows.  Stop rule as the GPU path:
 *   recurrence residual <= tol/2 ||b||, then the true residual ||b - M k|| /
 *   ||b|| is recomputed and CG restarts from k on the columns above tol.
 *
 * ko_lambda_max -- lambda_max(A), which sets the convergence condition
 *   beta < 1 / lambda_max (Sec. 3.1) and c = beta * lambda_max: the Lanczos
 *   iteration on A from the all-ones vector (it overlaps the nonnegative
 *   Perron vector of a nonnegative A), without reorthogonalisation (the
 *   largest Ritz value is the first to converge and is not disturbed by the
 *   loss of orthogonality), the largest eigenvalue of each tridiagonal by
 *   Sturm-sequence bisection.
 *
 * Layout: panels are node-major, n x B, element (i, j) at [i * B + j].
 * Reductions over rows sum fixed blocks of kRowBlock rows and then the blocks
 * in order, so results do not depend on the thread count.
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <sys/mman.h>

#include <omp.h>

enum { kRowBlock = 4096, kAccMax = 64 };

/* n x B panels: 2 MiB aligned and advised for transparent huge pages, since
 * the products gather panel rows at random (fewer TLB misses; the arithmetic
 * is unchanged).  Zero-filled.  Freed with free(). */
static double* panel_alloc(int64_t elems) {
  void* p = NULL;
  const size_t bytes = (size_t)(elems > 0 ? elems : 1) * sizeof(double);
  if (posix_memalign(&p, (size_t)1 << 21, bytes) != 0) return NULL;
  (void)madvise(p, bytes, MADV_HUGEPAGE);
  memset(p, 0, bytes);
  return (double*)p;
}

/* y = beta A x (n x B panels).  Row i accumulates its entries in CSR order
 * from 0, one running sum per column (held in registers up to kAccMax
 * columns). */
static void spmm_beta(int32_t n, const int64_t* rp, const int32_t* col, const double* val, double beta, int B,
                      const double* restrict x, double* restrict y) {
#pragma omp parallel for schedule(dynamic, 1024)
  for (int32_t i = 0; i < n; i++) {
    double* yi = y + (int64_t)i * B;
    if (B <= kAccMax) {
      double acc[kAccMax];
      for (int j = 0; j < B; j++) acc[j] = 0.0;
      for (int64_t k = rp[i]; k < rp[i + 1]; k++) {
        const double a = beta * (val ? val[k] : 1.0);
        const double* xc = x + (int64_t)col[k] * B;
        for (int j = 0; j < B; j++) acc[j] += a * xc[j];
      }
      for (int j = 0; j < B; j++) yi[j] = acc[j];
    } else {
      for (int j = 0; j < B; j++) yi[j] = 0.0;
      for (int64_t k = rp[i]; k < rp[i + 1]; k++) {
        const double a = beta * (val ? val[k] : 1.0);
        const double* xc = x + (int64_t)col[k] * B;
        for (int j = 0; j < B; j++) yi[j] += a * xc[j];
      }
    }
  }
}

/* Column sums over fixed row blocks: part[blk * B + j]; reduce_blocks sums
 * them in block order into out[j]. */
static void reduce_blocks(const double* part, int64_t nblk, int B, double* out) {
  for (int j = 0; j < B; j++) out[j] = 0.0;
  for (int64_t b = 0; b < nblk; b++)
    for (int j = 0; j < B; j++) out[j] += part[b * B + j];
}

static int64_t nblocks(int32_t n) { return ((int64_t)n + kRowBlock - 1) / kRowBlock; }

static void set_threads(int threads) {
  if (threads > 0) omp_set_num_threads(threads);
}

/*
 * k[n*B]: Katz vectors of q[0..B) (node-major).  terms[B]: terms summed per
 * column; tail[B]: its final tail bound ||v_L|| c / (1 - c) (absolute).
 * threads: OpenMP threads (0: the runtime's default); *threads_used receives
 * the count.  Returns 0, -1 for bad arguments, -2 if some column needed more
 * than max_terms (its k is the partial sum).
 */
int ko_series(int32_t n, const int64_t* rp, const int32_t* col, const double* val, double beta, double c, int32_t B,
              const int32_t* q, double tol, int32_t max_terms, int32_t threads, double* k, int32_t* terms,
              double* tail, int32_t* threads_used) {
  if (n <= 0 || B <= 0 || !(c > 0.0 && c < 1.0) || !(beta > 0.0)) return -1;
  for (int j = 0; j < B; j++)
    if (q[j] < 0 || q[j] >= n) return -1;
  set_threads(threads);
  if (threads_used) *threads_used = omp_get_max_threads();
  const int64_t nB = (int64_t)n * B, nblk = nblocks(n);
  double* v = panel_alloc(nB);
  double* w = panel_alloc(nB);
  double* pv = (double*)malloc((size_t)nblk * B * sizeof(double));
  double* ps = (double*)malloc((size_t)nblk * B * sizeof(double));
  double* nv = (double*)malloc((size_t)B * sizeof(double));
  double* ns = (double*)malloc((size_t)B * sizeof(double));
  unsigned char* live = (unsigned char*)malloc((size_t)B);
  if (!v || !w || !pv || !ps || !nv || !ns || !live) {
    free(v); free(w); free(pv); free(ps); free(nv); free(ns); free(live);
    return -1;
  }
  memset(k, 0, (size_t)nB * sizeof(double));
  for (int j = 0; j < B; j++) {
    v[(int64_t)q[j] * B + j] = 1.0; /* v_0 = e_q */
    live[j] = 1;
    terms[j] = 0;
    tail[j] = 0.0;
  }
  const double ratio = c / (1.0 - c);
  int remaining = B, rc = 0;
  for (int32_t L = 1; remaining > 0; L++) {
    if (L > max_terms) {
      rc = -2;
      break;
    }
    spmm_beta(n, rp, col, val, beta, B, v, w); /* v_L = beta A v_{L-1} */
    double* t = v;
    v = w;
    w = t;
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < nblk; b++) {
      double* pvb = pv + b * B;
      double* psb = ps + b * B;
      for (int j = 0; j < B; j++) pvb[j] = psb[j] = 0.0;
      const int64_t i1 = (b + 1) * kRowBlock < n ? (b + 1) * kRowBlock : n;
      for (int64_t i = b * kRowBlock; i < i1; i++) {
        const double* vi = v + i * B;
        double* ki = k + i * B;
        for (int j = 0; j < B; j++) {
          if (live[j]) ki[j] += vi[j];
          pvb[j] += vi[j] * vi[j];
          psb[j] += ki[j] * ki[j];
        }
      }
    }
    reduce_blocks(pv, nblk, B, nv);
    reduce_blocks(ps, nblk, B, ns);
    for (int j = 0; j < B; j++) {
      if (!live[j]) continue;
      const double bound = sqrt(nv[j]) * ratio;
      terms[j] = L;
      tail[j] = bound;
      if (bound <= tol * sqrt(ns[j])) {
        live[j] = 0;
        remaining--;
      }
    }
  }
  free(v); free(w); free(pv); free(ps); free(nv); free(ns); free(live);
  return rc;
}

/* Number of eigenvalues of the symmetric tridiagonal (a[0..m), b[0..m-1))
 * below x: negative pivots of the LDL^T factorisation of T - x I (Sturm
 * sequence).  A zero pivot is nudged to a tiny negative value. */
static int sturm_below(int m, const double* a, const double* b, double x) {
  int cnt = 0;
  double d = 1.0;
  for (int i = 0; i < m; i++) {
    const double off = i > 0 ? b[i - 1] * b[i - 1] / d : 0.0;
    d = a[i] - x - off;
    if (d == 0.0) d = -1e-300;
    if (d < 0.0) cnt++;
  }
  return cnt;
}

/* Largest eigenvalue of the tridiagonal by bisection inside its Gershgorin
 * interval, to a relative width of 4 ulp. */
static double tridiag_max_eig(int m, const double* a, const double* b) {
  double lo = a[0], hi = a[0];
  for (int i = 0; i < m; i++) {
    const double r = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i < m - 1 ? fabs(b[i]) : 0.0);
    if (a[i] - r < lo) lo = a[i] - r;
    if (a[i] + r > hi) hi = a[i] + r;
  }
  for (int it = 0; it < 200; it++) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (hi - lo <= 4.0 * 2.220446049250313e-16 * fmax(fabs(lo), fabs(hi))) break;
    if (sturm_below(m, a, b, mid) == m) hi = mid; /* every eigenvalue is below mid */
    else lo = mid;
  }
  return hi;
}

/* Fixed-order dot product of two n-vectors (row blocks, then blocks in
 * order). */
static double dot_blocks(int32_t n, const double* x, const double* y, double* part) {
  const int64_t nblk = nblocks(n);
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < nblk; b++) {
    const int64_t i1 = (b + 1) * kRowBlock < n ? (b + 1) * kRowBlock : n;
    double s = 0.0;
    for (int64_t i = b * kRowBlock; i < i1; i++) s += x[i] * y[i];
    part[b] = s;
  }
  double s = 0.0;
  for (int64_t b = 0; b < nblk; b++) s += part[b];
  return s;
}

/*
 * *lam: lambda_max(A) (0 for a graph with no edges).  Runs Lanczos steps
 * until the largest Ritz value changes by at most tol (relative) over two
 * consecutive steps, the Krylov space is exhausted, or max_steps.  *steps
 * receives the steps taken.  Returns 0, -1 for bad arguments or memory, -2
 * when max_steps ended the run (*lam is then the last Ritz value, a lower
 * bound).
 */
int ko_lambda_max(int32_t n, const int64_t* rp, const int32_t* col, const double* val, int32_t max_steps, double tol,
                  int32_t threads, double* lam, int32_t* steps, int32_t* threads_used) {
  if (n <= 0 || max_steps < 1 || !lam) return -1;
  set_threads(threads);
  if (threads_used) *threads_used = omp_get_max_threads();
  const int64_t nblk = nblocks(n);
  double* q0 = panel_alloc(n);
  double* q1 = panel_alloc(n);
  double* w = panel_alloc(n);
  double* part = (double*)malloc((size_t)nblk * sizeof(double));
  double* a = (double*)malloc((size_t)max_steps * sizeof(double));
  double* b = (double*)malloc((size_t)max_steps * sizeof(double));
  if (!q0 || !q1 || !w || !part || !a || !b) {
    free(q0); free(q1); free(w); free(part); free(a); free(b);
    return -1;
  }
  const double inv = 1.0 / sqrt((double)n);
  for (int32_t i = 0; i < n; i++) q1[i] = inv;
  double theta = 0.0, prev = -1.0;
  int stable = 0, rc = -2, m = 0;
  for (int j = 0; j < max_steps; j++) {
    /* w = A q1 - b_{j-1} q0 */
    spmm_beta(n, rp, col, val, 1.0, 1, q1, w);
    if (j > 0) {
#pragma omp parallel for schedule(static)
      for (int32_t i = 0; i < n; i++) w[i] -= b[j - 1] * q0[i];
    }
    a[j] = dot_blocks(n, w, q1, part);
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; i++) w[i] -= a[j] * q1[i];
    const double bj = sqrt(dot_blocks(n, w, w, part));
    b[j] = bj;
    m = j + 1;
    theta = tridiag_max_eig(m, a, b);
    if (bj <= 1e-14 * fmax(fabs(theta), 1e-300)) { /* invariant subspace: theta is exact */
      rc = 0;
      break;
    }
    stable = (prev >= 0.0 && fabs(theta - prev) <= tol * fabs(theta)) ? stable + 1 : 0;
    if (stable >= 2) {
      rc = 0;
      break;
    }
    prev = theta;
    double* t = q0;
    q0 = q1;
    q1 = t;
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; i++) q1[i] = w[i] / bj;
  }
  *lam = theta;
  if (steps) *steps = m;
  free(q0); free(q1); free(w); free(part); free(a); free(b);
  return rc;
}

/* q = p - beta A p on the active columns, and block partials of <p, q>. */
static void apply_m(int32_t n, const int64_t* rp, const int32_t* col, const double* val, double beta, int B,
                    const double* restrict p, double* restrict qv, const unsigned char* act, double* part) {
  const int64_t nblk = nblocks(n);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t b = 0; b < nblk; b++) {
    double* pb = part + b * B;
    for (int j = 0; j < B; j++) pb[j] = 0.0;
    const int64_t i1 = (b + 1) * kRowBlock < n ? (b + 1) * kRowBlock : n;
    double acc[kAccMax];
    for (int64_t i = b * kRowBlock; i < i1; i++) {
      double* qi = qv + i * B;
      const double* pi = p + i * B;
      if (B <= kAccMax) {
        for (int j = 0; j < B; j++) acc[j] = 0.0;
        for (int64_t e = rp[i]; e < rp[i + 1]; e++) {
          const double a = val ? val[e] : 1.0;
          const double* pc = p + (int64_t)col[e] * B;
          for (int j = 0; j < B; j++) acc[j] += a * pc[j];
        }
        for (int j = 0; j < B; j++) qi[j] = acc[j];
      } else {
        for (int j = 0; j < B; j++) qi[j] = 0.0;
        for (int64_t e = rp[i]; e < rp[i + 1]; e++) {
          const double a = val ? val[e] : 1.0;
          const double* pc = p + (int64_t)col[e] * B;
          for (int j = 0; j < B; j++) qi[j] += a * pc[j];
        }
      }
      for (int j = 0; j < B; j++) {
        if (!act[j]) continue;
        qi[j] = pi[j] - beta * qi[j];
        pb[j] += pi[j] * qi[j];
      }
    }
  }
}

/*
 * x[n*B]: solutions of (I - beta A) x = beta A e_q for q[0..B), node-major.
 * iters[B]: CG iterations per column (over all restarts); relres[B]: true
 * FP64 ||b - M x|| / ||b|| of the returned x (0 for an isolated query).
 * Returns 0, -1 for bad arguments, -2 if some column missed tol within
 * max_iter iterations.
 */
int ko_cg(int32_t n, const int64_t* rp, const int32_t* col, const double* val, double beta, int32_t B,
          const int32_t* q, double tol, int32_t max_iter, int32_t threads, double* x, int32_t* iters,
          double* relres, int32_t* threads_used) {
  if (n <= 0 || B <= 0 || !(beta > 0.0)) return -1;
  for (int j = 0; j < B; j++)
    if (q[j] < 0 || q[j] >= n) return -1;
  set_threads(threads);
  if (threads_used) *threads_used = omp_get_max_threads();
  const int64_t nB = (int64_t)n * B, nblk = nblocks(n);
  double* b = panel_alloc(nB);
  double* r = panel_alloc(nB);
  double* p = panel_alloc(nB);
  double* qv = panel_alloc(nB);
  double* part = (double*)malloc((size_t)nblk * B * sizeof(double));
  double* s = (double*)malloc((size_t)B * 6 * sizeof(double));
  unsigned char* act = (unsigned char*)malloc((size_t)B);
  unsigned char* todo = (unsigned char*)malloc((size_t)B);
  if (!b || !r || !p || !qv || !part || !s || !act || !todo) {
    free(b); free(r); free(p); free(qv); free(part); free(s); free(act); free(todo);
    return -1;
  }
  double *bn = s, *rr = s + B, *pq = s + 2 * B, *al = s + 3 * B, *rr2 = s + 4 * B, *tr = s + 5 * B;
  /* b = beta A e_q: the product of the CSR with the unit panel */
  memset(p, 0, (size_t)nB * sizeof(double));
  for (int j = 0; j < B; j++) p[(int64_t)q[j] * B + j] = 1.0;
  spmm_beta(n, rp, col, val, beta, B, p, b);
  memset(x, 0, (size_t)nB * sizeof(double));
#pragma omp parallel for schedule(static)
  for (int64_t b0 = 0; b0 < nblk; b0++) {
    double* pb = part + b0 * B;
    for (int j = 0; j < B; j++) pb[j] = 0.0;
    const int64_t i1 = (b0 + 1) * kRowBlock < n ? (b0 + 1) * kRowBlock : n;
    for (int64_t i = b0 * kRowBlock; i < i1; i++)
      for (int j = 0; j < B; j++) pb[j] += b[i * B + j] * b[i * B + j];
  }
  reduce_blocks(part, nblk, B, bn);
  for (int j = 0; j < B; j++) {
    bn[j] = sqrt(bn[j]);
    iters[j] = 0;
    relres[j] = 0.0;
    todo[j] = bn[j] > 0.0;
  }
  memcpy(r, b, (size_t)nB * sizeof(double)); /* r = b - M x with x = 0 */
  int rc = 0;
  int total = 0;
  for (int restart = 0;; restart++) {
    int any = 0;
    for (int j = 0; j < B; j++) any |= todo[j];
    if (!any) break;
    if (total >= max_iter || restart >= 50) {
      rc = -2;
      break;
    }
    /* (re)start on the columns above tolerance: p = r, rr = <r, r> */
    memcpy(p, r, (size_t)nB * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t b0 = 0; b0 < nblk; b0++) {
      double* pb = part + b0 * B;
      for (int j = 0; j < B; j++) pb[j] = 0.0;
      const int64_t i1 = (b0 + 1) * kRowBlock < n ? (b0 + 1) * kRowBlock : n;
      for (int64_t i = b0 * kRowBlock; i < i1; i++)
        for (int j = 0; j < B; j++) pb[j] += r[i * B + j] * r[i * B + j];
    }
    reduce_blocks(part, nblk, B, rr);
    for (int j = 0; j < B; j++) act[j] = todo[j] && sqrt(rr[j]) > 0.5 * tol * bn[j];
    for (; total < max_iter; total++) {
      int na = 0;
      for (int j = 0; j < B; j++) na += act[j];
      if (!na) break;
      apply_m(n, rp, col, val, beta, B, p, qv, act, part);
      reduce_blocks(part, nblk, B, pq);
      for (int j = 0; j < B; j++) {
        al[j] = 0.0;
        if (!act[j]) continue;
        if (!(pq[j] > 0.0)) { /* breakdown: leave the column to the residual check */
          act[j] = 0;
          continue;
        }
        al[j] = rr[j] / pq[j];
        iters[j]++;
      }
#pragma omp parallel for schedule(static)
      for (int64_t b0 = 0; b0 < nblk; b0++) {
        double* pb = part + b0 * B;
        for (int j = 0; j < B; j++) pb[j] = 0.0;
        const int64_t i1 = (b0 + 1) * kRowBlock < n ? (b0 + 1) * kRowBlock : n;
        for (int64_t i = b0 * kRowBlock; i < i1; i++)
          for (int j = 0; j < B; j++) {
            if (!act[j]) continue;
            const int64_t o = i * B + j;
            x[o] += al[j] * p[o];
            r[o] -= al[j] * qv[o];
            pb[j] += r[o] * r[o];
          }
      }
      reduce_blocks(part, nblk, B, rr2);
      for (int j = 0; j < B; j++) {
        tr[j] = 0.0;
        if (!act[j]) continue;
        tr[j] = rr2[j] / rr[j];
        rr[j] = rr2[j];
        if (sqrt(rr2[j]) <= 0.5 * tol * bn[j]) act[j] = 0;
      }
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < n; i++)
        for (int j = 0; j < B; j++)
          if (act[j]) p[i * B + j] = r[i * B + j] + tr[j] * p[i * B + j];
    }
    /* true residual r = b - (x - beta A x) */
    for (int j = 0; j < B; j++) act[j] = 1;
    apply_m(n, rp, col, val, beta, B, x, qv, act, part);
#pragma omp parallel for schedule(static)
    for (int64_t b0 = 0; b0 < nblk; b0++) {
      double* pb = part + b0 * B;
      for (int j = 0; j < B; j++) pb[j] = 0.0;
      const int64_t i1 = (b0 + 1) * kRowBlock < n ? (b0 + 1) * kRowBlock : n;
      for (int64_t i = b0 * kRowBlock; i < i1; i++)
        for (int j = 0; j < B; j++) {
          const int64_t o = i * B + j;
          r[o] = b[o] - qv[o];
          pb[j] += r[o] * r[o];
        }
    }
    reduce_blocks(part, nblk, B, rr);
    for (int j = 0; j < B; j++) {
      if (!(bn[j] > 0.0)) continue;
      relres[j] = sqrt(rr[j]) / bn[j];
      todo[j] = relres[j] > tol;
    }
  }
  free(b); free(r); free(p); free(qv); free(part); free(s); free(act); free(todo);
  return rc;
}
