/*
 * Seeded synthetic graph generators for the Katz workloads.
 *
 * This file builds the inputs only: undirected simple graphs in CSR form
 * (symmetric, sorted rows, no self loops, no duplicates) and seeded query
 * node lists.  It holds none of the Katz method's arithmetic, and both the
 * CPU oracle and the HIP library consume its output unchanged.
 *
 * Random numbers: SplitMix64 (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014), one stream per generator
 * call, seeded by the caller.
 *
 * Generators:
 *   - stochastic block model with per-block p_in and a uniform p_out,
 *     sampled pair by pair with geometric skipping (Batagelj and Brandes,
 *     "Efficient generation of large random networks", Phys. Rev. E 71, 2005);
 *   - lognormal community sizes for the SBM;
 *   - exact Chung-Lu (p_uv = min(1, w_u w_v / sum w)) by the skipping method
 *     of Miller and Hagberg ("Efficient generation of networks with given
 *     expected degrees", WAW 2011), O(n + m);
 *   - a degree-corrected SBM hybrid: Chung-Lu inside each community plus a
 *     global Chung-Lu layer for the inter-community share of the edge mass.
 *
 * Every generator can relabel nodes by a seeded uniform permutation, so the
 * node ids carry no structure of the generating process.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ RNG */
typedef struct { uint64_t s; } kg_rng;

static uint64_t kg_next(kg_rng* r) {
  uint64_t z = (r->s += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
/* uniform in the open interval (0, 1) */
static double kg_unif(kg_rng* r) {
  return ((double)(kg_next(r) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}
static double kg_normal(kg_rng* r) { /* Box-Muller, one value per call */
  double u1 = kg_unif(r), u2 = kg_unif(r);
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925 * u2);
}
static uint64_t kg_below(kg_rng* r, uint64_t m) { /* uniform in [0, m) */
  /* rejection to avoid modulo bias */
  uint64_t lim = UINT64_MAX - (UINT64_MAX % m);
  uint64_t x;
  do { x = kg_next(r); } while (x >= lim);
  return x % m;
}

/* --------------------------------------------------------- edge buffer */
typedef struct { int64_t len, cap; int32_t* uv; } kg_edges;

static int kg_push(kg_edges* e, int32_t u, int32_t v) {
  if (e->len == e->cap) {
    int64_t nc = e->cap ? e->cap * 2 : (1 << 16);
    int32_t* p = (int32_t*)realloc(e->uv, (size_t)nc * 2 * sizeof(int32_t));
    if (!p) return -1;
    e->uv = p; e->cap = nc;
  }
  e->uv[2 * e->len] = u; e->uv[2 * e->len + 1] = v; e->len++;
  return 0;
}

/* ------------------------------------------------------------ the graph */
typedef struct kg_graph {
  int32_t n;
  int64_t nnz;
  int32_t* row_ptr;  /* n+1 */
  int32_t* col;      /* nnz */
  int32_t* labels;   /* n, community label or NULL */
  int32_t ncomm;
} kg_graph;

void kg_graph_free(kg_graph* g) {
  if (!g) return;
  free(g->row_ptr); free(g->col); free(g->labels); free(g);
}
int32_t kg_graph_n(const kg_graph* g) { return g->n; }
int64_t kg_graph_nnz(const kg_graph* g) { return g->nnz; }
int32_t kg_graph_ncomm(const kg_graph* g) { return g->labels ? g->ncomm : 0; }
void kg_graph_copy(const kg_graph* g, int32_t* row_ptr, int32_t* col, int32_t* labels) {
  if (row_ptr) memcpy(row_ptr, g->row_ptr, sizeof(int32_t) * (size_t)(g->n + 1));
  if (col) memcpy(col, g->col, sizeof(int32_t) * (size_t)g->nnz);
  if (labels && g->labels) memcpy(labels, g->labels, sizeof(int32_t) * (size_t)g->n);
}

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/* Relabels by perm (if non-NULL) and builds a symmetric CSR with sorted,
 * de-duplicated rows.  Frees the edge buffer. */
static kg_graph* kg_to_csr(int32_t n, kg_edges* e, const int32_t* perm) {
  kg_graph* g = (kg_graph*)calloc(1, sizeof(kg_graph));
  int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  if (!g || !cnt) { free(g); free(cnt); free(e->uv); return NULL; }
  for (int64_t k = 0; k < e->len; k++) {
    int32_t u = e->uv[2 * k], v = e->uv[2 * k + 1];
    if (perm) { u = perm[u]; v = perm[v]; e->uv[2 * k] = u; e->uv[2 * k + 1] = v; }
    cnt[u + 1]++; cnt[v + 1]++;
  }
  for (int32_t i = 0; i < n; i++) cnt[i + 1] += cnt[i];
  int64_t total = cnt[n];
  if (total >= 2147483647LL) { free(cnt); free(g); free(e->uv); return NULL; }
  int32_t* col = (int32_t*)malloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1));
  int64_t* pos = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  if (!col || !pos) { free(col); free(pos); free(cnt); free(g); free(e->uv); return NULL; }
  for (int32_t i = 0; i < n; i++) pos[i] = cnt[i];
  for (int64_t k = 0; k < e->len; k++) {
    int32_t u = e->uv[2 * k], v = e->uv[2 * k + 1];
    col[pos[u]++] = v; col[pos[v]++] = u;
  }
  free(e->uv); e->uv = NULL; e->len = e->cap = 0;
  /* sort rows, drop duplicates, compact */
  int32_t* rp = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
  int64_t w = 0;
  rp[0] = 0;
  for (int32_t i = 0; i < n; i++) {
    int64_t b = cnt[i], len = cnt[i + 1] - cnt[i];
    qsort(col + b, (size_t)len, sizeof(int32_t), cmp_i32);
    int32_t last = -1;
    for (int64_t k = 0; k < len; k++) {
      int32_t c = col[b + k];
      if (c == i || c == last) continue;
      col[w++] = c; last = c;
    }
    rp[i + 1] = (int32_t)w;
  }
  free(pos); free(cnt);
  g->n = n; g->nnz = w; g->row_ptr = rp;
  g->col = (int32_t*)realloc(col, sizeof(int32_t) * (size_t)(w > 0 ? w : 1));
  return g;
}

static int32_t* kg_random_perm(int32_t n, kg_rng* r) {
  int32_t* p = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  if (!p) return NULL;
  for (int32_t i = 0; i < n; i++) p[i] = i;
  for (int32_t i = n - 1; i > 0; i--) {
    int32_t j = (int32_t)kg_below(r, (uint64_t)i + 1);
    int32_t t = p[i]; p[i] = p[j]; p[j] = t;
  }
  return p;
}

/* pair index m in [0, s(s-1)/2) -> (i, j), 0 <= i < j < s, ordered by j */
static void kg_pair(int64_t m, int32_t* i, int32_t* j) {
  int64_t jj = (int64_t)((1.0 + sqrt(1.0 + 8.0 * (double)m)) * 0.5);
  while (jj * (jj - 1) / 2 > m) jj--;
  while ((jj + 1) * jj / 2 <= m) jj++;
  *j = (int32_t)jj;
  *i = (int32_t)(m - jj * (jj - 1) / 2);
}

/* Geometric skipping over N Bernoulli(p) trials; calls emit for successes. */
typedef int (*kg_emit_fn)(void* ctx, int64_t m);
static int kg_skip(int64_t N, double p, kg_rng* r, kg_emit_fn emit, void* ctx) {
  if (N <= 0 || p <= 0.0) return 0;
  if (p >= 1.0) {
    for (int64_t m = 0; m < N; m++) if (emit(ctx, m)) return -1;
    return 0;
  }
  double lq = log1p(-p);
  int64_t m = -1;
  for (;;) {
    double skip = floor(log(kg_unif(r)) / lq);
    if (skip >= (double)N) break;
    m += (int64_t)skip + 1;
    if (m >= N) break;
    if (emit(ctx, m)) return -1;
  }
  return 0;
}

typedef struct {
  kg_edges* e;
  int32_t off;              /* node offset of the block (intra) */
  const int32_t* block_of;  /* node -> block (inter) */
} kg_sbm_ctx;

static int kg_emit_intra(void* vctx, int64_t m) {
  kg_sbm_ctx* c = (kg_sbm_ctx*)vctx;
  int32_t i, j;
  kg_pair(m, &i, &j);
  return kg_push(c->e, c->off + i, c->off + j);
}
static int kg_emit_inter(void* vctx, int64_t m) {
  kg_sbm_ctx* c = (kg_sbm_ctx*)vctx;
  int32_t i, j;
  kg_pair(m, &i, &j);
  if (c->block_of[i] == c->block_of[j]) return 0; /* intra pairs use p_in */
  return kg_push(c->e, i, j);
}

/* Stochastic block model.  Block c holds sizes[c] consecutive nodes before
 * relabelling; each intra pair is an edge with probability p_in[c] and each
 * inter pair with probability p_out, independently. */
kg_graph* kg_sbm(int32_t nblocks, const int32_t* sizes, const double* p_in, double p_out,
                 uint64_t seed, int relabel) {
  kg_rng r = {seed};
  int64_t n64 = 0;
  for (int32_t c = 0; c < nblocks; c++) n64 += sizes[c];
  if (n64 <= 0 || n64 >= 2147483647LL) return NULL;
  int32_t n = (int32_t)n64;
  int32_t* block_of = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  if (!block_of) return NULL;
  kg_edges e = {0, 0, NULL};
  kg_sbm_ctx ctx = {&e, 0, block_of};
  int32_t off = 0;
  for (int32_t c = 0; c < nblocks; c++) {
    for (int32_t k = 0; k < sizes[c]; k++) block_of[off + k] = c;
    ctx.off = off;
    int64_t s = sizes[c];
    if (kg_skip(s * (s - 1) / 2, p_in[c], &r, kg_emit_intra, &ctx)) goto fail;
    off += sizes[c];
  }
  if (kg_skip(n64 * (n64 - 1) / 2, p_out, &r, kg_emit_inter, &ctx)) goto fail;
  {
    int32_t* perm = relabel ? kg_random_perm(n, &r) : NULL;
    kg_graph* g = kg_to_csr(n, &e, perm);
    if (g) {
      g->labels = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
      g->ncomm = nblocks;
      for (int32_t v = 0; v < n; v++) g->labels[perm ? perm[v] : v] = block_of[v];
    }
    free(perm); free(block_of);
    return g;
  }
fail:
  free(e.uv); free(block_of);
  return NULL;
}

/* Community sizes: lognormal(mu, sigma) draws, rescaled and rounded so that
 * they sum exactly to n_total, each at least min_size. */
int kg_lognormal_sizes(int32_t ncomm, int32_t n_total, double mu, double sigma,
                       int32_t min_size, uint64_t seed, int32_t* out) {
  if (ncomm <= 0 || (int64_t)ncomm * min_size > n_total) return -1;
  kg_rng r = {seed};
  double* x = (double*)malloc(sizeof(double) * (size_t)ncomm);
  if (!x) return -1;
  double sum = 0;
  for (int32_t c = 0; c < ncomm; c++) { x[c] = exp(mu + sigma * kg_normal(&r)); sum += x[c]; }
  int64_t tot = 0;
  for (int32_t c = 0; c < ncomm; c++) {
    int64_t s = (int64_t)llround(x[c] * (double)n_total / sum);
    if (s < min_size) s = min_size;
    out[c] = (int32_t)s; tot += s;
  }
  /* fix the rounding drift on the largest communities (deterministic) */
  while (tot != n_total) {
    int32_t best = 0;
    for (int32_t c = 1; c < ncomm; c++) if (out[c] > out[best]) best = c;
    if (tot > n_total) {
      int64_t d = tot - n_total, room = out[best] - min_size;
      int64_t t = d < room ? d : room;
      if (t <= 0) { free(x); return -1; }
      out[best] -= (int32_t)t; tot -= t;
    } else {
      out[best] += (int32_t)(n_total - tot); tot = n_total;
    }
  }
  free(x);
  return 0;
}

/* Power-law expected-degree weights w_i ~ (i + 1)^(-1/(gamma-1)), i = 0..n-1
 * (non-increasing), scaled to sum n*mean_deg and capped at sqrt(n*mean_deg). */
static void kg_powerlaw_weights(int32_t n, double gamma, double mean_deg, double* w) {
  double ex = -1.0 / (gamma - 1.0);
  double target = (double)n * mean_deg, cap = sqrt(target);
  for (int32_t i = 0; i < n; i++) w[i] = pow((double)i + 1.0, ex);
  for (int it = 0; it < 8; it++) {
    double s = 0;
    for (int32_t i = 0; i < n; i++) s += w[i];
    double f = target / s;
    for (int32_t i = 0; i < n; i++) { w[i] *= f; if (w[i] > cap) w[i] = cap; }
  }
}

/* Chung-Lu edges among nodes ids[0..m) with non-increasing weights w[0..m):
 * pair (a, b) is an edge with probability min(1, w_a w_b / S). */
static int kg_chung_lu_core(int32_t m, const double* w, double S, const int32_t* ids,
                            kg_rng* r, kg_edges* e, const int32_t* block_of) {
  for (int32_t u = 0; u + 1 < m; u++) {
    int32_t v = u + 1;
    double p = w[u] * w[v] / S;
    if (p > 1.0) p = 1.0;
    while (v < m && p > 0.0) {
      if (p != 1.0) {
        double sk = floor(log(kg_unif(r)) / log1p(-p));
        if (sk >= (double)(m - v)) break;
        v += (int32_t)sk;
      }
      if (v >= m) break;
      double q = w[u] * w[v] / S;
      if (q > 1.0) q = 1.0;
      if (kg_unif(r) < q / p) {
        int32_t a = ids ? ids[u] : u, b = ids ? ids[v] : v;
        if (!block_of || block_of[a] != block_of[b])
          if (kg_push(e, a, b)) return -1;
      }
      p = q;
      v++;
    }
  }
  return 0;
}

/* Chung-Lu power-law graph on n nodes. */
kg_graph* kg_chung_lu(int32_t n, double gamma, double mean_deg, uint64_t seed, int relabel) {
  if (n <= 1 || gamma <= 1.0 || mean_deg <= 0) return NULL;
  kg_rng r = {seed};
  double* w = (double*)malloc(sizeof(double) * (size_t)n);
  if (!w) return NULL;
  kg_powerlaw_weights(n, gamma, mean_deg, w);
  double S = 0;
  for (int32_t i = 0; i < n; i++) S += w[i];
  kg_edges e = {0, 0, NULL};
  if (kg_chung_lu_core(n, w, S, NULL, &r, &e, NULL)) { free(w); free(e.uv); return NULL; }
  free(w);
  int32_t* perm = relabel ? kg_random_perm(n, &r) : NULL;
  kg_graph* g = kg_to_csr(n, &e, perm);
  free(perm);
  return g;
}

/* Degree-corrected SBM hybrid.  Communities have the given sizes; node weights
 * follow the power law (gamma) over all n nodes, assigned to nodes in a
 * seeded random order.  A fraction f_in of each node's expected degree is
 * realised as Chung-Lu inside its community and the rest as a global Chung-Lu
 * layer restricted to inter-community pairs. */
kg_graph* kg_dcsbm(int32_t ncomm, const int32_t* sizes, double gamma, double mean_deg,
                   double f_in, uint64_t seed, int relabel) {
  kg_rng r = {seed};
  int64_t n64 = 0;
  for (int32_t c = 0; c < ncomm; c++) n64 += sizes[c];
  if (n64 <= 1 || n64 >= 2147483647LL) return NULL;
  int32_t n = (int32_t)n64;
  double* wsorted = (double*)malloc(sizeof(double) * (size_t)n);
  double* wnode = (double*)malloc(sizeof(double) * (size_t)n);
  int32_t* block_of = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* order = NULL;
  double* wl = NULL;
  int32_t* ids = NULL;
  kg_edges e = {0, 0, NULL};
  if (!wsorted || !wnode || !block_of) goto fail;
  kg_powerlaw_weights(n, gamma, mean_deg, wsorted);
  order = kg_random_perm(n, &r); /* node order[i] receives the i-th largest weight */
  if (!order) goto fail;
  for (int32_t i = 0; i < n; i++) wnode[order[i]] = wsorted[i];
  {
    int32_t off = 0;
    for (int32_t c = 0; c < ncomm; c++) {
      for (int32_t k = 0; k < sizes[c]; k++) block_of[off + k] = c;
      off += sizes[c];
    }
  }
  wl = (double*)malloc(sizeof(double) * (size_t)n);
  ids = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  if (!wl || !ids) goto fail;
  /* intra-community layer: per community, nodes sorted by weight */
  {
    int32_t off = 0;
    for (int32_t c = 0; c < ncomm; c++) {
      int32_t s = sizes[c];
      /* selection of this community's nodes in descending weight order:
       * nodes off..off+s-1; sort ids by wnode descending (insertion sort on
       * small s, qsort-free to keep determinism obvious) */
      for (int32_t k = 0; k < s; k++) ids[k] = off + k;
      /* shell sort by descending weight, ties by id */
      for (int32_t gap = s / 2; gap > 0; gap /= 2)
        for (int32_t a = gap; a < s; a++) {
          int32_t t = ids[a];
          int32_t b = a;
          while (b >= gap && (wnode[ids[b - gap]] < wnode[t] ||
                              (wnode[ids[b - gap]] == wnode[t] && ids[b - gap] > t))) {
            ids[b] = ids[b - gap]; b -= gap;
          }
          ids[b] = t;
        }
      double S = 0;
      for (int32_t k = 0; k < s; k++) { wl[k] = f_in * wnode[ids[k]]; S += wl[k]; }
      if (s > 1 && S > 0)
        if (kg_chung_lu_core(s, wl, S, ids, &r, &e, NULL)) goto fail;
      off += s;
    }
  }
  /* inter-community layer over all nodes in descending weight order */
  {
    double S = 0;
    for (int32_t i = 0; i < n; i++) { ids[i] = order[i]; wl[i] = (1.0 - f_in) * wsorted[i]; S += wl[i]; }
    if (S > 0 && kg_chung_lu_core(n, wl, S, ids, &r, &e, block_of)) goto fail;
  }
  {
    int32_t* perm = relabel ? kg_random_perm(n, &r) : NULL;
    kg_graph* g = kg_to_csr(n, &e, perm);
    if (g) {
      g->labels = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
      g->ncomm = ncomm;
      for (int32_t v = 0; v < n; v++) g->labels[perm ? perm[v] : v] = block_of[v];
    }
    free(perm); free(wsorted); free(wnode); free(block_of); free(order); free(wl); free(ids);
    return g;
  }
fail:
  free(e.uv); free(wsorted); free(wnode); free(block_of); free(order); free(wl); free(ids);
  return NULL;
}

/* k distinct query nodes drawn uniformly from the nodes of degree >= 1,
 * in draw order.  Returns the number written (less than k only when fewer
 * candidates exist). */
int32_t kg_sample_queries(const kg_graph* g, int32_t k, uint64_t seed, int32_t* out) {
  kg_rng r = {seed};
  int32_t m = 0;
  int32_t* cand = (int32_t*)malloc(sizeof(int32_t) * (size_t)(g->n > 0 ? g->n : 1));
  if (!cand) return -1;
  for (int32_t v = 0; v < g->n; v++)
    if (g->row_ptr[v + 1] > g->row_ptr[v]) cand[m++] = v;
  if (k > m) k = m;
  for (int32_t i = 0; i < k; i++) { /* partial Fisher-Yates */
    int32_t j = i + (int32_t)kg_below(&r, (uint64_t)(m - i));
    int32_t t = cand[i]; cand[i] = cand[j]; cand[j] = t;
    out[i] = cand[i];
  }
  free(cand);
  return k;
}

/* Wraps caller-provided CSR arrays (copied) so kg_sample_queries can run on
 * graphs that were not generated here (tiny hand-made graphs in tests). */
kg_graph* kg_wrap_csr(int32_t n, const int32_t* row_ptr, const int32_t* col) {
  kg_graph* g = (kg_graph*)calloc(1, sizeof(kg_graph));
  if (!g) return NULL;
  g->n = n; g->nnz = row_ptr[n];
  g->row_ptr = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
  g->col = (int32_t*)malloc(sizeof(int32_t) * (size_t)(g->nnz > 0 ? g->nnz : 1));
  if (!g->row_ptr || !g->col) { kg_graph_free(g); return NULL; }
  memcpy(g->row_ptr, row_ptr, sizeof(int32_t) * ((size_t)n + 1));
  memcpy(g->col, col, sizeof(int32_t) * (size_t)g->nnz);
  return g;
}
