// Host-side index construction (Algorithm 1; Sec. 3.2 steps 1-4).
//
//  1. validate the CSR and compute lambda_max(A) (Lanczos) to fix beta;
//  2. partition: initial parts (caller labels, or BFS growing), each part cut
//     into BFS-ordered chunks of at most max_block nodes; a greedy vertex
//     cover of the cut edges becomes the separator, so the remaining blocks
//     have no edges between them and M11 is block diagonal (Lemma 1);
//  3. reorder: blocks contiguous (largest first), separator last;
//  4. factor every block M_bb = I - beta A_bb = L1 L1^T and store
//     M_bb^{-1} = L1^{-T} L1^{-1}; factor M22 when L is its Cholesky factor;
//  5. Lanczos with full reorthogonalisation on R = I - L^{-1} S L^{-T}
//     (eq. RMatrix; R is only applied, never formed) for the top r pairs.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <thread>

#include "katz_internal.h"

namespace katz {

void fail(int code, const std::string& msg) { throw Error{code, msg}; }

int host_threads() {
  static int n = [] {
    unsigned h = std::thread::hardware_concurrency();
    const char* e = getenv("KATZ_HOST_THREADS");
    if (e && atoi(e) > 0) return atoi(e);
    return (int)std::max(1u, std::min(h, 64u));
  }();
  return n;
}

void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)>& fn, int64_t grain) {
  if (n <= 0) return;
  int T = host_threads();
  int64_t chunks = (n + grain - 1) / grain;
  if (T <= 1 || chunks <= 1) { fn(0, n); return; }
  std::atomic<int64_t> next{0};
  auto work = [&] {
    for (;;) {
      int64_t c = next.fetch_add(1);
      if (c >= chunks) break;
      int64_t b = c * grain, e = std::min(n, b + grain);
      fn(b, e);
    }
  };
  int nt = (int)std::min<int64_t>(T, chunks);
  std::vector<std::thread> th;
  for (int t = 1; t < nt; t++) th.emplace_back(work);
  work();
  for (auto& t : th) t.join();
}

namespace {

// ------------------------------------------------------------ SplitMix64
struct Rng {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
  }
  double unif() { return ((double)(next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
  double normal() { return std::sqrt(-2.0 * std::log(unif())) * std::cos(6.283185307179586 * unif()); }
};

double dot(const double* a, const double* b, int64_t n) {
  int T = host_threads();
  if (n < 200000 || T == 1) {
    double s = 0;
    for (int64_t i = 0; i < n; i++) s += a[i] * b[i];
    return s;
  }
  const int64_t grain = 65536;
  int64_t chunks = (n + grain - 1) / grain;
  std::vector<double> part(chunks, 0.0);
  parallel_for(chunks, [&](int64_t c0, int64_t c1) {
    for (int64_t c = c0; c < c1; c++) {
      double s = 0;
      int64_t lo = c * grain, hi = std::min(n, lo + grain);
      for (int64_t i = lo; i < hi; i++) s += a[i] * b[i];
      part[c] = s;
    }
  }, 1);
  double s = 0;
  for (double v : part) s += v;
  return s;
}

// ------------------------------------------------ symmetric tridiagonal
// Eigen-decomposition of the symmetric tridiagonal T with diagonal d[0..m)
// and off-diagonal e[0..m-1) by the symmetric QR algorithm: implicit QR
// steps with the Wilkinson shift, applied as a chase of the bulge down the
// unreduced window by plane rotations, with deflation of negligible
// off-diagonal entries (Golub & Van Loan, Matrix Computations, 4th ed.,
// Sec. 8.3, Algorithms 8.3.2 and 8.3.3).  On return d holds the eigenvalues
// (unsorted) and z (m x m, row-major, z[row*m + k]) the orthonormal
// eigenvectors as columns (the product of all rotations).
namespace {

// Negligible off-diagonal entry: |e_i| <= u (|d_i| + |d_{i+1}|).
inline bool negligible(const std::vector<double>& d, const std::vector<double>& e, int i) {
  return std::fabs(e[i]) <= 2.220446049250313e-16 * (std::fabs(d[i]) + std::fabs(d[i + 1]));
}

// One implicit QR step on the unreduced window [lo, hi] of (d, e).  The shift
// mu is the eigenvalue of the trailing 2x2 block closer to its last diagonal
// entry.  The first rotation takes (d_lo - mu, e_lo) to (r, 0); each later
// rotation in plane (k, k+1) removes the bulge at T(k-1, k+1) that the
// previous one created, until the bulge leaves the window.  Every rotation
// R = [[c, s], [-s, c]] acts as T <- R T R^T and is accumulated as z <- z R^T.
void qr_step(std::vector<double>& d, std::vector<double>& e, std::vector<double>& z, int m, int lo, int hi) {
  const double t = e[hi - 1];
  const double delta = 0.5 * (d[hi - 1] - d[hi]);
  const double root = std::hypot(delta, t);
  const double mu = d[hi] - t * t / (delta + (delta >= 0.0 ? root : -root));
  double x = d[lo] - mu, y = e[lo];
  for (int k = lo; k < hi; k++) {
    const double r = std::hypot(x, y);
    const double c = r > 0.0 ? x / r : 1.0, s = r > 0.0 ? y / r : 0.0;
    if (k > lo) e[k - 1] = r;  // T(k-1, k) = r, the bulge T(k-1, k+1) = 0
    const double a0 = d[k], a1 = d[k + 1], b = e[k];
    d[k] = c * c * a0 + 2.0 * c * s * b + s * s * a1;
    d[k + 1] = s * s * a0 - 2.0 * c * s * b + c * c * a1;
    e[k] = c * s * (a1 - a0) + (c * c - s * s) * b;
    if (k + 1 < hi) {
      // rows k and k+1 mixed into column k+2: a new bulge at T(k, k+2)
      x = e[k];
      y = s * e[k + 1];
      e[k + 1] *= c;
    }
    for (int i = 0; i < m; i++) {
      double* zi = &z[(size_t)i * m];
      const double u = zi[k], v = zi[k + 1];
      zi[k] = c * u + s * v;
      zi[k + 1] = c * v - s * u;
    }
  }
}

}  // namespace

void tridiag_eig(std::vector<double>& d, std::vector<double> e, std::vector<double>& z, int m) {
  z.assign((size_t)m * m, 0.0);
  for (int i = 0; i < m; i++) z[(size_t)i * m + i] = 1.0;
  e.resize(std::max(m, 1), 0.0);
  int hi = m - 1, steps = 0;
  while (hi > 0) {
    if (negligible(d, e, hi - 1)) {  // d[hi] has converged
      e[hi - 1] = 0.0;
      hi--;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && !negligible(d, e, lo - 1)) lo--;
    if (lo > 0) e[lo - 1] = 0.0;
    if (++steps > 60 * std::max(m, 1)) fail(KATZ_EINVAL, "tridiagonal eigensolver did not converge");
    qr_step(d, e, z, m, lo, hi);
  }
}

// --------------------------------------------------------- dense helpers
// In-place lower Cholesky of the b x b row-major SPD matrix a (column by
// column; the rows below the diagonal of a column are independent and run in
// parallel for large b).
bool chol_lower(double* a, int b) {
  const bool par = b > 256;
  for (int j = 0; j < b; j++) {
    double s = a[(size_t)j * b + j];
    const double* aj = &a[(size_t)j * b];
    for (int k = 0; k < j; k++) s -= aj[k] * aj[k];
    if (!(s > 0.0)) return false;
    const double ljj = std::sqrt(s);
    a[(size_t)j * b + j] = ljj;
    auto rows = [&](int64_t i0, int64_t i1) {
      for (int64_t i = i0; i < i1; i++) {
        double* ai = &a[(size_t)i * b];
        double t = ai[j];
        for (int k = 0; k < j; k++) t -= ai[k] * aj[k];
        ai[j] = t / ljj;
      }
    };
    if (par) parallel_for(b - j - 1, [&](int64_t i0, int64_t i1) { rows(j + 1 + i0, j + 1 + i1); }, 64);
    else rows(j + 1, b);
  }
  for (int j = 0; j < b; j++)
    for (int k = j + 1; k < b; k++) a[(size_t)j * b + k] = 0.0;
  return true;
}

// Incomplete Cholesky with zero fill, IC(0), of the m x m row-major
// symmetric matrix a (lower triangle read), in place: the lower factor keeps
// the sparsity pattern of a's lower triangle, and fill outside it is dropped
// instead of stored.  Row i: l[i][k] = (a[i][k] - sum_j l[i][j] l[k][j]) /
// l[k][k] for k in the row's pattern (j over the pattern entries before k;
// entries of row k outside its own pattern are zero), then l[i][i] =
// sqrt(a[i][i] - sum_j l[i][j]^2).  The factor exists for symmetric
// M-matrices such as M22 = I - beta A22 (Meijerink and van der Vorst, 1977).
// Returns false on a nonpositive pivot.
bool ic0_lower(double* a, int m) {
  std::vector<std::vector<int>> pat(m);
  for (int i = 0; i < m; i++)
    for (int j = 0; j < i; j++)
      if (a[(size_t)i * m + j] != 0.0) pat[i].push_back(j);
  for (int i = 0; i < m; i++) {
    double* ai = &a[(size_t)i * m];
    const std::vector<int>& pi = pat[i];
    for (size_t t = 0; t < pi.size(); t++) {
      const int k = pi[t];
      const double* ak = &a[(size_t)k * m];
      double s = ai[k];
      for (size_t u = 0; u < t; u++) s -= ai[pi[u]] * ak[pi[u]];
      ai[k] = s / ak[k];
    }
    double d = ai[i];
    for (int j : pi) d -= ai[j] * ai[j];
    if (!(d > 0.0)) return false;
    ai[i] = std::sqrt(d);
  }
  for (int j = 0; j < m; j++)
    for (int k = j + 1; k < m; k++) a[(size_t)j * m + k] = 0.0;
  return true;
}

// Given the lower factor l (b x b), writes inv = (l l^T)^{-1} (full,
// symmetric): column j of l^{-1} is stored as row j of w (forward
// substitution on contiguous rows), then inv[i][j] = <w row i, w row j>.
void chol_inverse(const double* l, int b, double* inv, std::vector<double>& w) {
  w.assign((size_t)b * b, 0.0);
  const int64_t grain = b > 256 ? 16 : b;
  parallel_for(b, [&](int64_t j0, int64_t j1) {
    for (int64_t j = j0; j < j1; j++) {
      double* x = &w[(size_t)j * b];
      x[j] = 1.0 / l[(size_t)j * b + j];
      for (int i = (int)j + 1; i < b; i++) {
        const double* li = &l[(size_t)i * b];
        double s = 0;
        for (int k = (int)j; k < i; k++) s += li[k] * x[k];
        x[i] = -s / li[i];
      }
    }
  }, grain);
  parallel_for(b, [&](int64_t i0, int64_t i1) {
    for (int64_t i = i0; i < i1; i++) {
      const double* wi = &w[(size_t)i * b];
      for (int64_t j = 0; j <= i; j++) {
        const double* wj = &w[(size_t)j * b];
        double s = 0;
        for (int k = (int)i; k < b; k++) s += wi[k] * wj[k];
        inv[(size_t)i * b + j] = s;
        inv[(size_t)j * b + i] = s;
      }
    }
  }, grain);
}

// ------------------------------------------------------------ validation
void validate(int32_t n, int64_t nnz, const int32_t* rp, const int32_t* col, const double* val) {
  if (n <= 0) fail(KATZ_EINVAL, "n must be positive");
  if (!rp || (nnz > 0 && !col)) fail(KATZ_EINVAL, "null CSR array");
  if (nnz < 0 || nnz >= INT32_MAX) fail(KATZ_EINVAL, "nnz must be in [0, 2^31-1)");
  if (rp[0] != 0 || rp[n] != nnz) fail(KATZ_EINVAL, "row_ptr must start at 0 and end at nnz");
  // every row pointer first: non-decreasing from 0 to nnz keeps each row's
  // range, and the partner rows the symmetry check searches, inside col
  std::atomic<int> bad{0};
  parallel_for(n, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; i++)
      if (rp[i + 1] < rp[i]) { bad = 1; break; }
  }, 8192);
  if (bad.load()) fail(KATZ_EINVAL, "row_ptr is not non-decreasing");
  // symmetry: every entry (i, j) above the diagonal has its partner (j, i)
  // with the same value (a binary search in row j), and there are as many
  // entries below the diagonal as above.  The partners of distinct upper
  // entries are distinct lower entries, so equal counts make every lower
  // entry a partner: one search per pair instead of one per entry.
  std::atomic<int> asym{0};
  std::atomic<int64_t> n_upper{0}, n_lower{0};
  parallel_for(n, [&](int64_t b, int64_t e) {
    int64_t up = 0, lo = 0;
    for (int64_t i = b; i < e && !bad.load(std::memory_order_relaxed); i++) {
      int32_t s = rp[i], t = rp[i + 1];
      int32_t last = -1;
      for (int32_t k = s; k < t; k++) {
        int32_t j = col[k];
        if (j < 0 || j >= n) { bad = 2; break; }
        if (j <= last) { bad = 3; break; }
        if (j == i) { bad = 4; break; }
        if (val && !(val[k] >= 0.0 && std::isfinite(val[k]))) { bad = 5; break; }
        last = j;
        if (j < i) { lo++; continue; }
        up++;
        const int32_t* rb = col + rp[j];
        const int32_t* re = col + rp[j + 1];
        const int32_t* f = std::lower_bound(rb, re, (int32_t)i);
        if (f == re || *f != i || (val && val[f - col] != val[k])) asym = 1;
      }
    }
    n_upper += up;
    n_lower += lo;
  }, 2048);
  if (n_upper.load() != n_lower.load()) asym = 1;
  switch (bad.load()) {
    case 2: fail(KATZ_EINVAL, "column index out of range");
    case 3: fail(KATZ_EINVAL, "columns must be strictly increasing within a row");
    case 4: fail(KATZ_EINVAL, "diagonal entries (self loops) are not allowed");
    case 5: fail(KATZ_EINVAL, "values must be finite and nonnegative");
    default: break;
  }
  if (asym) fail(KATZ_ENOTSYM, "adjacency matrix is not symmetric");
}

// y = A x for the caller's CSR (original order)
void spmv(int32_t n, const int32_t* rp, const int32_t* col, const double* val, const double* x, double* y) {
  parallel_for(n, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; i++) {
      double s = 0;
      if (val)
        for (int32_t k = rp[i]; k < rp[i + 1]; k++) s += val[k] * x[col[k]];
      else
        for (int32_t k = rp[i]; k < rp[i + 1]; k++) s += x[col[k]];
      y[i] = s;
    }
  }, 8192);
}

// The vector work of lambda_max on the host: q, the previous vector qp and w
// in host memory, the products and sums on all host cores.
struct HostLambdaOps : LambdaOps {
  int32_t n;
  const int32_t *rp, *col;
  const double* val;
  std::vector<double> q, qp, w;
  HostLambdaOps(int32_t n_, const int32_t* rp_, const int32_t* col_, const double* val_)
      : n(n_), rp(rp_), col(col_), val(val_), q(n_), qp(n_, 0.0), w(n_) {}
  void start(const double* q0) override { std::copy(q0, q0 + n, q.begin()); }
  double apply_dot() override {
    spmv(n, rp, col, val, q.data(), w.data());
    return dot(q.data(), w.data(), n);
  }
  double update_norm2(double a, double bprev) override {
    parallel_for(n, [&](int64_t b, int64_t e) {
      for (int64_t i = b; i < e; i++) w[i] -= a * q[i] + bprev * qp[i];
    });
    return dot(w.data(), w.data(), n);
  }
  void advance(double bj) override {
    qp.swap(q);  // the previous vector; q = w / bj
    parallel_for(n, [&](int64_t lo, int64_t hi) {
      for (int64_t i = lo; i < hi; i++) q[i] = w[i] / bj;
    });
  }
};

}  // namespace

// Largest eigenvalue of A by Lanczos without reorthogonalisation (the top Ritz
// value is unaffected by the loss of orthogonality, which only duplicates
// converged values), the vector work done by `ops`.  Stops when the Ritz
// residual bound is below 1e-13 of the Ritz value.
double lambda_max_with(int32_t n, uint64_t seed, LambdaOps& ops) {
  std::vector<double> q(n);
  Rng rng{seed ^ 0x5A5A5A5AULL};
  for (int32_t i = 0; i < n; i++) q[i] = 0.5 + rng.unif();  // positive start: overlaps the Perron vector
  double nq = std::sqrt(dot(q.data(), q.data(), n));
  for (auto& v : q) v /= nq;
  ops.start(q.data());
  std::vector<double>().swap(q);
  std::vector<double> al, be;
  double theta = 0, bprev = 0;
  const int mmax = std::min<int64_t>(600, n);
  for (int j = 0; j < mmax; j++) {
    const double a = ops.apply_dot();
    const double bj = std::sqrt(ops.update_norm2(a, bprev));
    al.push_back(a);
    be.push_back(bj);
    int m = (int)al.size();
    if (m % 8 == 0 || bj <= 1e-14 * std::fabs(a) || j == mmax - 1) {
      std::vector<double> d(al), z;
      std::vector<double> e(be.begin(), be.end() - 1);
      tridiag_eig(d, e, z, m);
      int top = (int)(std::max_element(d.begin(), d.end()) - d.begin());
      theta = d[top];
      double resid = bj * std::fabs(z[(size_t)(m - 1) * m + top]);
      if (resid <= 1e-13 * std::fabs(theta) || bj <= 1e-14 * std::fabs(a)) break;
    }
    if (bj == 0.0) break;
    ops.advance(bj);
    bprev = bj;
  }
  return theta;
}

namespace {

double lambda_max(int32_t n, const int32_t* rp, const int32_t* col, const double* val, uint64_t seed) {
  if (rp[n] == 0) return 0.0;
  HostLambdaOps ops(n, rp, col, val);
  return lambda_max_with(n, seed, ops);
}

// ------------------------------------------------------------- partition
struct Partition {
  std::vector<int32_t> perm, iperm, blk_start;
  int32_t n1 = 0, n2 = 0;
  double seconds[5] = {0};  // BFS chunks, vertex cover, minimality, components, order
};

// Node marks are read across the parts that the BFS orders of different
// parts visit at once (a neighbour in another part never carries this part's
// tag, whichever of its two values a concurrent BFS leaves there): relaxed
// atomic accesses.
inline int32_t mark_get(const std::vector<int32_t>& m, int32_t v) { return __atomic_load_n(&m[v], __ATOMIC_RELAXED); }
inline void mark_set(std::vector<int32_t>& m, int32_t v, int32_t x) { __atomic_store_n(&m[v], x, __ATOMIC_RELAXED); }

// Frontiers at least this large are expanded on all host cores.
constexpr size_t kParFrontier = 16384;

// Appends to `out` the BFS order from s over the nodes with mark == tag (and
// marks them tag + 1): frontier by frontier, each frontier node in order
// appends its unreached neighbours in CSR order, and a node adjacent to
// several frontier nodes goes to the first of them -- the order of a FIFO
// queue.  Large frontiers run in parallel with that rule made explicit:
// claim[v] = the smallest frontier position that reaches v (claim holds
// INT32_MAX outside a call), then each frontier node writes the nodes it
// claimed at its prefix-sum offset.  `par`: whether parallel expansion is
// allowed (false inside a parallel loop over parts).
void bfs_levels(const int32_t* rp, const int32_t* col, std::vector<int32_t>& mark, int32_t tag, int32_t s,
                std::vector<int32_t>& out, std::vector<int32_t>& claim, bool par) {
  size_t f0 = out.size();
  out.push_back(s);
  mark_set(mark, s, tag + 1);
  std::vector<int64_t> off;
  while (f0 < out.size()) {
    const size_t f1 = out.size(), fn = f1 - f0;
    if (!par || fn < kParFrontier || host_threads() <= 1) {
      for (size_t h = f0; h < f1; h++) {
        const int32_t u = out[h];
        for (int32_t k = rp[u]; k < rp[u + 1]; k++) {
          const int32_t v = col[k];
          if (mark_get(mark, v) == tag) { mark_set(mark, v, tag + 1); out.push_back(v); }
        }
      }
      f0 = f1;
      continue;
    }
    // claim: the first frontier position reaching each unreached node
    parallel_for((int64_t)fn, [&](int64_t b, int64_t e) {
      for (int64_t t = b; t < e; t++) {
        const int32_t u = out[f0 + t];
        for (int32_t k = rp[u]; k < rp[u + 1]; k++) {
          const int32_t v = col[k];
          if (mark_get(mark, v) != tag) continue;
          int32_t cur = __atomic_load_n(&claim[v], __ATOMIC_RELAXED);
          while ((int32_t)t < cur &&
                 !__atomic_compare_exchange_n(&claim[v], &cur, (int32_t)t, true, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) {
          }
        }
      }
    }, 1024);
    // count and place each frontier node's claims in CSR order
    off.assign(fn + 1, 0);
    parallel_for((int64_t)fn, [&](int64_t b, int64_t e) {
      for (int64_t t = b; t < e; t++) {
        const int32_t u = out[f0 + t];
        int64_t c = 0;
        for (int32_t k = rp[u]; k < rp[u + 1]; k++) c += claim[col[k]] == (int32_t)t;
        off[t + 1] = c;
      }
    }, 1024);
    for (size_t t = 0; t < fn; t++) off[t + 1] += off[t];
    out.resize(f1 + (size_t)off[fn]);
    parallel_for((int64_t)fn, [&](int64_t b, int64_t e) {
      for (int64_t t = b; t < e; t++) {
        const int32_t u = out[f0 + t];
        size_t at = f1 + (size_t)off[t];
        for (int32_t k = rp[u]; k < rp[u + 1]; k++)
          if (claim[col[k]] == (int32_t)t) out[at++] = col[k];
      }
    }, 1024);
    parallel_for((int64_t)(out.size() - f1), [&](int64_t b, int64_t e) {
      for (int64_t t = b; t < e; t++) {
        const int32_t v = out[f1 + t];
        mark_set(mark, v, tag + 1);
        claim[v] = INT32_MAX;
      }
    }, 16384);
    f0 = f1;
  }
}

// BFS order of the nodes of `nodes` (a set marked by mark[v] == tag),
// restarting from the lowest unvisited node; the BFS of each component starts
// from a pseudo-peripheral node (the last node reached by a BFS from the
// seed).  Visited nodes end with mark tag + 1.
void bfs_order(const int32_t* rp, const int32_t* col, const std::vector<int32_t>& nodes,
               std::vector<int32_t>& mark, int32_t tag, std::vector<int32_t>& out,
               std::vector<int32_t>& claim, bool par) {
  out.clear();
  std::vector<int32_t> seen;
  for (int32_t s : nodes) {
    if (mark_get(mark, s) != tag) continue;
    seen.clear();
    bfs_levels(rp, col, mark, tag, s, seen, claim, par);
    const int32_t far = seen.back();
    for (int32_t v : seen) mark_set(mark, v, tag);  // unvisit the component
    bfs_levels(rp, col, mark, tag, far, out, claim, par);
  }
}

Partition make_partition(int32_t n, const int32_t* rp, const int32_t* col, const int32_t* labels,
                         int32_t max_block, int32_t order_kind) {
  const bool verbose = getenv("KATZ_VERBOSE") && atoi(getenv("KATZ_VERBOSE")) > 1;
  auto tp = std::chrono::steady_clock::now();
  double ph[5] = {0};
  int nph = 0;
  auto phase = [&](const char* what) {
    auto t = std::chrono::steady_clock::now();
    const double sec = std::chrono::duration<double>(t - tp).count();
    if (nph < 5) ph[nph++] = sec;
    if (verbose) std::fprintf(stderr, "katz partition: %-20s %8.3f s\n", what, sec);
    tp = t;
  };
  // (a) initial parts
  std::vector<int32_t> part(n);
  int32_t P = 0;
  if (labels) {
    std::vector<int32_t> lab(labels, labels + n);
    std::vector<int32_t> u(lab);
    std::sort(u.begin(), u.end());
    u.erase(std::unique(u.begin(), u.end()), u.end());
    for (int32_t v = 0; v < n; v++) part[v] = (int32_t)(std::lower_bound(u.begin(), u.end(), lab[v]) - u.begin());
    P = (int32_t)u.size();
  } else {
    std::fill(part.begin(), part.end(), 0);
    P = 1;
  }
  // (b) BFS chunking of every part into pieces of <= max_block nodes.  Parts
  // run in parallel (one BFS each) when there are several; one part runs
  // its large frontiers in parallel.  The orders, and so the pieces, are the
  // serial ones.
  std::vector<std::vector<int32_t>> members(P);
  for (int32_t v = 0; v < n; v++) members[part[v]].push_back(v);
  std::vector<int32_t> mark(n), claim(n, INT32_MAX);
  parallel_for(n, [&](int64_t b, int64_t e) {
    for (int64_t v = b; v < e; v++) mark[v] = 2 * part[v];
  }, 65536);
  std::vector<std::vector<int32_t>> orders(P);
  if (P == 1) {
    bfs_order(rp, col, members[0], mark, 0, orders[0], claim, true);
  } else {
    parallel_for(P, [&](int64_t b, int64_t e) {
      for (int64_t p = b; p < e; p++) bfs_order(rp, col, members[p], mark, 2 * (int32_t)p, orders[p], claim, false);
    }, 1);
  }
  std::vector<std::vector<int32_t>>().swap(members);
  std::vector<int32_t> piece(n, -1);
  std::vector<int64_t> visit(n, 0);  // position in the concatenated BFS orders
  std::vector<int64_t> vbase(P + 1, 0), pbase(P + 1, 0);
  for (int32_t p = 0; p < P; p++) {
    vbase[p + 1] = vbase[p] + (int64_t)orders[p].size();
    pbase[p + 1] = pbase[p] + ((int64_t)orders[p].size() + max_block - 1) / max_block;
  }
  parallel_for(P, [&](int64_t b, int64_t e) {
    for (int64_t p = b; p < e; p++) {
      const auto& ord = orders[p];
      for (size_t k = 0; k < ord.size(); k++) {
        piece[ord[k]] = (int32_t)(pbase[p] + (int64_t)(k / (size_t)max_block));
        visit[ord[k]] = vbase[p] + (int64_t)k;
      }
      std::vector<int32_t>().swap(orders[p]);
    }
  }, P > 1 ? 16 : 1);
  int32_t npiece = (int32_t)pbase[P];
  phase("BFS chunks");
  // (c) greedy vertex cover of the cut edges (largest remaining cut degree
  // first; among equal degrees the node listed last, node 0 first at the
  // start).  Each node's piece and remaining cut degree sit side by side (one
  // cache line per neighbour visit), and a cover node's degree is set to -1:
  // a neighbour u of a new cover node v across a cut has pd[u].deg >= 1
  // exactly when u is not in the cover yet.
  struct PD { int32_t piece, deg; };
  std::vector<PD> pd(n);
  parallel_for(n, [&](int64_t b, int64_t e) {  // independent per node
    for (int64_t v = b; v < e; v++) {
      int32_t c = 0;
      const int32_t pv = piece[v];
      for (int32_t k = rp[v]; k < rp[v + 1]; k++) c += piece[col[k]] != pv;
      pd[v] = {pv, c};
    }
  }, 16384);
  int32_t dmax = 0;
  for (int32_t v = 0; v < n; v++) dmax = std::max(dmax, pd[v].deg);
  // one stack per degree; an entry whose node has since moved on is stale
  std::vector<std::vector<int32_t>> bucket(dmax + 1);
  for (int32_t v = n - 1; v >= 0; v--)
    if (pd[v].deg > 0) bucket[pd[v].deg].push_back(v);
  std::vector<int32_t> sep_order;
  for (int32_t d = dmax; d > 0;) {
    if (bucket[d].empty()) { d--; continue; }
    const int32_t v = bucket[d].back();
    bucket[d].pop_back();
    if (pd[v].deg != d) continue;  // stale entry (or already in the cover: -1)
    pd[v].deg = -1;
    sep_order.push_back(v);
    const int32_t pv = pd[v].piece;
    const int32_t k0 = rp[v], k1 = rp[v + 1];
    for (int32_t k = k0; k < std::min(k1, k0 + 16); k++) __builtin_prefetch(&pd[col[k]], 1);
    for (int32_t k = k0; k < k1; k++) {
      if (k + 16 < k1) __builtin_prefetch(&pd[col[k + 16]], 1);
      PD& u = pd[col[k]];
      if (u.deg > 0 && u.piece != pv)
        if (--u.deg > 0) bucket[u.deg].push_back(col[k]);
    }
  }
  std::vector<std::vector<int32_t>>().swap(bucket);
  std::vector<char> insep(n, 0);
  for (int32_t v : sep_order) insep[v] = 1;
  std::vector<PD>().swap(pd);
  phase("vertex cover");
  // (d) minimality: a separator node whose non-separator neighbours all lie in
  // one piece (with room) joins that piece; one with none becomes a singleton.
  std::vector<int32_t> psize(npiece, 0);
  for (int32_t v = 0; v < n; v++) if (!insep[v]) psize[piece[v]]++;
  for (auto it = sep_order.rbegin(); it != sep_order.rend(); ++it) {
    int32_t v = *it;
    int32_t target = -1;
    bool ok = true;
    for (int32_t k = rp[v]; k < rp[v + 1] && ok; k++) {
      int32_t u = col[k];
      if (insep[u]) continue;
      if (target < 0) target = piece[u];
      else if (piece[u] != target) ok = false;
    }
    if (!ok) continue;
    if (target < 0) {
      piece[v] = npiece++;
      psize.push_back(1);
      insep[v] = 0;
    } else if (psize[target] < max_block) {
      piece[v] = target;
      psize[target]++;
      insep[v] = 0;
    }
  }
  phase("minimality");
  // (e) blocks = connected components of the graph without the separator;
  // each lies inside one piece, so it has at most max_block nodes.
  std::vector<int32_t> comp(n, -1);
  std::vector<std::vector<int32_t>> blocks;
  for (int32_t s = 0; s < n; s++) {
    if (insep[s] || comp[s] >= 0) continue;
    int32_t id = (int32_t)blocks.size();
    blocks.emplace_back();
    auto& b = blocks.back();
    b.push_back(s);
    comp[s] = id;
    for (size_t h = 0; h < b.size(); h++) {
      int32_t u = b[h];
      for (int32_t k = rp[u]; k < rp[u + 1]; k++) {
        int32_t v = col[k];
        if (!insep[v] && comp[v] < 0) { comp[v] = id; b.push_back(v); }
      }
    }
  }
  phase("components");
  // Block order.  DEGREE: largest blocks first (a descending work list for the
  // block kernel).  LOCALITY: blocks and their nodes in BFS visit order, so
  // neighbours stay close in every panel.
  const bool locality = order_kind == KATZ_ORDER_LOCALITY;
  const int32_t nbk = (int32_t)blocks.size();
  std::vector<int32_t> bo(nbk);
  std::iota(bo.begin(), bo.end(), 0);
  Partition R;
  R.perm.assign(n, -1);
  R.blk_start.push_back(0);
  std::vector<int32_t> ord;  // LOCALITY: the nodes in BFS visit order
  if (locality) {
    // blocks by their first node in visit order, nodes within a block in
    // visit order: rank the blocks by that key, then place the nodes while
    // walking the visit order (O(n))
    ord.assign(n, -1);
    for (int32_t v = 0; v < n; v++) {
      if (visit[v] < 0 || visit[v] >= n || ord[visit[v]] >= 0) fail(KATZ_EDEVICE, "internal: BFS visit order");
      ord[visit[v]] = v;
    }
    // the visit positions are distinct, so walking the visit order meets
    // the blocks in the order of their first nodes
    std::vector<int32_t> slot(nbk, -1);
    int32_t run = 0, t = 0;
    for (int32_t pos = 0; pos < n; pos++) {
      const int32_t v = ord[pos];
      if (insep[v] || slot[comp[v]] >= 0) continue;
      bo[t++] = comp[v];
      slot[comp[v]] = run;
      run += (int32_t)blocks[comp[v]].size();
      R.blk_start.push_back(run);
    }
    if (t != nbk) fail(KATZ_EDEVICE, "internal: block order");
    R.iperm.assign(run, -1);
    for (int32_t pos = 0; pos < n; pos++) {
      const int32_t v = ord[pos];
      if (insep[v]) continue;
      const int32_t at = slot[comp[v]]++;
      R.perm[v] = at;
      R.iperm[at] = v;
    }
  } else {
    std::stable_sort(bo.begin(), bo.end(), [&](int32_t a, int32_t b) { return blocks[a].size() > blocks[b].size(); });
    R.iperm.reserve(n);
    for (size_t t = 0; t < bo.size(); t++) {
      for (int32_t v : blocks[bo[t]]) { R.perm[v] = (int32_t)R.iperm.size(); R.iperm.push_back(v); }
      R.blk_start.push_back((int32_t)R.iperm.size());
    }
  }
  R.n1 = (int32_t)R.iperm.size();
  // separator order.  DEGREE: largest first, then by id (the hubs, which most
  // adjacency entries point to, share few cache lines of every gathered
  // panel).  LOCALITY: BFS visit order.
  if (locality) {
    for (int32_t pos = 0; pos < n; pos++) {
      const int32_t v = ord[pos];
      if (insep[v]) { R.perm[v] = (int32_t)R.iperm.size(); R.iperm.push_back(v); }
    }
  } else {
    std::vector<std::pair<int64_t, int32_t>> sk;
    for (int32_t v = 0; v < n; v++)
      if (insep[v]) sk.emplace_back(-(int64_t)(rp[v + 1] - rp[v]), v);
    std::sort(sk.begin(), sk.end());
    for (auto& kv : sk) { R.perm[kv.second] = (int32_t)R.iperm.size(); R.iperm.push_back(kv.second); }
  }
  R.n2 = n - R.n1;
  phase("order");
  for (int t = 0; t < 5; t++) R.seconds[t] = ph[t];
  return R;
}

// ----------------------------------------------------- separator operators
// Applies S x = M22 x - M12^T M11^{-1} M12 x on the host (n2-vectors), using
// the permuted CSR: with u = M11^{-1} (beta A12 x),
//   S x = x - beta (A21 u + A22 x).
struct SchurOp {
  const HostIndex& H;
  std::vector<double> t1;  // n1 scratch
  explicit SchurOp(const HostIndex& h) : H(h), t1(h.n1) {}
  void apply(const double* x, double* y) {
    const int32_t n1 = H.n1, n = H.n;
    const double beta = H.beta;
    const bool w = H.weighted;
    // t1 = beta * A12 x, block by block, then t1 <- M11^{-1} t1
    int32_t nb = (int32_t)H.blk_start.size() - 1;
    parallel_for(nb, [&](int64_t b0, int64_t b1) {
      std::vector<double> tmp;
      for (int64_t b = b0; b < b1; b++) {
        int32_t s = H.blk_start[b], e = H.blk_start[b + 1], sz = e - s;
        tmp.assign(sz, 0.0);
        for (int32_t i = s; i < e; i++) {
          double acc = 0;
          for (int32_t k = H.split[i]; k < H.rp[i + 1]; k++) acc += (w ? H.val[k] : 1.0) * x[H.col[k] - n1];
          tmp[i - s] = beta * acc;
        }
        const double* mi = &H.minv[H.blk_off[b]];
        for (int32_t i = 0; i < sz; i++) {
          double acc = 0;
          for (int32_t k = 0; k < sz; k++) acc += mi[(size_t)i * sz + k] * tmp[k];
          t1[s + i] = acc;
        }
      }
    }, 64);
    parallel_for(n - n1, [&](int64_t r0, int64_t r1) {
      for (int64_t r = r0; r < r1; r++) {
        int32_t i = n1 + (int32_t)r;
        double acc = 0;
        for (int32_t k = H.rp[i]; k < H.rp[i + 1]; k++) {
          int32_t j = H.col[k];
          double xv = j < n1 ? t1[j] : x[j - n1];
          acc += (w ? H.val[k] : 1.0) * xv;
        }
        y[r] = x[r] - beta * acc;
      }
    }, 4096);
  }
};

// lower-triangular dense solves with L (n2 x n2 row-major)
void lsolve(const std::vector<double>& L, int m, double* x) {  // x <- L^{-1} x
  for (int i = 0; i < m; i++) {
    double s = x[i];
    const double* li = &L[(size_t)i * m];
    for (int k = 0; k < i; k++) s -= li[k] * x[k];
    x[i] = s / li[i];
  }
}
void ltsolve(const std::vector<double>& L, int m, double* x) {  // x <- L^{-T} x
  for (int i = m - 1; i >= 0; i--) {
    double s = x[i];
    for (int k = i + 1; k < m; k++) s -= L[(size_t)k * m + i] * x[k];
    x[i] = s / L[(size_t)i * m + i];
  }
}

// Top-r eigenpairs of R = I - L^{-1} S L^{-T} by Lanczos with full
// reorthogonalisation (Algorithm 1, Lanczos step; R as a matrix-vector
// product only).  An exhausted Krylov space restarts from a fresh random
// vector orthogonal to the basis, so m = n2 steps give the whole spectrum.
void lanczos_R(HostIndex& H, int32_t r, int32_t steps, uint64_t seed) {
  const int32_t m2 = H.n2;
  r = std::min(r, m2);
  H.rank = r;
  if (r <= 0) return;
  int32_t m = steps > 0 ? steps : std::max(2 * r, r + 20);
  m = std::min(m, m2);
  SchurOp S(H);
  const bool chol = H.l_kind != KATZ_L_IDENTITY;  // a dense lower factor L (CHOL or IC0)
  std::vector<double> Q((size_t)m * m2);
  std::vector<double> w(m2), tmp(m2);
  std::vector<double> al, be;
  uint64_t rs = seed;
  auto random_start = [&](double* q, int32_t j) {
    lanczos_normals(rs, q, m2);
    for (int pass = 0; pass < 2; pass++)
      for (int32_t k = 0; k < j; k++) {
        const double* qk = &Q[(size_t)k * m2];
        double h = dot(qk, q, m2);
        for (int32_t i = 0; i < m2; i++) q[i] -= h * qk[i];
      }
    double nn = std::sqrt(dot(q, q, m2));
    for (int32_t i = 0; i < m2; i++) q[i] /= nn;
  };
  random_start(&Q[0], 0);
  auto applyR = [&](const double* x, double* y) {
    // y = x - L^{-1} S L^{-T} x
    std::copy(x, x + m2, tmp.begin());
    if (chol) ltsolve(H.lchol, m2, tmp.data());
    S.apply(tmp.data(), y);
    if (chol) lsolve(H.lchol, m2, y);
    for (int32_t i = 0; i < m2; i++) y[i] = x[i] - y[i];
  };
  double tnorm = 0;
  for (int32_t j = 0; j < m; j++) {
    double* qj = &Q[(size_t)j * m2];
    applyR(qj, w.data());
    double a = dot(qj, w.data(), m2);
    al.push_back(a);
    tnorm = std::max(tnorm, std::fabs(a));
    // full reorthogonalisation, two classical Gram-Schmidt passes
    for (int pass = 0; pass < 2; pass++) {
      std::vector<double> h(j + 1);
      parallel_for(j + 1, [&](int64_t k0, int64_t k1) {
        for (int64_t k = k0; k < k1; k++) {
          const double* qk = &Q[(size_t)k * m2];
          double s = 0;
          for (int32_t i = 0; i < m2; i++) s += qk[i] * w[i];
          h[k] = s;
        }
      }, 1);
      parallel_for(m2, [&](int64_t i0, int64_t i1) {
        for (int32_t k = 0; k <= j; k++) {
          const double* qk = &Q[(size_t)k * m2];
          double hk = h[k];
          for (int64_t i = i0; i < i1; i++) w[i] -= hk * qk[i];
        }
      }, 16384);
    }
    if (j + 1 == m) {
      be.push_back(std::sqrt(dot(w.data(), w.data(), m2)));
      break;
    }
    double b = std::sqrt(dot(w.data(), w.data(), m2));
    double* qn = &Q[(size_t)(j + 1) * m2];
    if (b <= 1e-12 * std::max(tnorm, 1e-300)) {
      be.push_back(0.0);  // invariant subspace: T decouples, restart
      random_start(qn, j + 1);
    } else {
      be.push_back(b);
      for (int32_t i = 0; i < m2; i++) qn[i] = w[i] / b;
    }
    tnorm = std::max(tnorm, b);
  }
  const int32_t mm = (int32_t)al.size();
  const std::vector<double> z = lanczos_ritz(H, al, be, r);
  // Ritz vectors u_t = Q^T y_t, stored row-major n2 x r
  H.U.assign((size_t)m2 * r, 0.0);
  parallel_for(m2, [&](int64_t i0, int64_t i1) {
    for (int64_t i = i0; i < i1; i++)
      for (int32_t t = 0; t < r; t++) {
        double s = 0;
        for (int32_t k = 0; k < mm; k++) s += Q[(size_t)k * m2 + i] * z[(size_t)t * mm + k];
        H.U[(size_t)i * r + t] = s;
      }
  }, 4096);
  // V = L^{-T} U
  H.V = H.U;
  if (chol) {
    std::vector<double> colv(m2);
    for (int32_t t = 0; t < r; t++) {
      for (int32_t i = 0; i < m2; i++) colv[i] = H.U[(size_t)i * r + t];
      ltsolve(H.lchol, m2, colv.data());
      for (int32_t i = 0; i < m2; i++) H.V[(size_t)i * r + t] = colv[i];
    }
  }
}

}  // namespace

void lanczos_normals(uint64_t& state, double* out, int64_t n) {
  Rng rng{state};
  for (int64_t i = 0; i < n; i++) out[i] = rng.normal();
  state = rng.s;
}

// Largest correction weight D_i for which auto stores V in BF16.
constexpr double kBf16MaxWeight = 16.0;

std::vector<double> lanczos_ritz(HostIndex& H, const std::vector<double>& al, const std::vector<double>& be,
                                 int32_t r) {
  const int32_t mm = (int32_t)al.size();
  std::vector<double> d(al), z;
  std::vector<double> e(be.begin(), be.begin() + (mm - 1));
  tridiag_eig(d, e, z, mm);
  std::vector<int32_t> idx(mm);
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) { return d[a] > d[b]; });
  H.rank = r;
  H.sigma.resize(r);
  H.D.resize(r);
  std::vector<double> zr((size_t)mm * r);
  for (int32_t t = 0; t < r; t++) {
    const int32_t col = idx[t];
    double s = d[col];
    if (s >= 1.0 - 1e-12) s = 1.0 - 1e-12;  // R < I exactly since S is SPD
    H.sigma[t] = s;
    H.D[t] = s / (1.0 - s);
    for (int32_t k = 0; k < mm; k++) zr[(size_t)t * mm + k] = z[(size_t)k * mm + col];
  }
  H.sigma_next = mm > r ? d[idx[r]] : 0.0;
  H.lanczos_steps = mm;
  if (H.u_precision_req == 0) {
    // auto storage of V: BF16 unless a large weight would amplify its rounding
    double dmax = 0.0;
    for (double x : H.D) dmax = std::max(dmax, std::fabs(x));
    H.u_precision = dmax <= kBf16MaxWeight ? 3 : 2;
  }
  return zr;
}

bool lanczos_on_device(const HostIndex& H, const katz_build_opts& o) {
  if (o.device < 0 || o.rank <= 0 || H.l_kind != KATZ_L_IDENTITY) return false;
  const int64_t r = std::min<int64_t>(o.rank, H.n2);
  const int64_t m = o.lanczos_steps > 0 ? o.lanczos_steps : std::max<int64_t>(2 * r, r + 20);
  if (std::min<int64_t>(m, H.n2) > 512) return false;  // the device Ritz step's limit
  if (const char* e = getenv("KATZ_LANCZOS")) {  // 1 host, 2 device (tests and timing runs)
    const int v = atoi(e);
    if (v == 1) return false;
    if (v == 2) return true;
  }
  return H.n2 >= 65536;
}

namespace {

// Checks the options and sets the index fields that come from them alone.
void apply_options(const katz_build_opts& o, HostIndex& H) {
  if (o.rank < 0) fail(KATZ_EINVAL, "rank must be >= 0");
  if (o.max_block < 0) fail(KATZ_EINVAL, "max_block must be >= 0");
  if (o.l_kind < KATZ_L_AUTO || o.l_kind > KATZ_L_IC0) fail(KATZ_EINVAL, "bad l_kind");
  if (o.precision != KATZ_PREC_FP64 && o.precision != KATZ_PREC_MIXED) fail(KATZ_EINVAL, "bad precision");
  if (o.order < KATZ_ORDER_AUTO || o.order > KATZ_ORDER_LOCALITY) fail(KATZ_EINVAL, "bad order");
  H.precision = o.precision;
  H.u_precision_req = o.u_precision;
  H.u_precision = o.u_precision == 0 ? 2 : o.u_precision;  // auto: settled in lanczos_ritz
}

// beta from the options (beta, or beta_frac / lambda_max) and c = beta lambda_max.
void set_beta(const katz_build_opts& o, HostIndex& H) {
  if (o.beta > 0) {
    H.beta = o.beta;
  } else {
    if (!(o.beta_frac > 0)) fail(KATZ_EINVAL, "give beta > 0 or beta_frac > 0");
    if (H.lambda_max <= 0) fail(KATZ_EINVAL, "graph has no edges: beta_frac needs lambda_max > 0");
    H.beta = o.beta_frac / H.lambda_max;
  }
  H.c = H.beta * H.lambda_max;
}

// The part of the index that depends on beta (Sec. 3.2 step 4 and the
// low-rank correction): the M11 block inverses, the separator factor and the
// Lanczos on R, from the permuted CSR and the blocks already in H.
void build_factors(const katz_build_opts& o, HostIndex& H, bool defer_lanczos,
                   const std::function<void(const char*)>& phase) {
  // M11 block inverses
  int32_t nb = (int32_t)H.blk_start.size() - 1;
  H.blk_off.assign(nb + 1, 0);
  for (int32_t b = 0; b < nb; b++) {
    int64_t sz = H.blk_start[b + 1] - H.blk_start[b];
    H.blk_off[b + 1] = H.blk_off[b] + sz * sz;
  }
  H.minv.assign(H.blk_off[nb], 0.0);
  std::atomic<int> notpd{0};
  parallel_for(nb, [&](int64_t b0, int64_t b1) {
    std::vector<double> a, w;
    for (int64_t b = b0; b < b1; b++) {
      int32_t s = H.blk_start[b], sz = H.blk_start[b + 1] - s;
      a.assign((size_t)sz * sz, 0.0);
      for (int32_t i = 0; i < sz; i++) {
        a[(size_t)i * sz + i] = 1.0;
        for (int32_t k = H.rp[s + i]; k < H.split[s + i]; k++) {
          int32_t j = H.col[k] - s;  // within the block by construction
          a[(size_t)i * sz + j] -= H.beta * (H.weighted ? H.val[k] : 1.0);
        }
      }
      if (!chol_lower(a.data(), sz)) { notpd = 1; continue; }
      chol_inverse(a.data(), sz, &H.minv[H.blk_off[b]], w);
    }
  }, 16);
  if (notpd) fail(KATZ_EDIVERGE, "an M11 block is not positive definite (beta too large)");
  phase("block inverses");

  // separator factor
  int32_t lk = o.l_kind;
  if (lk == KATZ_L_AUTO) lk = (H.n2 > 0 && H.n2 <= 1024) ? KATZ_L_CHOL : KATZ_L_IDENTITY;
  if ((lk == KATZ_L_CHOL || lk == KATZ_L_IC0) && H.n2 > 4096)
    fail(KATZ_EINVAL, "l_kind CHOL and IC0 need a separator of at most 4096 nodes");
  H.l_kind = lk;
  if ((lk == KATZ_L_CHOL || lk == KATZ_L_IC0) && H.n2 > 0) {
    const int32_t m2 = H.n2, n1 = H.n1;
    H.lchol.assign((size_t)m2 * m2, 0.0);
    for (int32_t r = 0; r < m2; r++) {
      H.lchol[(size_t)r * m2 + r] = 1.0;
      int32_t i = n1 + r;
      for (int32_t k = H.split[i]; k < H.rp[i + 1]; k++)
        H.lchol[(size_t)r * m2 + (H.col[k] - n1)] -= H.beta * (H.weighted ? H.val[k] : 1.0);
    }
    const bool ok = lk == KATZ_L_CHOL ? chol_lower(H.lchol.data(), m2) : ic0_lower(H.lchol.data(), m2);
    if (!ok) fail(KATZ_EDIVERGE, "M22 is not positive definite (beta too large)");
    H.ginv.assign((size_t)m2 * m2, 0.0);
    std::vector<double> w;
    chol_inverse(H.lchol.data(), m2, H.ginv.data(), w);
  }
  phase("M22 factor");
  if (defer_lanczos && lanczos_on_device(H, o)) {
    H.rank = 0;
    H.lanczos_rank = std::min(o.rank, H.n2);
    H.lanczos_steps_req = o.lanczos_steps;
    H.lanczos_seed = o.seed;
  } else {
    lanczos_R(H, std::min(o.rank, H.n2), o.lanczos_steps, o.seed);
    phase("Lanczos on R");
  }
}

}  // namespace

void build_host_index(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col,
                      const double* val, const katz_build_opts& o, HostIndex& H, bool defer_lanczos) {
  auto t0 = std::chrono::steady_clock::now();
  // KATZ_VERBOSE=1: phase times of the build on stderr
  const bool verbose = getenv("KATZ_VERBOSE") && atoi(getenv("KATZ_VERBOSE")) > 0;
  auto tp = t0;
  int slot = 0;
  auto phase = [&](const char* what) {
    auto t = std::chrono::steady_clock::now();
    const double sec = std::chrono::duration<double>(t - tp).count();
    // phase slots: validate 0, lambda_max 1, (partition 2-6), CSR 7, inverses 8, M22 9, Lanczos 10
    if (slot < 12) H.phase_seconds[slot] = sec;
    slot = slot == 1 ? 7 : slot + 1;
    if (verbose) std::fprintf(stderr, "katz build: %-22s %8.3f s\n", what, sec);
    tp = t;
  };
  validate(n, nnz, row_ptr, col, val);
  phase("validate");
  apply_options(o, H);
  H.n = n;
  H.nnz = nnz;
  H.weighted = val != nullptr;
  // large graphs with a device: the Lanczos vectors and products on the GPU
  // (the same steps and stopping rule; sums in a fixed order)
  int lam_dev = o.device >= 0 && n >= kLambdaDeviceMin && row_ptr[n] > 0;
  if (const char* e = getenv("KATZ_LAMBDA_DEVICE")) lam_dev = lam_dev && atoi(e) != 0;
  H.lambda_max = lam_dev ? device_lambda_max(o.device, n, nnz, row_ptr, col, val, o.seed)
                         : lambda_max(n, row_ptr, col, val, o.seed);
  set_beta(o, H);
  phase("lambda_max");
  if (!(H.c < 1.0)) fail(KATZ_EDIVERGE, "beta * lambda_max(A) >= 1: Katz series diverges and I - beta A is not positive definite");
  if (o.labels)
    for (int32_t v = 0; v < n; v++)
      if (o.labels[v] < 0) fail(KATZ_EINVAL, "labels must be >= 0");

  int32_t max_block = o.max_block > 0 ? o.max_block : 64;
  int32_t order_kind = o.order;
  if (const char* e = getenv("KATZ_ORDER")) order_kind = atoi(e);
  if (order_kind == KATZ_ORDER_AUTO) order_kind = KATZ_ORDER_LOCALITY;
  Partition P = make_partition(n, row_ptr, col, o.labels, max_block, order_kind);
  H.perm = std::move(P.perm);
  H.iperm = std::move(P.iperm);
  H.blk_start = std::move(P.blk_start);
  H.n1 = P.n1;
  H.n2 = P.n2;
  for (int t = 0; t < 5; t++) H.phase_seconds[2 + t] = P.seconds[t];
  if (verbose) std::fprintf(stderr, "katz build: %-22s %8.3f s\n", "partition",
                            std::chrono::duration<double>(std::chrono::steady_clock::now() - tp).count());
  tp = std::chrono::steady_clock::now();

  // permuted CSR with sorted rows and the separator split
  H.rp.assign(n + 1, 0);
  for (int32_t i = 0; i < n; i++) {
    int32_t v = H.iperm[i];
    H.rp[i + 1] = H.rp[i] + (row_ptr[v + 1] - row_ptr[v]);
  }
  H.col.resize(nnz);
  H.split.resize(n);
  if (val) H.val.resize(nnz);
  parallel_for(n, [&](int64_t b, int64_t e) {
    std::vector<std::pair<int32_t, double>> tmp;
    for (int64_t i = b; i < e; i++) {
      int32_t v = H.iperm[i];
      tmp.clear();
      for (int32_t k = row_ptr[v]; k < row_ptr[v + 1]; k++) tmp.emplace_back(H.perm[col[k]], val ? val[k] : 1.0);
      std::sort(tmp.begin(), tmp.end());
      int32_t o2 = H.rp[i];
      int32_t sp = H.rp[i + 1];
      for (size_t k = 0; k < tmp.size(); k++) {
        H.col[o2 + k] = tmp[k].first;
        if (val) H.val[o2 + k] = tmp[k].second;
        if (tmp[k].first >= H.n1 && sp == H.rp[i + 1]) sp = o2 + (int32_t)k;
      }
      H.split[i] = sp;
    }
  }, 4096);

  phase("permuted CSR");
  build_factors(o, H, defer_lanczos, phase);
  H.build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// The index of the same graph for other options (another beta, rank,
// factor kind, precision, storage, seed or step count): the validated CSR,
// lambda_max, the partition, the node order and the permuted CSR of S are
// reused (Sec. 3.2 steps 1-3 do not depend on beta); the block inverses, the
// separator factor and the Lanczos on R are computed afresh as a build with
// these options computes them.  max_block, labels and order are S's.
void rebuild_host_index(const HostIndex& S, const katz_build_opts& o, HostIndex& H, bool defer_lanczos) {
  auto t0 = std::chrono::steady_clock::now();
  const bool verbose = getenv("KATZ_VERBOSE") && atoi(getenv("KATZ_VERBOSE")) > 0;
  auto tp = t0;
  int slot = 8;  // the build's slots of the block inverses, M22 and Lanczos phases
  auto phase = [&](const char* what) {
    auto t = std::chrono::steady_clock::now();
    const double sec = std::chrono::duration<double>(t - tp).count();
    if (slot < 12) H.phase_seconds[slot++] = sec;
    if (verbose) std::fprintf(stderr, "katz rebuild: %-22s %8.3f s\n", what, sec);
    tp = t;
  };
  apply_options(o, H);
  H.n = S.n;
  H.n1 = S.n1;
  H.n2 = S.n2;
  H.nnz = S.nnz;
  H.weighted = S.weighted;
  H.lambda_max = S.lambda_max;
  set_beta(o, H);
  if (!(H.c < 1.0)) fail(KATZ_EDIVERGE, "beta * lambda_max(A) >= 1: Katz series diverges and I - beta A is not positive definite");
  H.perm = S.perm;
  H.iperm = S.iperm;
  H.rp = S.rp;
  H.col = S.col;
  H.split = S.split;
  H.val = S.val;
  H.blk_start = S.blk_start;
  build_factors(o, H, defer_lanczos, phase);
  H.build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// ------------------------------------------------------------ communities
// Initial parts for the partition of an unlabeled graph (Sec. 3.2, step 2
// partitions with METIS, which this library does not have): the
// local-moving phase of the Louvain method (Blondel et al., 2008) on the
// Newman-Girvan modularity of the weighted graph, with every community
// capped at `cap` nodes.  Each node starts alone; a pass visits the nodes in
// id order, takes each out of its community and puts it into the neighbouring
// community (or back into its own) of the largest gain
//   w(v, C) - k_v tot(C) / 2m
// (w(v, C): the weight of v's edges into C; k_v: v's weighted degree; tot(C):
// the summed degrees of C; 2m: the summed degrees of the graph), which is the
// modularity change of the move up to the positive factor 1 / m.  Its own
// community wins ties, and among the others the first reached in v's CSR
// row.  Communities at the cap take no one.  Passes stop when one moves no
// node or after `passes`.  No aggregation levels: the partition wants
// communities no larger than a block, and the cap is reached within the
// first level.  Serial and deterministic; O(nnz) per pass.  labels[v]:
// community ids 0, 1, ... in breadth-first order (below).
int32_t communities(int32_t n, int64_t nnz, const int32_t* rp, const int32_t* col, const double* val,
                    int32_t cap, int32_t passes, int32_t* labels) {
  validate(n, nnz, rp, col, val);
  if (cap < 1) fail(KATZ_EINVAL, "cap must be >= 1");
  if (passes < 0) fail(KATZ_EINVAL, "passes must be >= 0");
  if (!labels) fail(KATZ_EINVAL, "null labels array");
  std::vector<double> k(n, 0.0), tot(n);
  std::vector<int32_t> comm(n), size(n, 1);
  double m2 = 0.0;
  for (int32_t v = 0; v < n; v++) {
    double d = 0.0;
    for (int32_t e = rp[v]; e < rp[v + 1]; e++) d += val ? val[e] : 1.0;
    k[v] = d;
    tot[v] = d;
    comm[v] = v;
    m2 += d;
  }
  int32_t done = 0;
  if (m2 > 0.0) {
    // wto[c] holds w(v, C) for the communities stamped with this visit's tick
    std::vector<double> wto(n, 0.0);
    std::vector<int64_t> stamp(n, -1);
    std::vector<int32_t> touched;
    int64_t tick = 0;
    for (int32_t pass = 0; pass < passes; pass++) {
      int64_t moved = 0;
      for (int32_t v = 0; v < n; v++) {
        if (!(k[v] > 0.0)) continue;
        const int32_t c0 = comm[v];
        touched.clear();
        tick++;
        stamp[c0] = tick;
        wto[c0] = 0.0;
        for (int32_t e = rp[v]; e < rp[v + 1]; e++) {
          const int32_t c = comm[col[e]];
          if (stamp[c] != tick) {
            stamp[c] = tick;
            wto[c] = 0.0;
            touched.push_back(c);
          }
          wto[c] += val ? val[e] : 1.0;
        }
        tot[c0] -= k[v];
        size[c0]--;
        const double kv = k[v] / m2;
        int32_t best = c0;
        double gbest = wto[c0] - kv * tot[c0];
        for (int32_t c : touched) {
          if (c == c0 || size[c] >= cap) continue;
          const double g = wto[c] - kv * tot[c];
          if (g > gbest) {
            gbest = g;
            best = c;
          }
        }
        comm[v] = best;
        tot[best] += k[v];
        size[best]++;
        moved += best != c0;
      }
      done = pass + 1;
      if (moved == 0) break;
    }
  }
  // ids in the order a breadth-first search first reaches each community
  // (from node 0, neighbours in CSR order, restarting at the smallest
  // unreached node): the partition lays the parts out in id order, so
  // neighbouring communities get nearby positions
  std::vector<int32_t> id(n, -1), queue;
  std::vector<char> seen(n, 0);
  queue.reserve(n);
  int32_t next = 0;
  for (int32_t s = 0; s < n; s++) {
    if (seen[s]) continue;
    seen[s] = 1;
    queue.push_back(s);
    for (size_t h = queue.size() - 1; h < queue.size(); h++) {
      const int32_t u = queue[h];
      if (id[comm[u]] < 0) id[comm[u]] = next++;
      for (int32_t e = rp[u]; e < rp[u + 1]; e++)
        if (!seen[col[e]]) {
          seen[col[e]] = 1;
          queue.push_back(col[e]);
        }
    }
  }
  for (int32_t v = 0; v < n; v++) labels[v] = id[comm[v]];
  return done;
}

}  // namespace katz
