// C ABI of the Katz library (include/katz.h): argument checks, error codes,
// thread-local error messages; no exceptions cross the boundary.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>
#include <new>
#include <string>

#include "katz.h"
#include "katz_internal.h"

namespace {
thread_local std::string g_last_error;

int set_error(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

template <typename F>
int guarded(F&& f) {
  try {
    g_last_error.clear();
    return f();
  } catch (const katz::Error& e) {
    return set_error(e.code, e.msg);
  } catch (const std::bad_alloc&) {
    return set_error(KATZ_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return set_error(KATZ_EINVAL, e.what());
  }
}

int check_queries(const katz_index* idx, const int32_t* q, int32_t nq) {
  if (!idx) return set_error(KATZ_EINVAL, "null index");
  if (nq < 0) return set_error(KATZ_EINVAL, "nq must be >= 0");
  if (nq > 0 && !q) return set_error(KATZ_EINVAL, "null query array");
  for (int32_t i = 0; i < nq; i++)
    if (q[i] < 0 || q[i] >= idx->host.n) return set_error(KATZ_EINVAL, "query id out of range");
  if (!idx->dev) return set_error(KATZ_EDEVICE, "index was built without a device (device = -1)");
  return KATZ_OK;
}

katz_query_opts resolve(const katz_query_opts* o);

// An index whose host part is complete: with a device (>= 0), upload it and
// run the Lanczos on R there when the host part left it for the device.
void finish_on_device(katz_index* idx, int32_t device) {
  idx->device = device;
  if (device < 0) return;
  const auto t0 = std::chrono::steady_clock::now();
  idx->dev = katz::device_upload(idx->host, device);
  idx->host.phase_seconds[11] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  idx->host.build_seconds += idx->host.phase_seconds[11];
  if (idx->host.lanczos_rank > 0) katz::device_lanczos_R(idx->host, idx->dev);
}

// K[dst[i], src[i]] for validated pairs into host out[], per-pair stats
// (nullable); the distinct sources run as the columns of batched solves.
int pair_scores_host(const katz_index* idx, const int32_t* src, const int32_t* dst, int32_t npairs,
                     const katz_query_opts* opts, double* out_h, katz_query_stats* st, void* stream) {
  std::vector<int32_t> order(npairs);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return src[a] < src[b]; });
  std::vector<int32_t> q, pcol(npairs), prow(npairs);
  for (int32_t t = 0; t < npairs; t++) {
    const int32_t i = order[t];
    if (q.empty() || q.back() != src[i]) q.push_back(src[i]);
    pcol[t] = (int32_t)q.size() - 1;
    prow[t] = idx->host.perm[dst[i]];
  }
  std::vector<double> out(npairs);
  std::vector<katz_query_stats> qst(q.size());
  katz::QueryArgs a{};
  a.q = q.data(); a.nq = (int32_t)q.size(); a.opts = resolve(opts); a.scores = nullptr; a.topk = 0;
  a.st = qst.data(); a.stream = stream;
  a.npairs = npairs; a.pair_col = pcol.data(); a.pair_row = prow.data(); a.pair_out = out.data();
  const int rc = katz::device_query(idx->host, idx->dev, a);
  for (int32_t t = 0; t < npairs; t++) {
    out_h[order[t]] = out[t];
    if (st) st[order[t]] = qst[pcol[t]];
  }
  return rc;
}

katz_query_opts resolve(const katz_query_opts* o) {
  katz_query_opts r;
  katz_query_opts_default(&r);
  if (o) r = *o;
  if (!(r.rel_tol > 0)) r.rel_tol = 1e-6;
  if (r.max_iter <= 0) r.max_iter = 1000;
  if (r.max_sweeps <= 0) r.max_sweeps = 6;
  if (r.check_every < 0) r.check_every = 0;  // 0: adaptive polling
  if (r.method != KATZ_METHOD_LRC && r.method != KATZ_METHOD_CG && r.method != KATZ_METHOD_PCGNR)
    katz::fail(KATZ_EINVAL, "bad method");
  return r;
}
}  // namespace

extern "C" {

void katz_build_opts_default(katz_build_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->beta = 0.0;
  o->beta_frac = 0.5;
  o->rank = 32;
  o->max_block = 64;
  o->labels = nullptr;
  o->l_kind = KATZ_L_AUTO;
  o->precision = KATZ_PREC_FP64;
  o->seed = 12345;
  o->device = 0;
  o->lanczos_steps = 0;
  o->order = KATZ_ORDER_AUTO;
  o->u_precision = 0;
}

void katz_query_opts_default(katz_query_opts* o) {
  if (!o) return;
  o->rel_tol = 1e-6;
  o->max_iter = 1000;
  o->method = KATZ_METHOD_LRC;
  o->max_sweeps = 6;
  o->check_every = 0;
  o->force_fallback = 0;
}

int katz_index_build(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                     const double* val, const katz_build_opts* opts, katz_index** out) {
  return guarded([&]() -> int {
    if (!out) return set_error(KATZ_EINVAL, "null output pointer");
    *out = nullptr;
    katz_build_opts o;
    katz_build_opts_default(&o);
    if (opts) o = *opts;
    if (o.max_block > 256) return set_error(KATZ_EINVAL, "max_block must be <= 256");
    if (o.u_precision < 0 || o.u_precision > 3) return set_error(KATZ_EINVAL, "bad u_precision");
    auto* idx = new katz_index();
    try {
      // with a device, a large Lanczos on R runs there after the upload
      katz::build_host_index(n, nnz, row_ptr, col_idx, val, o, idx->host, o.device >= 0);
      finish_on_device(idx, o.device);
    } catch (...) {
      katz_index_free(idx);
      throw;
    }
    *out = idx;
    return KATZ_OK;
  });
}

int katz_index_rebuild(const katz_index* src, const katz_build_opts* opts, katz_index** out) {
  return guarded([&]() -> int {
    if (!out) return set_error(KATZ_EINVAL, "null output pointer");
    *out = nullptr;
    if (!src) return set_error(KATZ_EINVAL, "null source index");
    katz_build_opts o;
    katz_build_opts_default(&o);
    if (opts) o = *opts;
    if (o.u_precision < 0 || o.u_precision > 3) return set_error(KATZ_EINVAL, "bad u_precision");
    auto* idx = new katz_index();
    try {
      katz::rebuild_host_index(src->host, o, idx->host, o.device >= 0);
      finish_on_device(idx, o.device);
    } catch (...) {
      katz_index_free(idx);
      throw;
    }
    *out = idx;
    return KATZ_OK;
  });
}

int katz_communities(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx, const double* val,
                     int32_t cap, int32_t passes, int32_t* labels, int32_t* passes_run) {
  return guarded([&]() -> int {
    const int32_t done = katz::communities(n, nnz, row_ptr, col_idx, val, cap, passes, labels);
    if (passes_run) *passes_run = done;
    return KATZ_OK;
  });
}

int katz_index_save(const katz_index* idx, const char* path) {
  return guarded([&]() -> int {
    if (!idx || !path) return set_error(KATZ_EINVAL, "null index or path");
    katz::save_host_index(idx->host, path);
    return KATZ_OK;
  });
}

int katz_index_load(const char* path, int32_t device, katz_index** out) {
  return guarded([&]() -> int {
    if (!out || !path) return set_error(KATZ_EINVAL, "null path or output pointer");
    *out = nullptr;
    auto* idx = new katz_index();
    try {
      katz::load_host_index(path, idx->host);
      idx->device = device;
      if (device >= 0) idx->dev = katz::device_upload(idx->host, device);
    } catch (...) {
      katz_index_free(idx);
      throw;
    }
    *out = idx;
    return KATZ_OK;
  });
}

int katz_query(const katz_index* idx, const int32_t* q, int32_t nq, const katz_query_opts* opts,
               double* scores, katz_query_stats* st, void* stream) {
  return guarded([&]() -> int {
    int rc = check_queries(idx, q, nq);
    if (rc) return rc;
    if (nq == 0) return KATZ_OK;
    if (!scores) return set_error(KATZ_EINVAL, "null scores buffer");
    katz::QueryArgs a{};
    a.q = q; a.nq = nq; a.opts = resolve(opts); a.scores = scores; a.topk = 0;
    a.st = st; a.stream = stream;
    rc = katz::device_query(idx->host, idx->dev, a);
    if (rc == KATZ_ENOCONV) set_error(rc, "some queries did not reach the tolerance (see stats)");
    return rc;
  });
}

int katz_query_noalloc(const katz_index* idx, const int32_t* q, int32_t nq, const katz_query_opts* opts,
                       double* scores, katz_query_stats* st, void* stream) {
  return guarded([&]() -> int {
    int rc = check_queries(idx, q, nq);
    if (rc) return rc;
    if (nq == 0) return KATZ_OK;
    if (!scores) return set_error(KATZ_EINVAL, "null scores buffer");
    katz::QueryArgs a{};
    a.q = q; a.nq = nq; a.opts = resolve(opts); a.scores = scores; a.topk = 0;
    a.st = st; a.stream = stream;
    rc = katz::device_query_noalloc(idx->host, idx->dev, a);
    if (rc == KATZ_ENOCONV) set_error(rc, "some queries did not reach the tolerance (see stats)");
    return rc;
  });
}

int katz_pair_scores(const katz_index* idx, const int32_t* src, const int32_t* dst, int32_t npairs,
                     const katz_query_opts* opts, double* scores, katz_query_stats* st, void* stream) {
  return guarded([&]() -> int {
    if (!idx) return set_error(KATZ_EINVAL, "null index");
    if (npairs < 0) return set_error(KATZ_EINVAL, "npairs must be >= 0");
    if (npairs == 0) return KATZ_OK;
    if (!src || !dst || !scores) return set_error(KATZ_EINVAL, "null pair or output array");
    int rc = check_queries(idx, src, npairs);
    if (rc) return rc;
    rc = check_queries(idx, dst, npairs);
    if (rc) return rc;
    std::vector<double> res(npairs);
    rc = pair_scores_host(idx, src, dst, npairs, opts, res.data(), st, stream);
    katz::copy_to_caller(scores, res.data(), sizeof(double) * (size_t)npairs);
    if (rc == KATZ_ENOCONV) set_error(rc, "some queries did not reach the tolerance (see stats)");
    return rc;
  });
}

int katz_sparse_katz(const katz_index* idx, const int32_t* q, int32_t nq, int32_t s, int32_t T,
                     const katz_query_opts* opts, int32_t* ids, double* corr, katz_query_stats* st,
                     void* stream) {
  return guarded([&]() -> int {
    int rc = check_queries(idx, q, nq);
    if (rc) return rc;
    if (s < 0 || T < 2 || T > 4096 || s > 4096) return set_error(KATZ_EINVAL, "need 0 <= s <= 4096 and 2 <= T <= 4096");
    if (nq == 0 || s == 0) return KATZ_OK;
    if (!ids) return set_error(KATZ_EINVAL, "null ids buffer");
    // (1) k_q and its top max(s, T) candidates (q and its neighbours excluded)
    const int32_t K = std::max(s, T);
    std::vector<int32_t> top((size_t)nq * K);
    std::vector<double> topsc((size_t)nq * K);
    katz::QueryArgs a{};
    a.q = q; a.nq = nq; a.opts = resolve(opts); a.scores = nullptr; a.topk = K; a.ids = top.data();
    a.topk_scores = topsc.data(); a.st = st; a.stream = stream;
    int rc1 = katz::device_query(idx->host, idx->dev, a);
    // (2) the T modular nodes t of each query: K_T[v][t] = K[v, t] = K[t, v]
    // for v = q and every listed candidate, gathered from the Katz vectors of
    // the t (pair entries, batched over the distinct t)
    std::vector<int32_t> ncand(nq), nmod(nq);
    std::vector<int64_t> base(nq);
    int64_t total = 0;
    for (int32_t i = 0; i < nq; i++) {
      const int32_t* li = top.data() + (size_t)i * K;
      int32_t nc = 0;
      while (nc < K && li[nc] >= 0) nc++;
      ncand[i] = std::min(nc, s);
      nmod[i] = std::min(nc, T);
      base[i] = total;
      total += (int64_t)nmod[i] * (ncand[i] + 1);
    }
    if (total > INT32_MAX)
      return set_error(KATZ_EINVAL, "too many correlation entries in one call (nq * T * (s + 1) > 2^31 - 1)");
    std::vector<int32_t> ps, pd;
    ps.reserve((size_t)total);
    pd.reserve((size_t)total);
    std::vector<int32_t> cand((size_t)nq * s, -1);
    for (int32_t i = 0; i < nq; i++) {
      const int32_t* li = top.data() + (size_t)i * K;
      for (int32_t j = 0; j < ncand[i]; j++) cand[(size_t)i * s + j] = li[j];
      for (int32_t t = 0; t < nmod[i]; t++) {
        ps.push_back(li[t]);
        pd.push_back(q[i]);
        for (int32_t j = 0; j < ncand[i]; j++) {
          ps.push_back(li[t]);
          pd.push_back(li[j]);
        }
      }
    }
    // pairs sorted by their source (stable), one batch column per distinct source
    const int32_t np = (int32_t)ps.size();
    std::vector<int32_t> order(np), inv(np), qsrc, pcol(np), prow(np);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return ps[x] < ps[y]; });
    for (int32_t t = 0; t < np; t++) {
      const int32_t p = order[t];
      if (qsrc.empty() || qsrc.back() != ps[p]) qsrc.push_back(ps[p]);
      pcol[t] = (int32_t)qsrc.size() - 1;
      prow[t] = idx->host.perm[pd[p]];
      inv[p] = t;
    }
    std::vector<katz_query_stats> pst(qsrc.size());
    // (3) Pearson correlation of row q with each candidate's row and the
    // re-ranking, on the device; only the lists return
    int rc2 = katz::device_sparse_katz(idx->host, idx->dev, resolve(opts), stream, qsrc, pcol, prow, inv, base,
                                       ncand, nmod, cand, nq, s, pst.data(), ids, corr);
    rc = rc1 != KATZ_OK ? rc1 : rc2;
    if (rc == KATZ_ENOCONV) set_error(rc, "some solves did not reach the tolerance");
    return rc;
  });
}

int katz_topk_links(const katz_index* idx, const int32_t* q, int32_t nq, int32_t k,
                    const katz_query_opts* opts, int32_t* ids, double* scores, katz_query_stats* st,
                    void* stream) {
  return guarded([&]() -> int {
    int rc = check_queries(idx, q, nq);
    if (rc) return rc;
    if (k < 0) return set_error(KATZ_EINVAL, "k must be >= 0");
    if (nq == 0 || k == 0) return KATZ_OK;
    if (!ids) return set_error(KATZ_EINVAL, "null ids buffer");
    katz::QueryArgs a{};
    a.q = q; a.nq = nq; a.opts = resolve(opts); a.scores = nullptr; a.topk = k; a.ids = ids;
    a.topk_scores = scores; a.st = st; a.stream = stream;
    rc = katz::device_query(idx->host, idx->dev, a);
    if (rc == KATZ_ENOCONV) set_error(rc, "some queries did not reach the tolerance (see stats)");
    return rc;
  });
}

void katz_index_free(katz_index* idx) {
  if (!idx) return;
  try {
    katz::device_free(idx->dev);
  } catch (...) {
  }
  delete idx;
}

int katz_index_info(const katz_index* idx, katz_index_info_t* info) {
  if (!idx || !info) return set_error(KATZ_EINVAL, "null argument");
  const katz::HostIndex& H = idx->host;
  std::memset(info, 0, sizeof(*info));
  info->n = H.n;
  info->n1 = H.n1;
  info->n2 = H.n2;
  info->nnz = H.nnz;
  info->nblocks = (int32_t)H.blk_start.size() - 1;
  int32_t mb = 0;
  for (size_t b = 0; b + 1 < H.blk_start.size(); b++) mb = std::max(mb, H.blk_start[b + 1] - H.blk_start[b]);
  info->max_block_size = mb;
  info->rank = H.rank;
  info->l_kind = H.l_kind;
  info->precision = H.precision;
  info->device = idx->dev ? idx->device : -1;
  info->beta = H.beta;
  info->lambda_max = H.lambda_max;
  info->c = H.c;
  info->sigma_max = H.rank > 0 ? H.sigma[0] : 0.0;
  info->sigma_next = H.sigma_next;
  info->factor_bytes = idx->dev ? katz::device_factor_bytes(idx->dev) : (int64_t)H.minv.size() * 8;
  info->device_bytes = katz::device_bytes(idx->dev);
  info->build_seconds = H.build_seconds;
  info->u_precision = H.u_precision;
  for (int t = 0; t < 12; t++) info->build_phase_seconds[t] = H.phase_seconds[t];
  return KATZ_OK;
}

int katz_index_partition(const katz_index* idx, int32_t* perm, int32_t* block_ptr) {
  if (!idx) return set_error(KATZ_EINVAL, "null index");
  const katz::HostIndex& H = idx->host;
  if (perm) std::memcpy(perm, H.perm.data(), sizeof(int32_t) * H.perm.size());
  if (block_ptr) std::memcpy(block_ptr, H.blk_start.data(), sizeof(int32_t) * H.blk_start.size());
  return KATZ_OK;
}

int katz_index_lowrank(const katz_index* idx, double* U, double* sigma) {
  if (!idx) return set_error(KATZ_EINVAL, "null index");
  const katz::HostIndex& H = idx->host;
  if (U && !H.U.empty()) std::memcpy(U, H.U.data(), sizeof(double) * H.U.size());
  if (sigma && !H.sigma.empty()) std::memcpy(sigma, H.sigma.data(), sizeof(double) * H.sigma.size());
  return KATZ_OK;
}

int katz_profile_enable(int on) { return katz::profile_enable(on); }
void katz_profile_reset(void) { katz::profile_reset(); }
int katz_profile_read(katz_kernel_stat* out, int max) {
  if (!out || max <= 0) return 0;
  return katz::profile_read(out, max);
}

const char* katz_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
