// Serving loop for top-K link-prediction requests (Sec. 3.3: a request is a
// set of query nodes; each gets its K best non-neighbours by Katz score).
//
// Continuous batching over worker slots: every worker owns a device workspace
// of fixed column capacity and its own stream.  An idle worker takes query
// columns from the request queue -- a whole small request, several small
// requests merged, or a slice of a large one -- and solves them as one batch
// (Algorithm 2 with the top-K selection), the queue served in arrival order.
// Requests that arrive while others are on the GPU start as soon as a worker
// slot is free; the workers' batches run concurrently on the device.  The number of
// workers and their capacity are admitted against free HBM at creation (each
// resident column costs a fixed number of node-length panels), so requests
// are queued, split and admitted by memory footprint, never over-subscribed.
//
// Per-column solver state and deterministic reductions make a column's result
// independent of the other columns in its batch for a given batch width;
// batches of different widths agree within the solve tolerance.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include <hip/hip_runtime.h>

#include "katz.h"
#include "katz_internal.h"

namespace katz {
namespace {

using Clock = std::chrono::steady_clock;

// Narrowest batch the spreading rule makes (narrower LRC batches lose more
// per column than the extra parallel slot gains).
constexpr int kMinSlice = 16;

struct Request {
  int64_t ticket;
  std::vector<int32_t> q;
  std::vector<int32_t> ids;       // nq * k
  std::vector<double> scores;     // nq * k
  std::vector<katz_query_stats> st;
  int32_t next = 0;               // first query not yet taken by a worker
  int32_t remaining = 0;          // queries not yet finished
  int32_t inflight = 0;           // slices of this request being solved
  int status = KATZ_OK;
  Clock::time_point t_submit, t_done;
  bool done = false;
};

}  // namespace

struct Server {
  const katz_index* idx = nullptr;
  katz_server_opts opts{};
  int k = 100;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Request>> queue;               // requests with untaken queries
  std::unordered_map<int64_t, std::shared_ptr<Request>> live;
  int64_t next_ticket = 1;
  bool stop = false;
  std::vector<std::thread> workers;
  std::vector<Workspace*> ws;
  std::atomic<int64_t> live_columns{0}, done_queries{0}, done_requests{0};
  int busy = 0;                                              // workers solving a batch (under mu)
  // Batches are full (max_batch columns) and taken in arrival order.
  // KATZ_SERVE_SPREAD=1 (measurements only) adds two rules: a free worker
  // takes ceil(queued columns / idle workers) columns (at least kMinSlice),
  // and one request holds at most W - 1 workers while others wait.  They
  // gave no better latency than arrival order (the same at 1M nodes, 5-15%
  // higher p50 at 4M), so they are off by default.
  const bool spread_rules = getenv("KATZ_SERVE_SPREAD") && atoi(getenv("KATZ_SERVE_SPREAD")) > 0;
  int64_t queued_cols = 0;                                   // untaken columns in the queue (under mu)
  std::vector<double> latencies_ms;                          // completed requests
  int64_t max_latency_samples = 1 << 20;
  std::string init_error;
  std::atomic<int> init_failed{0};

  void worker_main(int wid) {
    try {
      if (hipSetDevice(idx->dev ? idx->device : 0) != hipSuccess) throw Error{KATZ_EDEVICE, "hipSetDevice"};
    } catch (...) {
      init_failed = 1;
      return;
    }
    hipStream_t stream = nullptr;
    hipError_t se;
    {
      std::lock_guard<std::recursive_mutex> lk(hip_global_mu());
      se = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
    }
    if (se != hipSuccess) {
      init_failed = 1;
      return;
    }
    Workspace* w = ws[wid];
    const int cap = ws_capacity(w);
    std::vector<int32_t> q;
    struct Slice { std::shared_ptr<Request> r; int32_t off, cnt; };
    std::vector<Slice> slices;
    std::vector<int32_t> ids;
    std::vector<double> sc;
    std::vector<katz_query_stats> st;
    for (;;) {
      slices.clear();
      q.clear();
      {
        std::unique_lock<std::mutex> g(mu);
        const int W = (int)ws.size();
        // the first request this worker may take from: the queue head (with
        // the spread rules, skipping one that holds W - 1 workers while
        // others wait)
        auto pick = [&]() -> int {
          const int share = (queue.size() > 1 && spread_rules) ? std::max(1, W - 1) : W;
          for (size_t t = 0; t < queue.size(); t++)
            if (queue[t]->inflight < share) return (int)t;
          return -1;
        };
        cv_work.wait(g, [&] { return (stop && queue.empty()) || pick() >= 0; });
        if (stop && queue.empty()) break;
        const int idle = std::max(1, W - busy);
        const int64_t spread = (queued_cols + idle - 1) / idle;
        const int want = !spread_rules ? cap
                                   : (int)std::min<int64_t>(cap, std::max<int64_t>(std::min(kMinSlice, cap), spread));
        for (int t = pick(); t >= 0 && t < (int)queue.size() && (int)q.size() < want;) {
          auto r = queue[t];
          const int32_t take = std::min<int32_t>(want - (int32_t)q.size(), (int32_t)r->q.size() - r->next);
          slices.push_back({r, r->next, take});
          q.insert(q.end(), r->q.begin() + r->next, r->q.begin() + r->next + take);
          r->next += take;
          r->inflight++;
          queued_cols -= take;
          if (r->next == (int32_t)r->q.size()) queue.erase(queue.begin() + t);
          else t++;
        }
        if (q.empty()) continue;
        busy++;
      }
      const int nq = (int)q.size();
      live_columns += nq;
      ids.assign((size_t)nq * k, -1);
      sc.assign((size_t)nq * k, 0.0);
      st.assign(nq, katz_query_stats{});
      QueryArgs a{};
      a.q = q.data();
      a.nq = nq;
      a.opts = opts.query;
      a.scores = nullptr;
      a.topk = k;
      a.ids = ids.data();
      a.topk_scores = sc.data();
      a.st = st.data();
      a.stream = stream;
      int rc;
      try {
        rc = device_query_ws(idx->host, idx->dev, a, w);
      } catch (const Error& e) {
        rc = e.code;
      } catch (...) {
        rc = KATZ_EDEVICE;
      }
      live_columns -= nq;
      std::lock_guard<std::mutex> g(mu);
      int pos = 0;
      for (auto& s : slices) {
        Request& r = *s.r;
        std::memcpy(&r.ids[(size_t)s.off * k], &ids[(size_t)pos * k], sizeof(int32_t) * (size_t)s.cnt * k);
        std::memcpy(&r.scores[(size_t)s.off * k], &sc[(size_t)pos * k], sizeof(double) * (size_t)s.cnt * k);
        std::memcpy(&r.st[s.off], &st[pos], sizeof(katz_query_stats) * s.cnt);
        if (rc != KATZ_OK && r.status == KATZ_OK) r.status = rc;
        r.remaining -= s.cnt;
        r.inflight--;
        pos += s.cnt;
        if (r.remaining == 0) {
          r.done = true;
          r.t_done = Clock::now();
          done_requests++;
          if ((int64_t)latencies_ms.size() < max_latency_samples)
            latencies_ms.push_back(std::chrono::duration<double, std::milli>(r.t_done - r.t_submit).count());
        }
      }
      done_queries += nq;
      busy--;
      cv_done.notify_all();
      cv_work.notify_all();  // a slot is free, and a request may be below its share again
    }
    std::lock_guard<std::recursive_mutex> lk(hip_global_mu());
    (void)hipStreamDestroy(stream);
  }
};

}  // namespace katz

struct katz_server {
  katz::Server s;
};

using katz::Clock;

extern "C" {

void katz_server_opts_default(katz_server_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->workers = 0;
  o->max_batch = 64;
  o->hbm_fraction = 0.8;
  o->k = 100;
  katz_query_opts_default(&o->query);
}

}  // extern "C"

namespace katz {
// Bytes of device workspace per resident query column.
int64_t bytes_per_column(const katz_index* idx) { return ws_bytes_per_column(idx->dev); }
}  // namespace katz

extern "C" {

int katz_server_create(const katz_index* idx, const katz_server_opts* o, katz_server** out) {
  try {
    if (!idx || !out) return KATZ_EINVAL;
    *out = nullptr;
    if (!idx->dev) return KATZ_EDEVICE;
    katz_server_opts op;
    katz_server_opts_default(&op);
    if (o) op = *o;
    if (op.k <= 0 || op.k > 4096) return KATZ_EINVAL;
    if (op.max_batch <= 0 || op.max_batch > 512) return KATZ_EINVAL;
    if (!(op.hbm_fraction > 0 && op.hbm_fraction <= 0.95)) return KATZ_EINVAL;
    if (hipSetDevice(idx->device) != hipSuccess) return KATZ_EDEVICE;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return KATZ_EDEVICE;
    // admission by footprint: workers x capacity columns must fit the budget
    const int64_t per_col = katz::bytes_per_column(idx);
    const int64_t budget_cols = (int64_t)((double)free_b * op.hbm_fraction) / per_col;
    int workers = op.workers > 0 ? op.workers : 4;
    int cap = op.max_batch;
    while (workers > 1 && (int64_t)workers * cap > budget_cols) workers--;
    while (cap > 1 && (int64_t)workers * cap > budget_cols) cap /= 2;
    if ((int64_t)workers * cap > budget_cols) return KATZ_ENOMEM;
    auto* S = new katz_server();
    katz::Server& s = S->s;
    s.idx = idx;
    s.opts = op;
    s.opts.workers = workers;
    s.opts.max_batch = cap;
    s.k = op.k;
    try {
      for (int i = 0; i < workers; i++) s.ws.push_back(katz::ws_create(idx->dev, cap));
    } catch (...) {
      for (auto* w : s.ws) katz::ws_destroy(idx->dev, w);
      delete S;
      return KATZ_ENOMEM;
    }
    for (int i = 0; i < workers; i++) s.workers.emplace_back([&s, i] { s.worker_main(i); });
    *out = S;
    return KATZ_OK;
  } catch (...) {
    return KATZ_EDEVICE;
  }
}

int katz_server_submit(katz_server* S, const int32_t* q, int32_t nq, int64_t* ticket) {
  if (!S || !ticket || nq <= 0 || !q) return KATZ_EINVAL;
  katz::Server& s = S->s;
  const int32_t n = s.idx->host.n;
  for (int32_t i = 0; i < nq; i++)
    if (q[i] < 0 || q[i] >= n) return KATZ_EINVAL;
  try {
    // the request's result slots (nq x k) are allocated here: a host
    // allocation failure is reported, never thrown across the C ABI
    auto r = std::make_shared<katz::Request>();
    r->q.assign(q, q + nq);
    r->ids.assign((size_t)nq * s.k, -1);
    r->scores.assign((size_t)nq * s.k, 0.0);
    r->st.assign(nq, katz_query_stats{});
    r->remaining = nq;
    r->t_submit = Clock::now();
    {
      std::lock_guard<std::mutex> g(s.mu);
      if (s.stop) return KATZ_EBUSY;
      r->ticket = s.next_ticket++;
      s.live[r->ticket] = r;
      try {
        s.queue.push_back(r);
      } catch (...) {
        s.live.erase(r->ticket);
        throw;
      }
      s.queued_cols += nq;
      *ticket = r->ticket;
    }
  } catch (const std::bad_alloc&) {
    return KATZ_ENOMEM;
  } catch (...) {
    return KATZ_EDEVICE;
  }
  s.cv_work.notify_one();
  return KATZ_OK;
}

int katz_server_poll(katz_server* S, int64_t ticket, int32_t* ids, double* scores, katz_query_stats* st,
                     double* latency_ms, int64_t timeout_us) {
  if (!S) return KATZ_EINVAL;
  katz::Server& s = S->s;
  std::unique_lock<std::mutex> g(s.mu);
  auto it = s.live.find(ticket);
  if (it == s.live.end()) return KATZ_EINVAL;
  auto r = it->second;
  if (!r->done) {
    if (timeout_us == 0) return KATZ_EBUSY;
    auto pred = [&] { return r->done; };
    if (timeout_us < 0)
      s.cv_done.wait(g, pred);
    else if (!s.cv_done.wait_for(g, std::chrono::microseconds(timeout_us), pred))
      return KATZ_EBUSY;
  }
  const size_t nq = r->q.size();
  if (ids) std::memcpy(ids, r->ids.data(), sizeof(int32_t) * nq * s.k);
  if (scores) std::memcpy(scores, r->scores.data(), sizeof(double) * nq * s.k);
  if (st) std::memcpy(st, r->st.data(), sizeof(katz_query_stats) * nq);
  if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
  const int rc = r->status;
  s.live.erase(it);
  return rc;
}

int katz_server_info(katz_server* S, katz_server_info_t* info) {
  if (!S || !info) return KATZ_EINVAL;
  katz::Server& s = S->s;
  std::memset(info, 0, sizeof(*info));
  std::lock_guard<std::mutex> g(s.mu);
  info->workers = s.opts.workers;
  info->capacity = s.opts.max_batch;
  info->k = s.k;
  int64_t queued = 0;
  for (auto& r : s.queue) queued += (int64_t)r->q.size() - r->next;
  info->queued_queries = queued;
  info->live_columns = s.live_columns.load();
  info->done_queries = s.done_queries.load();
  info->done_requests = s.done_requests.load();
  info->bytes_per_column = katz::bytes_per_column(s.idx);
  return KATZ_OK;
}

void katz_server_destroy(katz_server* S) {
  if (!S) return;
  katz::Server& s = S->s;
  {
    std::lock_guard<std::mutex> g(s.mu);
    s.stop = true;
  }
  s.cv_work.notify_all();
  for (auto& t : s.workers) t.join();
  for (auto* w : s.ws) katz::ws_destroy(s.idx->dev, w);
  delete S;
}

}  // extern "C"
