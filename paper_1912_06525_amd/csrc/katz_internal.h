// Internal structures shared by the host index builder, the HIP solver and
// the C ABI.  Not part of the public interface.
#pragma once

#include <cstdint>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "katz.h"

namespace katz {

// Error carrying a katz_status code.
struct Error {
  int code;
  std::string msg;
};
[[noreturn]] void fail(int code, const std::string& msg);

// parallel_for over [0, n) in contiguous chunks on the host's cores.
void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)>& fn, int64_t grain = 4096);
int host_threads();

// ------------------------------------------------------------ host index
struct HostIndex {
  int32_t n = 0, n1 = 0, n2 = 0;
  int64_t nnz = 0;
  double beta = 0, lambda_max = 0, c = 0;
  bool weighted = false;
  std::vector<int32_t> perm;   // perm[v]  = new position of original node v
  std::vector<int32_t> iperm;  // iperm[i] = original node at new position i
  // adjacency in the new order: rows sorted, split[i] = first entry of row i
  // whose column is a separator position (>= n1)
  std::vector<int32_t> rp, col, split;
  std::vector<double> val;
  // M11 blocks: block b covers new positions [blk_start[b], blk_start[b+1]);
  // its inverse (I - beta A_bb)^{-1} is stored row-major at minv[blk_off[b]]
  std::vector<int32_t> blk_start;
  std::vector<int64_t> blk_off;
  std::vector<double> minv;
  // separator: L L^T = M22 (CHOL) or L = I (IDENTITY)
  int32_t l_kind = KATZ_L_IDENTITY;
  std::vector<double> ginv;    // n2 x n2 M22^{-1} (CHOL only)
  std::vector<double> lchol;   // n2 x n2 lower factor of M22 (CHOL only)
  // rank-r preconditioner: V = L^{-T} U (row-major n2 x r), D = s/(1-s)
  int32_t rank = 0;
  std::vector<double> U, V, sigma, D;
  double sigma_next = 0;
  int32_t lanczos_steps = 0;
  int32_t lanczos_rank = 0, lanczos_steps_req = 0;  // a deferred Lanczos run
  uint64_t lanczos_seed = 0;
  int32_t precision = KATZ_PREC_FP64;
  int32_t u_precision = 0;  // resolved: 1 FP64, 2 FP32, 3 BF16 (FP64 path); BF16 on the mixed path
  int32_t u_precision_req = 0;  // as requested (0: auto, resolved once the Ritz values are known)
  double build_seconds = 0;
  double phase_seconds[12] = {0};  // see katz_index_info_t::build_phase_seconds
};

// defer_lanczos: leave the low-rank factor out (rank 0) and record what it
// needs in H.lanczos_rank / lanczos_steps_req / lanczos_seed, for a Lanczos
// run on the device (device_lanczos_R).
void build_host_index(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col,
                      const double* val, const katz_build_opts& o, HostIndex& H, bool defer_lanczos = false);
// Lanczos pieces shared by the host and device runs: the seeded normal
// stream of the start / restart vectors, and the Ritz pairs of the
// tridiagonal (fills rank, sigma, D, sigma_next, lanczos_steps; returns the
// coefficients z, Ritz vector t = sum_k z[t * mm + k] q_k).
void lanczos_normals(uint64_t& state, double* out, int64_t n);
std::vector<double> lanczos_ritz(HostIndex& H, const std::vector<double>& al, const std::vector<double>& be,
                                 int32_t r);
// The index of the same graph and partition for other options (beta, rank,
// factor kind, precision, storage, seed, steps): S's structure reused, the
// beta-dependent factors computed afresh (katz_index_rebuild).
void rebuild_host_index(const HostIndex& S, const katz_build_opts& o, HostIndex& H, bool defer_lanczos = false);
// Louvain local moving with communities capped at `cap` nodes, for the
// initial parts of an unlabeled graph (katz_communities); returns the passes
// run.
int32_t communities(int32_t n, int64_t nnz, const int32_t* rp, const int32_t* col, const double* val,
                    int32_t cap, int32_t passes, int32_t* labels);
// Whether the Lanczos on R should run on the device for these options.
bool lanczos_on_device(const HostIndex& H, const katz_build_opts& o);
// Index files (index_io.cpp): a loaded index is fully validated.
void save_host_index(const HostIndex& H, const char* path);
void load_host_index(const char* path, HostIndex& H);

// ------------------------------------------------------------ lambda_max
// The vector work of the Lanczos iteration for lambda_max(A) (host or
// device storage): start from q0 (unit norm), w = A q with <q, w>,
// w -= a q + bprev qp with <w, w>, then qp = q, q = w / bj.
struct LambdaOps {
  virtual ~LambdaOps() = default;
  virtual void start(const double* q0) = 0;
  virtual double apply_dot() = 0;
  virtual double update_norm2(double a, double bprev) = 0;
  virtual void advance(double bj) = 0;
};
double lambda_max_with(int32_t n, uint64_t seed, LambdaOps& ops);
// Graphs of at least this many nodes take lambda_max on the device when the
// build has one (KATZ_LAMBDA_DEVICE=0: on the host).
constexpr int32_t kLambdaDeviceMin = 2000000;
double device_lambda_max(int device, int32_t n, int64_t nnz, const int32_t* rp, const int32_t* col,
                         const double* val, uint64_t seed);

// ------------------------------------------------------- device index
struct DeviceIndex;            // defined in the HIP solver
DeviceIndex* device_upload(const HostIndex& H, int device);
// Top eigenpairs of R on the device (L = I), as the host Lanczos computes
// them; fills the low-rank fields of H and uploads the factors.
void device_lanczos_R(HostIndex& H, DeviceIndex* D);
void device_free(DeviceIndex* D);
int64_t device_bytes(const DeviceIndex* D);
int64_t device_factor_bytes(const DeviceIndex* D);

struct QueryArgs {
  const int32_t* q;
  int32_t nq;
  katz_query_opts opts;
  double* scores;          // nq*n or NULL
  int32_t topk;            // 0: no top-K
  int32_t* ids;            // nq*topk
  double* topk_scores;     // nq*topk or NULL
  katz_query_stats* st;
  void* stream;
  // pair mode (npairs > 0): entries K[row, q[col]] for pairs sorted by col;
  // pair_row in the permuted order; pair_out host FP64 [npairs]
  int32_t npairs = 0;
  const int32_t* pair_col = nullptr;
  const int32_t* pair_row = nullptr;
  double* pair_out = nullptr;   // host or device
};
int device_query(const HostIndex& H, DeviceIndex* D, const QueryArgs& a);
// Algorithm 3 after the k_q solve: the modular nodes' Katz vectors as one
// batched solve of the distinct sources q_src with device pair gathers
// (pair p: row prow[p], column pcol[p], sorted by column), then the
// correlation and re-ranking on the device (device_sparse_rerank).
int device_sparse_katz(const HostIndex& H, DeviceIndex* D, const katz_query_opts& opts, void* stream,
                       const std::vector<int32_t>& q_src, const std::vector<int32_t>& pcol,
                       const std::vector<int32_t>& prow, const std::vector<int32_t>& inv,
                       const std::vector<int64_t>& base, const std::vector<int32_t>& ncand,
                       const std::vector<int32_t>& nmod, const std::vector<int32_t>& cand, int nq, int s,
                       katz_query_stats* pst, int32_t* ids, double* corr);
// As device_query for scores only (no top-K or pairs), on the caller's
// stream, with every buffer of the solve in the library's static device
// scratch: no device or pinned allocation, no graph capture.
int device_query_noalloc(const HostIndex& H, DeviceIndex* D, const QueryArgs& a);
// Serializes an open HIP graph capture (one thread) with the operations of
// other threads that may synchronize with the legacy stream (allocation,
// frees, synchronous copies and memsets, stream and event creation, work on
// the NULL stream): HIP rejects those while a capture is open, and the
// capture fails with them.
std::recursive_mutex& hip_global_mu();
// Copies host bytes to a caller buffer that may be host or device memory.
void copy_to_caller(void* dst, const void* src, size_t bytes);
// Device workspace (panels, partial sums, stream) reusable across calls.
struct Workspace;
Workspace* ws_create(DeviceIndex* D, int cap);
void ws_destroy(DeviceIndex* D, Workspace* w);
int ws_capacity(const Workspace* w);
// Device bytes one column of workspace capacity takes.
int64_t ws_bytes_per_column(const DeviceIndex* D);
// As device_query, on the given workspace when it is large enough (NULL: pooled).
int device_query_ws(const HostIndex& H, DeviceIndex* D, const QueryArgs& a, Workspace* w);
int profile_enable(int on);
void profile_reset();
int profile_read(katz_kernel_stat* out, int max);

}  // namespace katz

namespace katz {
struct Server;
}

struct katz_index {
  katz::HostIndex host;
  katz::DeviceIndex* dev = nullptr;
  int device = -1;
};
