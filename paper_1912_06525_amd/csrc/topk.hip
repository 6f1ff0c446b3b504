// Top-K link prediction (Sec. 3.3: rank the nodes by their Katz score for the
// query; Algorithm 3 sorts k_q in descending order).  Candidates are all nodes
// except q and its neighbours; ties are broken by ascending original node id.
//
// Exact selection per column by radix select over the 96-bit key
// (order-preserving bits of the FP64 score, ~id): 8-bit digits from the top,
// one histogram pass + one select step per digit, stopping as soon as the
// bucket holding the K-th key is taken whole.  The <= K winners are then
// sorted in LDS (bitonic) by the same key.  Excluded nodes get the key of
// -inf, so they only fill slots when fewer than K candidates exist; such
// slots are reported as id -1, score NaN.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "katz_internal.h"
#include "kernels.h"

#define HIPCHECK(x)                                                                     \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess) fail(KATZ_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

namespace katz {
namespace tk {

constexpr int WG = 256;
constexpr int KMAX = 4096;

__device__ inline uint64_t score_key(double s) {
  uint64_t b = (uint64_t)__double_as_longlong(s);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ULL);
}
__device__ inline double key_score(uint64_t k) {
  uint64_t b = (k >> 63) ? (k & 0x7FFFFFFFFFFFFFFFULL) : ~k;
  return __longlong_as_double((long long)b);
}
// key of -inf: every finite score has a larger key
__device__ inline uint64_t excluded_key() { return ~(uint64_t)0xFFF0000000000000ULL; }

struct ColSel {
  uint64_t hi;    // selected prefix, high 64 bits
  uint32_t lo;    // selected prefix, low 32 bits (~id)
  int32_t krem;   // elements still to take inside the prefix bucket
  int32_t done;   // selection finished: take every key >= (hi, lo)
  int32_t count;  // collected winners
};

// digit p (0..11) of the 96-bit key, most significant first
__device__ inline uint32_t digit(uint64_t hi, uint32_t lo, int p) {
  return p < 8 ? (uint32_t)(hi >> (56 - 8 * p)) & 255u : (lo >> (24 - 8 * (p - 8))) & 255u;
}
// does (hi, lo) agree with the selected prefix on digits 0..p-1?
__device__ inline bool prefix_match(uint64_t hi, uint32_t lo, const ColSel& s, int p) {
  if (p == 0) return true;
  if (p <= 8) {
    int sh = 64 - 8 * p;
    return (hi >> sh) == (s.hi >> sh);
  }
  if (hi != s.hi) return false;
  int sh = 32 - 8 * (p - 8);
  return (lo >> sh) == (s.lo >> sh);
}

// Scores of excluded nodes (q and its neighbours) set to -inf, in place.
__global__ void k_exclude(const int32_t* qpos, int B, const int32_t* rp, const int32_t* col, double* K) {
  const int j = blockIdx.x;
  const int32_t r = qpos[j];
  if (threadIdx.x == 0) K[(int64_t)r * B + j] = -INFINITY;
  for (int32_t k = rp[r] + threadIdx.x; k < rp[r + 1]; k += blockDim.x) K[(int64_t)col[k] * B + j] = -INFINITY;
}

__global__ void k_init(ColSel* sel, int B, int K, unsigned* hist) {
  for (int j = threadIdx.x; j < B; j += blockDim.x) {
    sel[j].hi = 0;
    sel[j].lo = 0;
    sel[j].krem = K;
    sel[j].done = 0;
    sel[j].count = 0;
  }
  for (int i = threadIdx.x; i < B * 256; i += blockDim.x) hist[i] = 0;
}

__global__ __launch_bounds__(WG) void k_hist(int n, int B, const double* K, const int32_t* iperm, const ColSel* sel,
                                             int p, int chunk, unsigned* hist) {
  const int j = blockIdx.y;
  const ColSel s = sel[j];
  if (s.done) return;
  __shared__ unsigned h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int i0 = blockIdx.x * chunk, i1 = min(n, i0 + chunk);
  for (int i = i0 + threadIdx.x; i < i1; i += WG) {
    uint64_t hi = score_key(K[(int64_t)i * B + j]);
    uint32_t lo = p >= 8 ? ~(uint32_t)iperm[i] : 0u;
    if (prefix_match(hi, lo, s, p)) atomicAdd(&h[digit(hi, lo, p)], 1u);
  }
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&hist[j * 256 + threadIdx.x], h[threadIdx.x]);
}

// One workgroup per column: choose the digit of the K-th largest key.
__global__ void k_select(int B, ColSel* sel, unsigned* hist, int p) {
  const int j = blockIdx.x;
  __shared__ unsigned c[256];
  c[threadIdx.x] = hist[j * 256 + threadIdx.x];
  __syncthreads();
  hist[j * 256 + threadIdx.x] = 0;
  if (threadIdx.x == 0 && !sel[j].done) {
    ColSel s = sel[j];
    unsigned above = 0, total = 0;
    for (int d = 0; d < 256; d++) total += c[d];
    if (total <= (unsigned)s.krem) {
      // every element in the bucket is taken: threshold = prefix, digit 0
      s.done = 1;
    } else {
      int d = 255;
      for (; d > 0; d--) {
        if (above + c[d] >= (unsigned)s.krem) break;
        above += c[d];
      }
      if (p < 8) s.hi |= (uint64_t)d << (56 - 8 * p);
      else s.lo |= (uint32_t)d << (24 - 8 * (p - 8));
      s.krem -= (int)above;
      if (c[d] == (unsigned)s.krem || p == 11) s.done = 1;
    }
    sel[j] = s;
  }
}

// Collects every key >= the selected threshold (at most K per column).
__global__ __launch_bounds__(WG) void k_collect(int n, int B, const double* K, const int32_t* iperm, ColSel* sel,
                                                int chunk, int kcap, uint64_t* bhi, uint32_t* blo) {
  const int j = blockIdx.y;
  const uint64_t thi = sel[j].hi;
  const uint32_t tlo = sel[j].lo;
  const int i0 = blockIdx.x * chunk, i1 = min(n, i0 + chunk);
  for (int i = i0 + threadIdx.x; i < i1; i += WG) {
    uint64_t hi = score_key(K[(int64_t)i * B + j]);
    if (hi < thi) continue;
    uint32_t lo = ~(uint32_t)iperm[i];
    if (hi == thi && lo < tlo) continue;
    int slot = atomicAdd(&sel[j].count, 1);
    if (slot < kcap) {
      bhi[(int64_t)j * kcap + slot] = hi;
      blo[(int64_t)j * kcap + slot] = lo;
    }
  }
}

// Sorts a column's winners by (key desc) and writes ids / scores.
__global__ __launch_bounds__(WG) void k_sort_out(int B, int K, int kpow, const ColSel* sel, const uint64_t* bhi,
                                                 const uint32_t* blo, int kcap, int32_t* ids, double* scores) {
  extern __shared__ unsigned char smem[];
  uint64_t* sh = (uint64_t*)smem;
  uint32_t* sl = (uint32_t*)(sh + kpow);
  const int j = blockIdx.x;
  const int cnt = min(sel[j].count, kcap);
  for (int t = threadIdx.x; t < kpow; t += WG) {
    if (t < cnt) {
      sh[t] = bhi[(int64_t)j * kcap + t];
      sl[t] = blo[(int64_t)j * kcap + t];
    } else {
      sh[t] = 0;
      sl[t] = 0;
    }
  }
  __syncthreads();
  // bitonic sort, descending by (hi, lo)
  for (int size = 2; size <= kpow; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < kpow; t += WG) {
        int u = t ^ stride;
        if (u > t) {
          bool desc = (t & size) == 0;
          uint64_t ah = sh[t], bh = sh[u];
          uint32_t al = sl[t], bl = sl[u];
          bool a_lt_b = ah < bh || (ah == bh && al < bl);
          if (desc ? a_lt_b : !a_lt_b) {
            sh[t] = bh; sh[u] = ah;
            sl[t] = bl; sl[u] = al;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int t = threadIdx.x; t < K; t += WG) {
    int32_t id = -1;
    double sc = NAN;
    if (t < cnt && sh[t] > excluded_key()) {
      id = (int32_t)~sl[t];
      sc = key_score(sh[t]);
    }
    ids[(int64_t)j * K + t] = id;
    if (scores) scores[(int64_t)j * K + t] = sc;
  }
}

}  // namespace tk

// Runs the selection on the permuted score panel Kp (n x B, modified in place:
// excluded entries become -inf).  ids/scores are device buffers, query-major.
void device_topk(int n, int B, int K, double* Kp, const int32_t* qpos, const int32_t* rp, const int32_t* col,
                 const int32_t* iperm, void* scratch, size_t scratch_bytes, int32_t* ids, double* scores,
                 hipStream_t st) {
  using namespace tk;
  if (K > KMAX) fail(KATZ_EINVAL, "k must be <= 4096");
  size_t need = sizeof(ColSel) * B + sizeof(unsigned) * 256 * B + (sizeof(uint64_t) + sizeof(uint32_t)) * (size_t)K * B + 64;
  if (need > scratch_bytes) fail(KATZ_EDEVICE, "internal: top-K scratch too small");
  char* p = (char*)scratch;
  ColSel* sel = (ColSel*)p;
  p += ((sizeof(ColSel) * B + 15) / 16) * 16;
  unsigned* hist = (unsigned*)p;
  p += sizeof(unsigned) * 256 * B;
  uint64_t* bhi = (uint64_t*)p;
  p += sizeof(uint64_t) * (size_t)K * B;
  uint32_t* blo = (uint32_t*)p;
  k_exclude<<<B, WG, 0, st>>>(qpos, B, rp, col, Kp);
  k_init<<<1, WG, 0, st>>>(sel, B, K, hist);
  const int chunk = 4096;
  dim3 g((n + chunk - 1) / chunk, B);
  for (int pass = 0; pass < 12; pass++) {
    k_hist<<<g, WG, 0, st>>>(n, B, Kp, iperm, sel, pass, chunk, hist);
    k_select<<<B, 256, 0, st>>>(B, sel, hist, pass);
  }
  k_collect<<<g, WG, 0, st>>>(n, B, Kp, iperm, sel, chunk, K, bhi, blo);
  int kpow = 1;
  while (kpow < K) kpow <<= 1;
  size_t shm = (size_t)kpow * (sizeof(uint64_t) + sizeof(uint32_t));
  k_sort_out<<<B, WG, shm, st>>>(B, K, kpow, sel, bhi, blo, K, ids, scores);
}

}  // namespace katz
