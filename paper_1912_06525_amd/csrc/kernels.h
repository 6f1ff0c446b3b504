// Device kernels of the query path (gfx950, wave64).  Included by solver.hip
// only.  All panels are node-major: an m x B panel stores the B values of one
// node contiguously (element (i, j) at [i * B + j]), so one adjacency entry
// gathers one contiguous B-wide row.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace katz {
namespace dev {

constexpr int WG = 256;   // threads per workgroup (4 wave64s)
constexpr int MAXC = 8;   // column accumulators per lane in the SpMM (B <= 8 * CW)

// Per-column solver state in device memory (B entries each).
struct ColState {
  double* rz;      // <r, z> (<r, r> for plain CG)
  double* pq;      // <p, S p> or <p, M p>
  double* alpha;   // step length
  double* bcg;     // direction coefficient
  double* rr;      // <r, r> of the recurrence residual
  double* thr;     // stop when rr <= thr
  int* active;     // 1 while the column iterates
  int* status;     // 0 ok, 1 breakdown (<p, q> <= 0 or not finite), 2 iteration cap
  int* iters;      // iterations taken in this solve
  int* n_active;   // number of active columns (scalar)
  const int* mask; // columns taking part in this solve (1) or not (0)
  int max_iter;
};

// ----------------------------------------------------------- XCD slabs
// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b on XCD
// b % 8), and each XCD has its own L2.  xcd_slab gives workgroup `bid` of
// `nwg` the chunk range of its XCD: nchunks split into 8 contiguous slabs, the
// XCD's workgroups striding through the slab together, so rows processed at
// the same time on one XCD are neighbours in the node order.
struct Slab {
  int64_t first, end, stride;
};
// Workgroup bid of nwg: nchunks split into nx = min(8, nwg) balanced
// contiguous slabs; slab x is walked by the workgroups with bid % nx == x, in
// steps of their count.  Every chunk is visited exactly once.
// Contiguous alternative: workgroup bid takes chunks [bid * c, (bid + 1) * c).
__device__ inline Slab contiguous_slab(int bid, int nwg, int64_t nchunks) {
  const int64_t c = (nchunks + nwg - 1) / nwg;
  Slab s;
  s.first = (int64_t)bid * c;
  s.end = min<int64_t>(nchunks, s.first + c);
  s.stride = 1;
  return s;
}
__device__ inline Slab xcd_slab(int bid, int nwg, int64_t nchunks) {
  const int nx = nwg < 8 ? nwg : 8;
  const int x = bid % nx;
  const int64_t q = nchunks / nx, rem = nchunks % nx;
  const int64_t start = (int64_t)x * q + (x < rem ? x : rem);
  Slab s;
  s.first = start + bid / nx;
  s.end = start + q + (x < rem ? 1 : 0);
  s.stride = (nwg - x + nx - 1) / nx;
  return s;
}

// -------------------------------------------------------------- reduction
// Recounts the active columns (one thread) after an epilogue changed them.
__device__ inline void recount_active(const ColState& cs, int B) {
  __syncthreads();
  if (threadIdx.x == 0) {
    int c = 0;
    for (int j = 0; j < B; j++) c += cs.active[j];
    *cs.n_active = c;
  }
}

__device__ inline bool finite_pos(double x) { return x > 0.0 && x < 1.0e308; }

// One-workgroup reduction of NT threads: sums partials[w * nv + v] over
// w < nwg for every v < nv with all threads (lanes over v, then over w; fixed
// tree order, so the result is deterministic) and calls f(v, sum) once per v.
template <int NT, typename F>
__device__ inline void final_reduce(const double* partials, int nwg, int nv, F&& f) {
  __shared__ double red[NT];
  int VC = 1;
  while (VC < nv && VC < NT) VC <<= 1;
  const int WR = NT / VC;
  const int tid = threadIdx.x, vl = tid % VC, wl = tid / VC;
  for (int v0 = 0; v0 < nv; v0 += VC) {
    const int v = v0 + vl;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (v < nv) {
      int w = wl;
      // 16 loads in flight per lane (the partials come from other XCDs' L2s,
      // so each round trip is long), combined in a fixed order
      for (; w + 15 * WR < nwg; w += 16 * WR) {
        double t[16];
#pragma unroll
        for (int u = 0; u < 16; u++) t[u] = partials[(int64_t)(w + u * WR) * nv + v];
#pragma unroll
        for (int u = 0; u < 16; u += 4) {
          s0 += t[u];
          s1 += t[u + 1];
          s2 += t[u + 2];
          s3 += t[u + 3];
        }
      }
      for (; w + 3 * WR < nwg; w += 4 * WR) {
        s0 += partials[(int64_t)w * nv + v];
        s1 += partials[(int64_t)(w + WR) * nv + v];
        s2 += partials[(int64_t)(w + 2 * WR) * nv + v];
        s3 += partials[(int64_t)(w + 3 * WR) * nv + v];
      }
      for (; w < nwg; w += WR) s0 += partials[(int64_t)w * nv + v];
    }
    if (VC < 64) {
      // lanes of a wave that share a value (tid % VC) first combine by a
      // fixed shuffle tree, then the NT / 64 wave sums in order: two
      // barriers instead of one per tree level
      double s = (s0 + s1) + (s2 + s3);
#pragma unroll
      for (int off = VC; off < 64; off <<= 1) s += __shfl_xor(s, off, 64);
      const int wave = tid / 64, lane = tid % 64;
      if (lane < VC) red[wave * VC + lane] = s;
      __syncthreads();
      if (tid < VC) {
        double t = 0.0;
        for (int wv = 0; wv < NT / 64; wv++) t += red[wv * VC + tid];
        if (v < nv) f(v, t);
      }
      __syncthreads();
      continue;
    }
    red[tid] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    for (int off = WR / 2; off > 0; off >>= 1) {
      if (wl < off) red[tid] += red[tid + off * VC];
      __syncthreads();
    }
    if (wl == 0 && v < nv) f(v, red[tid]);
    __syncthreads();
  }
}

}  // namespace dev
}  // namespace katz
