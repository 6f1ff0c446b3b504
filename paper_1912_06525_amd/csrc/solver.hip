// Query path on the GPU: device index, kernels and the solve loops.
//
// Per query batch (B columns, node-major panels, permuted node order):
//   a1  b = beta A e_q                           (k_rhs_scatter)
//   a2  t = M11^{-1} b1, f = b2 - M12^T t        (k_m11_apply, k_spmm)
//   a3  PCG on S k2 = f with S~^{-1}             (k_m11_apply + k_spmm = S p,
//                                                 k_vt + k_lowrank = S~^{-1} r,
//                                                 k_update_r / k_update_p)
//   a4  k1 = M11^{-1} (b1 - M12 k2)              (k_m11_apply)
//   a6  true residual b - M k in FP64, refine    (k_spmm, k_axpy_mask)
//   a5  unpermute to query-major output          (k_unpermute)
//   a8  plain CG on M: k_spmm + k_update_r + k_update_p
// M12 = -beta A12, M22 = I - beta A22 and M11 = I - beta A11 are applied from
// one permuted CSR of A whose rows carry a split between block columns and
// separator columns.
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <map>
#include <tuple>
#include <memory>
#include <mutex>
#include <type_traits>

#include "katz_internal.h"
#include "kernels.h"

#define HIPCHECK(x)                                                                     \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess) fail(KATZ_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

namespace katz {
using namespace dev;

typedef __hip_bfloat16 bf16;
__device__ inline double to_d(double x) { return x; }
__device__ inline double to_d(float x) { return (double)x; }
__device__ inline double to_d(bf16 x) { return (double)__bfloat162float(x); }

enum Ep { EP_NONE = 0, EP_PQ = 1, EP_RES = 2, EP_RR_INIT = 3, EP_RR = 4, EP_RZ_INIT = 5, EP_RZ = 6,
          EP_RR_CG = 7, EP_NORM = 8, EP_VT = 9, EP_RR_VT = 10 };

// ==================================================================== kernels
// Fill a buffer with a value.
template <typename T>
__global__ void k_fill(T* p, int64_t n, T v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// a1: scatter b[:, j] = beta * A[:, q_j] (rows of the permuted CSR are the
// columns of A by symmetry).  The panel was zero-filled before.
template <typename T>
__global__ void k_rhs_scatter(const int32_t* qpos, int B, const int32_t* rp, const int32_t* col,
                              const double* val, double beta, T* b) {
  int j = blockIdx.x;
  if (j >= B) return;
  int32_t r = qpos[j];
  for (int32_t k = rp[r] + threadIdx.x; k < rp[r + 1]; k += blockDim.x)
    b[(int64_t)col[k] * B + j] = (T)(beta * (val ? val[k] : 1.0));
}

// ||b_j||^2 from the query row itself (its entries are distinct columns): the
// sum of (beta a_k)^2, one wave per column, instead of a pass over the panel.
__global__ void k_rhs_norm2(const int32_t* qpos, int B, const int32_t* rp, const double* val, double beta,
                            double* out) {
  const int j = blockIdx.x;
  if (j >= B) return;
  const int32_t r = qpos[j];
  double s = 0.0;
  for (int32_t k = rp[r] + (int)threadIdx.x; k < rp[r + 1]; k += (int)blockDim.x) {
    const double v = beta * (val ? val[k] : 1.0);
    s += v * v;
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (threadIdx.x == 0) out[j] = s;
}

// ------------------------------------------------------------------- SpMM
// y[i] = cv v[i] + cw w[i] + ca (A_<split x)[i] + cb (A_>=split x)[i] for the
// rows [row0, row1) of the permuted CSR; x is a full n-row panel, v, w, y are
// row-aligned to row0.  Short rows: teams of TS lanes per row, CW of them
// across columns and TS/CW across the row's entries (partials combined by
// cross-lane shuffles).  Rows longer than long_thr (hubs) get a whole
// workgroup each (the first n_long workgroups).  Optional per-column dot
// <d, y> (d = dotv or y) with a last-workgroup epilogue.  TX: the element
// type of x and w (FP32 for the precision form's residual update, whose sums
// and output stay FP64).
template <typename T, typename TX = T>
struct SpmmArgs {
  int row0, row1, rows_per_wg;  // rows_per_wg = rows per chunk
  int64_t nchunks;              // short-row chunks
  int xcd;                      // walk them in XCD slabs (1) or contiguously (0)
  const int32_t* rp;
  const int32_t* col;
  const int32_t* split;
  const double* val;
  const TX* x;
  T ca, cb;
  int parts;  // bit 0: entries left of the split, bit 1: right of it
  const T* v;
  T cv;
  const TX* w;
  T cw;
  T* y;
  int B;       // columns this launch computes
  int ld, j0;  // row stride of every panel (the batch width) and this launch's first column
  int ep;
  const T* dotv;
  double* partials;
  double* out;  // EP_RES destination
  ColState cs;
  const int* n_active;       // early exit when *n_active == 0 (NULL: never)
  const int32_t* long_rows;  // rows with more than long_thr entries, ascending
  int n_long, long_thr;
};

// Accumulates lane (nz, cl)'s share of row i: entries kb+nz, kb+nz+NZ, ...
// (four entries in flight per step).
// NCM: column groups per lane (CW = 64 takes B up to 64 * NCM; narrower
// layouts have B <= CW and NCM = 1), a compile-time count so that every
// gather of an entry is issued at once.

// VAL: weighted graph (entry values in a.val).  A compile-time switch: a
// runtime test between the loads makes the compiler wait for each one.
// Entry range [kb, ke) of row i taken by this launch and the split point sp
// (entries before sp take ca, the others cb); len = the row's full length.
struct RowRange {
  int32_t kb, ke, sp, len;
};
template <typename T, typename TX>
__device__ inline RowRange row_range(const SpmmArgs<T, TX>& a, int i) {
  RowRange r;
  const int32_t s = a.rp[i], e = a.rp[i + 1];
  r.len = e - s;
  r.sp = a.split[i];
  r.kb = (a.parts & 1) ? s : r.sp;
  r.ke = (a.parts & 2) ? e : r.sp;
  return r;
}

// Args: any argument struct with col, val, x, B, ca and cb.
template <typename T, int CW, int NZ, bool VAL, int NCM, typename Args>
__device__ inline void row_gather(const Args& a, const RowRange& rr, int nz, int cl, int NC, T* acc) {
  const int32_t kb = rr.kb, ke = rr.ke, sp = rr.sp;
  const int B = a.B;
  // the lane's column in each group, clamped into [0, B) for a ragged last
  // group: every gather is an in-bounds load issued unconditionally (so the
  // loads of an entry are in flight together) and only the accumulation is
  // masked
  int jc[NCM];
  bool jok[NCM];
#pragma unroll
  for (int cc = 0; cc < NCM; cc++) {
    const int j = cl + CW * cc;
    jok[cc] = cc < NC && j < B;
    jc[cc] = j < B ? j : B - 1;
  }
  int32_t k = kb + nz;
  for (; k + 3 * NZ < ke; k += 4 * NZ) {
    int32_t c[4];
    T cf[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const int32_t kk = k + u * NZ;
      c[u] = a.col[kk];
      cf[u] = (kk < sp) ? a.ca : a.cb;
      if (VAL) cf[u] *= (T)a.val[kk];
    }
    T xv[4][NCM];
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const auto* xr = a.x + (int64_t)c[u] * a.ld + a.j0;
#pragma unroll
      for (int cc = 0; cc < NCM; cc++) xv[u][cc] = (T)xr[jc[cc]];
    }
#pragma unroll
    for (int u = 0; u < 4; u++) {
#pragma unroll
      for (int cc = 0; cc < NCM; cc++)
        if (jok[cc]) acc[cc] += cf[u] * xv[u][cc];
    }
  }
  if (k < ke) {
    // tail of at most 3 entries per lane (most rows of a sparse graph end
    // here), branch-free so that all its loads are in flight together: an
    // index past the row's end is clamped to its last entry (a valid load)
    // and its product masked to 0
    int32_t c[3];
    T cf[3];
#pragma unroll
    for (int u = 0; u < 3; u++) {
      const int32_t kk = k + u * NZ;
      const bool ok = kk < ke;
      const int32_t kc = ok ? kk : ke - 1;
      c[u] = a.col[kc];
      cf[u] = (kk < sp) ? a.ca : a.cb;
      if (VAL) cf[u] *= (T)a.val[kc];
    }
    T xv[3][NCM];
#pragma unroll
    for (int u = 0; u < 3; u++) {
      const auto* xr = a.x + (int64_t)c[u] * a.ld + a.j0;
#pragma unroll
      for (int cc = 0; cc < NCM; cc++) xv[u][cc] = (T)xr[jc[cc]];
    }
#pragma unroll
    for (int cc = 0; cc < NCM; cc++) {
      if (jok[cc]) {
#pragma unroll
        for (int u = 0; u < 3; u++) acc[cc] += (k + u * NZ < ke) ? cf[u] * xv[u][cc] : (T)0;
      }
    }
  }
}

// Row-aligned operands of row i for the lane owning column group cl,
// loaded before they are needed (for one accumulator per lane, at the start
// of the row, so their latency overlaps the gather).
template <typename T, int NCM>
struct RowOps {
  T v[NCM], w[NCM];
  double d[NCM];
};
template <typename T, int CW, int NCM, typename TX>
__device__ inline void row_load(const SpmmArgs<T, TX>& a, int i, int cl, int NC, RowOps<T, NCM>& p) {
  const int B = a.B;
  const int64_t ro = (int64_t)(i - a.row0) * a.ld + a.j0;
  // clamped columns (a ragged last group reads column B - 1, unused): one
  // uniform branch per operand with all of its loads, none per column group,
  // so the loads are in flight together and no later store waits on them
  int jc[NCM];
#pragma unroll
  for (int cc = 0; cc < NCM; cc++) {
    const int j = cl + CW * cc;
    jc[cc] = j < B ? j : B - 1;
    p.v[cc] = p.w[cc] = (T)0;
    p.d[cc] = 0.0;
  }
  (void)NC;
  if (a.v) {
#pragma unroll
    for (int cc = 0; cc < NCM; cc++) p.v[cc] = a.v[ro + jc[cc]];
  }
  if (a.w) {
#pragma unroll
    for (int cc = 0; cc < NCM; cc++) p.w[cc] = (T)a.w[ro + jc[cc]];
  }
  if (a.ep != EP_NONE && a.dotv) {
    if (a.dotv == a.v) {
#pragma unroll
      for (int cc = 0; cc < NCM; cc++) p.d[cc] = (double)p.v[cc];
    } else {
#pragma unroll
      for (int cc = 0; cc < NCM; cc++) p.d[cc] = (double)a.dotv[ro + jc[cc]];
    }
  }
}

// Finishes row i for the lane owning column group cl: adds the row-aligned
// operands, stores y and accumulates the dot (in place, y == v, is allowed:
// the lane has loaded v before).  Every group's value is formed before the
// first store.
template <typename T, int CW, int NCM, typename TX>
__device__ inline void row_finish(const SpmmArgs<T, TX>& a, int i, int cl, int NC, const T* acc,
                                  const RowOps<T, NCM>& p, double* dacc) {
  const int B = a.B;
  const int64_t ro = (int64_t)(i - a.row0) * a.ld + a.j0;
  T yv[NCM];
#pragma unroll
  for (int cc = 0; cc < NCM; cc++) {
    yv[cc] = acc[cc];
    if (a.v) yv[cc] += a.cv * p.v[cc];
    if (a.w) yv[cc] += a.cw * p.w[cc];
  }
#pragma unroll
  for (int cc = 0; cc < NCM; cc++) {
    const int j = cl + CW * cc;
    if (cc < NC && j < B) {
      a.y[ro + j] = yv[cc];
      if (a.ep != EP_NONE) {
        double d = a.dotv ? p.d[cc] : (double)yv[cc];
        dacc[cc] += d * (double)yv[cc];
      }
    }
  }
}

// Per-column sums of the owners' dacc over the workgroup's teams (a fixed
// tree), stored as partial row `prow`: partials[prow * ld + j0 + j].  Called
// by every thread of the workgroup.
template <typename T, int TEAMS, int CW, int NCM, typename TX>
__device__ inline void spmm_store_partials(const SpmmArgs<T, TX>& a, double* sh, const double* dacc, bool owner,
                                           int slot, int cl_own, int64_t prow) {
  const int tid = threadIdx.x, B = a.B, NC = (B + CW - 1) / CW;
  for (int j = tid; j < TEAMS * B; j += WG) sh[j] = 0.0;
  __syncthreads();
  if (owner) {
#pragma unroll
    for (int c = 0; c < NCM; c++) {
      const int j = cl_own + CW * c;
      if (c < NC && j < B) sh[slot * B + j] = dacc[c];
    }
  }
  __syncthreads();
  double* out = a.partials + prow * a.ld + a.j0;
  if (B * TEAMS <= WG) {
    // tree over teams: thread (t, j) with t < TEAMS
    const int t = tid / B, j = tid % B;
    for (int off = TEAMS / 2; off > 0; off >>= 1) {
      if (t < off) sh[t * B + j] += sh[(t + off) * B + j];
      __syncthreads();
    }
    if (tid < B) out[tid] = sh[tid];
  } else {
    for (int j = tid; j < B; j += WG) {
      double s = 0.0;
      for (int t = 0; t < TEAMS; t++) s += sh[t * B + j];
      out[j] = s;
    }
  }
  __syncthreads();
}

template <typename T, int TS, int CW, bool VAL, int NCM, typename TX = T>
__global__ __launch_bounds__(WG) void k_spmm(SpmmArgs<T, TX> a) {
  if (a.n_active && *a.n_active == 0) return;
  constexpr int NZ = TS / CW;
  constexpr int TEAMS = WG / TS;
  constexpr int NZW = WG / CW;  // entry lanes of the long-row path
  extern __shared__ double sh[];
  const int tid = threadIdx.x;
  const int B = a.B;
  const int NC = (B + CW - 1) / CW;
  const bool ep = a.ep != EP_NONE;
  double dacc[NCM];
#pragma unroll
  for (int c = 0; c < NCM; c++) dacc[c] = 0.0;
  if ((int)blockIdx.x < a.n_long) {
    // ---- one hub row, whole workgroup; its dot terms are partial row blockIdx.x
    const int cl = tid % CW, nz = tid / CW;
    const int i = a.long_rows[blockIdx.x];
    RowOps<T, NCM> ops;
    if (tid < CW) row_load<T, CW, NCM>(a, i, tid, NC, ops);
    T acc[NCM];
#pragma unroll
    for (int c = 0; c < NCM; c++) acc[c] = (T)0;
    row_gather<T, CW, NZW, VAL, NCM>(a, row_range(a, i), nz, cl, NC, acc);
    // lanes of one wave sharing cl: xor over the wave; then across waves in LDS
#pragma unroll
    for (int c = 0; c < NCM; c++) {
#pragma unroll
      for (int off = CW; off < 64; off <<= 1) acc[c] += __shfl_xor(acc[c], off, 64);
    }
    const int wave = tid / 64, lw = tid % 64;
    if (lw < CW) {
#pragma unroll
      for (int c = 0; c < NCM; c++)
        if (c < NC) sh[(wave * NCM + c) * CW + lw] = (double)acc[c];
    }
    __syncthreads();
    if (tid < CW) {
#pragma unroll
      for (int c = 0; c < NCM; c++) {
        if (c < NC) {
          double t = 0.0;
          for (int wv = 0; wv < WG / 64; wv++) t += sh[(wv * NCM + c) * CW + tid];
          acc[c] = (T)t;
        }
      }
      row_finish<T, CW, NCM>(a, i, tid, NC, acc, ops, dacc);
    }
    __syncthreads();
    if (ep) spmm_store_partials<T, TEAMS, CW, NCM>(a, sh, dacc, tid < CW, 0, tid, blockIdx.x);
    return;
  }
  // ---- short rows: chunks of rows in XCD slabs or contiguously, one team per
  // row.  The dot terms of chunk ch are partial row n_long + ch, summed in the
  // same order whichever workgroup takes the chunk, so the reductions do not
  // depend on the chunk walk.
  const int team = tid / TS, lane = tid % TS;
  const int cl = lane % CW, nz = lane / CW;
  const Slab sl = a.xcd ? xcd_slab((int)blockIdx.x - a.n_long, (int)gridDim.x - a.n_long, a.nchunks)
                        : contiguous_slab((int)blockIdx.x - a.n_long, (int)gridDim.x - a.n_long, a.nchunks);
  for (int64_t ch = sl.first; ch < sl.end; ch += sl.stride) {
    for (int i = a.row0 + (int)ch * a.rows_per_wg + team,
             rend = min<int64_t>(a.row1, a.row0 + (ch + 1) * a.rows_per_wg); i < rend; i += TEAMS) {
      RowOps<T, NCM> ops;
      // one column group: row operands early, overlapping the gather (wider
      // lanes load them after it; loading them early measured no faster)
      if (NCM == 1) row_load<T, CW, NCM>(a, i, cl, NC, ops);
      const RowRange rr = row_range(a, i);
      if (a.long_rows && rr.len > a.long_thr) continue;  // done by its own workgroup
      T acc[NCM];
#pragma unroll
      for (int c = 0; c < NCM; c++) acc[c] = (T)0;
      row_gather<T, CW, NZ, VAL, NCM>(a, rr, nz, cl, NC, acc);
#pragma unroll
      for (int c = 0; c < NCM; c++) {
#pragma unroll
        for (int off = CW; off < TS; off <<= 1) acc[c] += __shfl_xor(acc[c], off, TS);
      }
      if (nz == 0) {
        if (NCM > 1) row_load<T, CW, NCM>(a, i, cl, NC, ops);
        row_finish<T, CW, NCM>(a, i, cl, NC, acc, ops, dacc);
      }
    }
    if (ep) {
      spmm_store_partials<T, TEAMS, CW, NCM>(a, sh, dacc, nz == 0, team, cl, a.n_long + ch);
#pragma unroll
      for (int c = 0; c < NCM; c++) dacc[c] = 0.0;
    }
  }
}

// ------------------------------------------------------- column-lane maps
// Elementwise kernels over an m x B panel: CL column lanes (power of two,
// <= WG), WG / CL row groups, each lane owning columns cl, cl + CL.
struct ColMap {
  int CL, RG, NCL;
};
__device__ inline ColMap colmap(int B) {
  int cl = 1;
  while (cl < B && cl < WG) cl <<= 1;
  ColMap m;
  m.CL = cl;
  m.RG = WG / cl;
  m.NCL = (B + cl - 1) / cl;
  return m;
}

// Reduces per-lane per-column values dacc[0..NCL) over the row groups of the
// workgroup into partials[blockIdx.x * B + j].
__device__ inline void wg_colsum(const ColMap& m, int B, const double* dacc, double* partials) {
  extern __shared__ double sh[];  // WG
  const int tid = threadIdx.x, cl = tid % m.CL, rg = tid / m.CL;
  for (int c = 0; c < m.NCL; c++) {
    __syncthreads();
    sh[tid] = dacc[c];
    __syncthreads();
    for (int off = m.RG / 2; off > 0; off >>= 1) {  // fixed-order tree over row groups
      if (rg < off) sh[tid] += sh[tid + off * m.CL];
      __syncthreads();
    }
    const int j = cl + m.CL * c;
    if (rg == 0 && j < B) partials[(int64_t)blockIdx.x * B + j] = sh[tid];
  }
}

// Per-column sum of squares of an m x B panel -> out[j] (FP64).
template <typename T>
__global__ __launch_bounds__(WG) void k_colnorm2(const T* p, int64_t m, int B, int rows_per_wg,
                                                 double* partials) {
  const ColMap cm = colmap(B);
  const int tid = threadIdx.x, cl = tid % cm.CL, rg = tid / cm.CL;
  double dacc[2] = {0.0, 0.0};
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg, r1 = min<int64_t>(m, r0 + rows_per_wg);
  for (int64_t i = r0 + rg; i < r1; i += cm.RG)
    for (int c = 0; c < cm.NCL; c++) {
      const int j = cl + cm.CL * c;
      if (j < B) {
        double v = (double)p[i * B + j];
        dacc[c] += v * v;
      }
    }
  wg_colsum(cm, B, dacc, partials);
}

// x += alpha p; r -= alpha q (active columns), then <r, r> per column.
// EP_RR: convergence / iteration-cap test.  EP_RR_CG: also the CG direction
// coefficient bcg = rr_new / rz and rz = rr_new (z = r).
template <typename T>
__global__ __launch_bounds__(WG) void k_update_r(int64_t m, int B, int rows_per_wg, T* x, const T* p, T* r,
                                                 const T* q, ColState cs, double* partials) {
  if (*cs.n_active == 0) return;
  const ColMap cm = colmap(B);
  const int tid = threadIdx.x, cl = tid % cm.CL, rg = tid / cm.CL;
  double dacc[2] = {0.0, 0.0};
  T al[2];
  int act[2];
  for (int c = 0; c < cm.NCL; c++) {
    const int j = cl + cm.CL * c;
    act[c] = (j < B) ? cs.active[j] : 0;
    al[c] = act[c] ? (T)cs.alpha[j] : (T)0;
  }
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg, r1 = min<int64_t>(m, r0 + rows_per_wg);
  for (int64_t i = r0 + rg; i < r1; i += cm.RG)
    for (int c = 0; c < cm.NCL; c++) {
      const int j = cl + cm.CL * c;
      if (j < B && act[c]) {
        const int64_t o = i * B + j;
        if (x) x[o] += al[c] * p[o];  // NULL: done with the search-direction update
        T rv = r[o] - al[c] * q[o];
        r[o] = rv;
        dacc[c] += (double)rv * (double)rv;
      }
    }
  wg_colsum(cm, B, dacc, partials);
}

// One row of a row-major BF16 factor with RMAX columns (RMAX * 2 bytes, 16-byte
// aligned) in 16-byte loads, as floats (a BF16 value is the top half of its
// float).
template <int RMAX>
__device__ inline void load_vrow(const bf16* Vr, int64_t i, float (&v)[RMAX]) {
  const uint4* p = reinterpret_cast<const uint4*>(Vr + i * RMAX);
#pragma unroll
  for (int c = 0; c < RMAX / 8; c++) {
    const uint4 u = p[c];
    const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
    for (int h = 0; h < 4; h++) {
      v[8 * c + 2 * h] = __uint_as_float(w[h] << 16);
      v[8 * c + 2 * h + 1] = __uint_as_float(w[h] & 0xFFFF0000u);
    }
  }
}

// Wave sums of R per-lane values (R a power of two, at most 64) by halving
// exchanges: at each step a lane keeps one half of its remaining values (the
// half picked by its lane bit O), adds the partner's copy of that half and
// hands the other half over, so R - 1 exchanges (plus log2(64 / R) for the
// last value) replace the 6 R of one butterfly per value.  On return a[0] of
// lane l holds the wave sum of value l / (64 / R).  The order is fixed, so the
// sums are deterministic.
template <int C, int R>
__device__ inline void wave_sum_spread(double (&a)[R], int lane) {
  if constexpr (C > 1) {
    constexpr int H = C / 2, O = 64 * H / R;
    const bool up = (lane & O) != 0;
#pragma unroll
    for (int h = 0; h < H; h++) {
      const double send = up ? a[h] : a[h + H];
      const double keep = up ? a[h + H] : a[h];
      a[h] = keep + __shfl_xor(send, O, 64);
    }
    wave_sum_spread<H, R>(a, lane);
  } else {
#pragma unroll
    for (int o = 32 / R; o > 0; o >>= 1) a[0] += __shfl_xor(a[0], o, 64);
  }
}

// The halving exchanges of wave_sum_spread over the lane bits O = 32, 16,
// ..., OMIN only: afterwards a[0, R * OMIN / 64) of lane l hold the sums,
// over the lanes that differ from l only in those bits, of the values
// base(l) + c, base(l) = sum over the steps of (bit O of l set ? the size of
// the half kept : 0).
template <int C, int R, int O, int OMIN>
__device__ inline void wave_halve(double (&a)[R], int lane) {
  if constexpr (O >= OMIN && C > 1) {
    constexpr int H = C / 2;
    const bool up = (lane & O) != 0;
#pragma unroll
    for (int h = 0; h < H; h++) {
      const double send = up ? a[h] : a[h + H];
      const double keep = up ? a[h + H] : a[h];
      a[h] = keep + __shfl_xor(send, O, 64);
    }
    wave_halve<H, R, O / 2, OMIN>(a, lane);
  }
}

// One column (B = 1): x += alpha p; r -= alpha q; then, in the same pass,
// the partial sums of V^T r (rank values, registers) and <r, r>; partials
// per workgroup: [W_0 .. W_{rank-1}, rr].  Finalized by EP_RR_VT.
// VR: V is the row-major BF16 copy with rank == RMAX (16-byte row loads).
template <typename T, typename TV, int RMAX, bool VR = false>
__global__ __launch_bounds__(WG) void k_update_r_vt1(int64_t m, int rows_per_wg, T* x, const T* p, T* r,
                                                     const T* q, int rank, const TV* V, ColState cs,
                                                     double* partials) {
  if (*cs.n_active == 0) return;
  __shared__ double sh[(WG / 64) * (RMAX + 1)];
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg, r1 = min<int64_t>(m, r0 + rows_per_wg);
  const T al = (T)cs.alpha[0];
  double acc[RMAX + 1];
#pragma unroll
  for (int k = 0; k <= RMAX; k++) acc[k] = 0.0;
  for (int64_t i = r0 + tid; i < r1; i += WG) {
    // the factor row first (it does not depend on the update), then the update
    double vd[RMAX];
    if constexpr (VR) {
      float vf[RMAX];
      load_vrow<RMAX>((const bf16*)V, i, vf);
#pragma unroll
      for (int k = 0; k < RMAX; k++) vd[k] = (double)vf[k];
    } else {
      TV vv[RMAX];
#pragma unroll
      for (int k = 0; k < RMAX; k++) vv[k] = V[(int64_t)(k < rank ? k : rank - 1) * m + i];
#pragma unroll
      for (int k = 0; k < RMAX; k++) vd[k] = to_d(vv[k]);
    }
    const T pv = p[i], qv = q[i], xv = x[i], r0v = r[i];
    x[i] = xv + al * pv;
    const T rv = r0v - al * qv;
    r[i] = rv;
    const double rd = (double)rv;
    acc[RMAX] += rd * rd;
#pragma unroll
    for (int k = 0; k < RMAX; k++) acc[k] += vd[k] * rd;
  }
  const int wave = tid / 64, lane = tid % 64;
  double rr = acc[RMAX];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) rr += __shfl_xor(rr, off, 64);
  if (lane == 0) sh[wave * (RMAX + 1) + RMAX] = rr;
  double vs[RMAX];
#pragma unroll
  for (int k = 0; k < RMAX; k++) vs[k] = acc[k];
  wave_sum_spread<RMAX, RMAX>(vs, lane);
  if (lane % (64 / RMAX) == 0) sh[wave * (RMAX + 1) + lane / (64 / RMAX)] = vs[0];
  __syncthreads();
  if (tid <= rank) {
    const int k = tid < rank ? tid : RMAX;
    double sum = 0.0;
    for (int wv = 0; wv < WG / 64; wv++) sum += sh[wv * (RMAX + 1) + k];
    partials[(int64_t)blockIdx.x * (rank + 1) + tid] = sum;
  }
}

// p = z + bcg p on the active columns; init: p = z on them (a column whose
// start residual already meets its threshold is inactive and keeps its p).
// x (non-NULL, not at init): also x += alpha p with the old p on the columns
// whose step this iteration set (fresh), active or just converged.
template <typename T>
__global__ __launch_bounds__(WG) void k_update_p(int64_t m, int B, const T* z, T* p, int init, ColState cs,
                                                 T* x = nullptr, const int* fresh = nullptr) {
  if (!init && *cs.n_active == 0 && !x) return;
  const ColMap cm = colmap(B);
  const int tid = threadIdx.x, cl = tid % cm.CL, rg = tid / cm.CL;
  for (int c = 0; c < cm.NCL; c++) {
    const int j = cl + cm.CL * c;
    if (j >= B) continue;
    const bool on = cs.active[j] != 0, xu = x && !init, xf = xu && fresh[j];
    if (!on && !xf) continue;
    // a just-converged column (xf, not on) gets p = z: its p is not read again
    const T b = (init || !on) ? (T)0 : (T)cs.bcg[j];
    const T al = xf ? (T)cs.alpha[j] : (T)0;
    if (xu) {
      for (int64_t i = (int64_t)blockIdx.x * cm.RG + rg; i < m; i += (int64_t)gridDim.x * cm.RG) {
        const int64_t o = i * B + j;
        const T po = p[o];
        x[o] += al * po;
        p[o] = z[o] + b * po;
      }
    } else {
      for (int64_t i = (int64_t)blockIdx.x * cm.RG + rg; i < m; i += (int64_t)gridDim.x * cm.RG) {
        const int64_t o = i * B + j;
        p[o] = init ? z[o] : z[o] + b * p[o];
      }
    }
  }
}

// dst[:, j] (+)= src[:, j] for columns with mask[j] (copy when add == 0).
template <typename T, typename S>
__global__ __launch_bounds__(WG) void k_axpy_mask(int64_t m, int B, T* dst, const S* src, const int* mask,
                                                  const double* scale, int add) {
  const ColMap cm = colmap(B);
  const int tid = threadIdx.x, cl = tid % cm.CL, rg = tid / cm.CL;
  for (int c = 0; c < cm.NCL; c++) {
    const int j = cl + cm.CL * c;
    if (j >= B || (mask && !mask[j])) continue;
    const double sc = scale ? scale[j] : 1.0;
    for (int64_t i = (int64_t)blockIdx.x * cm.RG + rg; i < m; i += (int64_t)gridDim.x * cm.RG) {
      const int64_t o = i * B + j;
      T v = (T)(sc * (double)src[o]);
      dst[o] = add ? (T)(dst[o] + v) : v;
    }
  }
}

// Precision form, after a sweep's FP32 solve of the scaled system: the
// correction d = fl32(fwd_j x_j) on the sweep's columns (mask; every column
// when NULL) and 0 on the others, written back to x for the residual update
// r -= M d, and K = d (add == 0) or K += d on those columns.  d is exactly an
// FP32 value, so M d summed in FP64 is the FP64 residual change of the K
// actually stored, up to the rounding of K + d.
__global__ __launch_bounds__(WG) void k_take_correction(int64_t m, int B, float* x, double* K, const int* mask,
                                                        const double* fwd, int add) {
  const ColMap cm = colmap(B);
  const int tid = threadIdx.x, cl = tid % cm.CL, rg = tid / cm.CL;
  for (int c = 0; c < cm.NCL; c++) {
    const int j = cl + cm.CL * c;
    if (j >= B) continue;
    const bool on = !mask || mask[j];
    const double sc = fwd[j];
    for (int64_t i = (int64_t)blockIdx.x * cm.RG + rg; i < m; i += (int64_t)gridDim.x * cm.RG) {
      const int64_t o = i * B + j;
      const float d = on ? (float)(sc * (double)x[o]) : 0.0f;
      x[o] = d;
      if (on) K[o] = add ? K[o] + (double)d : (double)d;
    }
  }
}

// ------------------------------------------------------ M11 block solves
// out[i] = scale * M_bb^{-1} u[i] for every row i of the tile's blocks, with
// u[i] = cv v[i] + ca (A12 x2)[i] staged in LDS (x2: separator panel indexed
// by column - n1).  The block inverse is symmetric, so thread i reads column
// i of row k (coalesced across the block's rows).
template <typename T>
struct M11Args {
  const int32_t* tile_row0;
  const int32_t* row_blk;
  const int32_t* blk_start;
  const int64_t* blk_off;
  const T* minv;
  const int32_t* rp;
  const int32_t* col;
  const int32_t* split;
  const double* val;
  int n1;
  const T* v;
  T cv;
  const T* x2;
  T ca;
  T* out;
  int B, CB, sub, xcd;
  const int* n_active;
  const int32_t* tile_row1;  // k_m11_cols: tile ends when tiles are not adjacent (NULL: tile_row0[t + 1])
};

template <typename T>
__global__ __launch_bounds__(WG) void k_m11_apply(M11Args<T> a) {
  if (a.n_active && *a.n_active == 0) return;
  extern __shared__ unsigned char smem[];
  T* u = reinterpret_cast<T*>(smem);
  // one tile per workgroup, tiles taken in XCD slabs
  const int tile = a.xcd ? (int)xcd_slab(blockIdx.x, gridDim.x, gridDim.x).first : (int)blockIdx.x;
  const int r0 = a.tile_row0[tile], r1 = a.tile_row0[tile + 1], R = r1 - r0;
  const int B = a.B;
  const int SUB = a.sub, PPP = WG / SUB;  // SUB lanes share one (row, column) gather
  for (int jc = 0; jc < B; jc += a.CB) {
    const int cb = min(a.CB, B - jc);
    const int P = R * cb;
    for (int pb = 0; pb < P; pb += PPP) {
      const int p = pb + (int)threadIdx.x / SUB, sl = (int)threadIdx.x % SUB;
      T s = (T)0;
      int gi = 0, j = 0;
      if (p < P) {
        const int i = p / cb, jj = p - i * cb;
        gi = r0 + i;
        j = jc + jj;
        if (a.x2) {
          // four entries per lane in flight (indices past the row end clamped
          // to its last entry, products masked); same order of the sums
          const int32_t ke = a.rp[gi + 1];
          for (int32_t k = a.split[gi] + sl; k < ke; k += 4 * SUB) {
            int32_t c[4];
#pragma unroll
            for (int q = 0; q < 4; q++) c[q] = a.col[k + q * SUB < ke ? k + q * SUB : ke - 1];
            T xv[4];
#pragma unroll
            for (int q = 0; q < 4; q++) xv[q] = a.x2[(int64_t)(c[q] - a.n1) * B + j];
            __builtin_amdgcn_sched_barrier(0);  // keep the gathers together
#pragma unroll
            for (int q = 0; q < 4; q++) {
              const int32_t kk = k + q * SUB;
              if (kk < ke) s += a.val ? (T)a.val[kk] * xv[q] : xv[q];
            }
          }
        }
      }
      for (int off = 1; off < SUB; off <<= 1) s += __shfl_xor(s, off, SUB);
      if (p < P && sl == 0) {
        s *= a.ca;
        if (a.v) s += a.cv * a.v[(int64_t)gi * B + j];
        u[p] = s;
      }
    }
    __syncthreads();
    for (int p = threadIdx.x; p < P; p += WG) {
      const int i = p / cb, jj = p - i * cb, gi = r0 + i, j = jc + jj;
      const int blk = a.row_blk[gi];
      const int bs = a.blk_start[blk], bsz = a.blk_start[blk + 1] - bs, li = gi - bs;
      const T* mi = a.minv + a.blk_off[blk];
      const T* ub = u + (int64_t)(bs - r0) * cb + jj;
      T s = (T)0;
      for (int k = 0; k < bsz; k++) s += mi[(int64_t)k * bsz + li] * ub[(int64_t)k * cb];
      a.out[(int64_t)gi * B + j] = s;
    }
    __syncthreads();
  }
}

// One column, first sweep: the Schur right-hand side f = b2 + beta A21 t,
// t = M11^{-1} b1, when b = beta A e_q reaches few rows.  The lists (from
// the host, structure only): rows[0, nt) the rows of the blocks that hold a
// neighbour of q (t there, into x1, which is zero elsewhere); rows[nt, nt +
// ns) the separator rows next to q or to those blocks, ascending; for
// separator row s, the block-row entries that reach it, off[s] .. off[s + 1]
// of (pj: the block row, pk: its CSR entry), in block-row order.  f there
// into f2 (zero elsewhere), <f, f> in a fixed order and the column's start
// state as EP_RR_INIT sets it.  One workgroup; every loop is short (hub rows
// never appear whole: only their entries towards the listed blocks do).
template <typename T>
__global__ __launch_bounds__(WG) void k_schur_rhs1(const int32_t* rows, int nt, int ns, const int32_t* off,
                                                   const int32_t* pj, const int32_t* pk, const T* rhs, int32_t n1,
                                                   const int32_t* row_blk, const int32_t* blk_start,
                                                   const int64_t* blk_off, const T* minv, const double* val,
                                                   T beta, T* x1, T* f2, ColState cs) {
  __shared__ double sh[WG / 64];
  const int tid = threadIdx.x;
  for (int t = tid; t < nt; t += WG) {
    const int gi = rows[t];
    const int blk = row_blk[gi], bs = blk_start[blk], bsz = blk_start[blk + 1] - bs, li = gi - bs;
    const T* mi = minv + blk_off[blk];
    T u = (T)0;
    for (int k = 0; k < bsz; k++) u += mi[(int64_t)k * bsz + li] * rhs[bs + k];
    x1[gi] = u;
  }
  __syncthreads();
  double acc = 0.0;
  for (int t = tid; t < ns; t += WG) {
    const int i = rows[nt + t];
    T g = (T)0;
    for (int p = off[t]; p < off[t + 1]; p++) g += (val ? (T)val[pk[p]] : (T)1) * x1[pj[p]];
    const T f = rhs[i] + beta * g;
    f2[i - n1] = f;
    acc += (double)f * (double)f;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (tid % 64 == 0) sh[tid / 64] = acc;
  __syncthreads();
  if (tid == 0) {
    double rr = 0.0;
    for (int wv = 0; wv < WG / 64; wv++) rr += sh[wv];
    cs.rr[0] = rr;
    cs.iters[0] = 0;
    cs.status[0] = 0;
    cs.active[0] = (cs.mask[0] && rr > cs.thr[0]) ? 1 : 0;
  }
  recount_active(cs, 1);
}

// Block solve for B >= 16 columns.  Workgroup (tile, column chunk) with CBW
// lanes per row (64 / CBW rows per wave, coalesced panel rows):
//   phase 1: u[i][:] = ca (A12 x2)[i][:] + cv v[i][:] for the tile's rows
//            into LDS (4 entries of the A12 gather in flight per lane);
//   phase 2: out[i][:] = sum_k Minv_b[li][k] u[bs + k][:] with row li of the
//            block inverse (stored symmetric, so its row is contiguous).
template <typename T, int CBW, bool VAL>
__global__ __launch_bounds__(WG) void k_m11_cols(M11Args<T> a) {
  if (a.n_active && *a.n_active == 0) return;
  extern __shared__ unsigned char smem[];
  T* u = reinterpret_cast<T*>(smem);  // tile rows x CBW
  constexpr int RPG = WG / CBW;       // rows in flight per workgroup
  const int r0 = a.tile_row0[blockIdx.x];
  const int r1 = a.tile_row1 ? a.tile_row1[blockIdx.x] : a.tile_row0[blockIdx.x + 1], R = r1 - r0;
  const int B = a.B;
  const int lane = threadIdx.x % CBW, rs = threadIdx.x / CBW;
  const int j = blockIdx.y * CBW + lane;
  const bool ok = j < B;
  const int jc = ok ? j : B - 1;  // clamped: loads stay in bounds, results unused
  for (int i = rs; i < R; i += RPG) {
    const int gi = r0 + i;
    T s = (T)0;
    if (a.x2) {
      const int32_t kb = a.split[gi], ke = a.rp[gi + 1];
      for (int32_t k = kb; k < ke; k += 4) {
        int32_t c[4];
        T f[4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
          const int32_t kk = k + q < ke ? k + q : ke - 1;
          c[q] = a.col[kk];
          f[q] = k + q < ke ? (VAL ? (T)a.val[kk] : (T)1) : (T)0;
        }
        T xv[4];
#pragma unroll
        for (int q = 0; q < 4; q++) xv[q] = a.x2[(int64_t)(c[q] - a.n1) * B + jc];
#pragma unroll
        for (int q = 0; q < 4; q++) s += (k + q < ke) ? f[q] * xv[q] : (T)0;
      }
    }
    s *= a.ca;
    if (a.v) s += a.cv * a.v[(int64_t)gi * B + jc];
    u[i * CBW + lane] = s;
  }
  __syncthreads();
  for (int i = rs; i < R; i += RPG) {
    const int gi = r0 + i;
    const int blk = a.row_blk[gi];
    const int bs = a.blk_start[blk], bsz = a.blk_start[blk + 1] - bs, li = gi - bs;
    const T* mi = a.minv + a.blk_off[blk] + (int64_t)li * bsz;
    const T* ub = u + (bs - r0) * CBW + lane;
    T s0 = (T)0, s1 = (T)0, s2 = (T)0, s3 = (T)0;
    int k = 0;
    for (; k + 3 < bsz; k += 4) {
      s0 += mi[k] * ub[k * CBW];
      s1 += mi[k + 1] * ub[(k + 1) * CBW];
      s2 += mi[k + 2] * ub[(k + 2) * CBW];
      s3 += mi[k + 3] * ub[(k + 3) * CBW];
    }
    for (; k < bsz; k++) s0 += mi[k] * ub[k * CBW];
    if (ok) a.out[(int64_t)gi * B + j] = (s0 + s1) + (s2 + s3);
  }
}

// Block solve for blocks of at most S rows and B >= 5 columns.  A team of CW
// lanes (8, 16, 32 or 64; WG / CW teams per workgroup) takes consecutive
// blocks (chunks of blocks_per_chunk, in XCD slabs) and all columns, CW * NCM
// of them per team, lane = column within each group.  For
// each block the lane keeps the block's rows of
//   u = ca (A12 x2) + cv v
// in registers (the A12 part is the SpMM row gather over the entries right of
// the split, summed with weight 1 and scaled by ca after), then writes
// out = Minv_b u with row i of the symmetric block inverse read at
// wave-uniform addresses.  No LDS and no per-row index chain: blocks are
// almost all 1-4 rows, so this is an SpMM over the A12 rows with a tiny
// epilogue.  Blocks with more than S rows are skipped here and solved by
// k_m11_cols over tiles of their own.
template <typename T>
struct M11SmallArgs {
  const int32_t* blk_start;
  const int64_t* blk_off;
  const T* minv;
  const int32_t* rp;
  const int32_t* col;
  const int32_t* split;
  const double* val;
  const T* x;  // full n-row panel whose rows >= n1 are x2 (NULL: no A12 term)
  T ca, cb;    // row_gather coefficients: ca unused (no entries left of the split), cb = 1
  T cu;        // scale of the A12 sum
  const T* v;
  T cv;
  T* out;
  int B, nblocks, blocks_per_chunk, xcd;
  int ld, j0;  // panel row stride and first column (row_gather); B and 0 here
  int64_t nchunks;
  const int* n_active;
};

template <typename T, int CW, int NCM, int S, bool VAL>
__global__ __launch_bounds__(WG) void k_m11_small(M11SmallArgs<T> a) {
  if (a.n_active && *a.n_active == 0) return;
  constexpr int TEAMS = WG / CW;
  // a 64-lane team is a wave: its block indices are wave-uniform (scalar loads)
  const int team = CW == 64 ? __builtin_amdgcn_readfirstlane((int)threadIdx.x / 64) : (int)threadIdx.x / CW;
  const int cl = (int)threadIdx.x % CW;
  const int B = a.B, NC = (B + CW - 1) / CW;
  int jc[NCM];
  bool jok[NCM];
#pragma unroll
  for (int cc = 0; cc < NCM; cc++) {
    const int j = cl + CW * cc;
    jok[cc] = cc < NC && j < B;
    jc[cc] = j < B ? j : B - 1;
  }
  const Slab sl = a.xcd ? xcd_slab((int)blockIdx.x, (int)gridDim.x, a.nchunks)
                        : contiguous_slab((int)blockIdx.x, (int)gridDim.x, a.nchunks);
  for (int64_t ch = sl.first; ch < sl.end; ch += sl.stride) {
    const int bend = (int)min<int64_t>(a.nblocks, (ch + 1) * a.blocks_per_chunk);
    for (int b = (int)(ch * a.blocks_per_chunk) + team; b < bend; b += TEAMS) {
      const int bs = CW == 64 ? __builtin_amdgcn_readfirstlane(a.blk_start[b]) : a.blk_start[b];
      const int bsz = (CW == 64 ? __builtin_amdgcn_readfirstlane(a.blk_start[b + 1]) : a.blk_start[b + 1]) - bs;
      if (bsz > S) continue;
      const T* mi = a.minv + a.blk_off[b];
      T u[S][NCM];
#pragma unroll
      for (int k = 0; k < S; k++) {
        if (k < bsz) {
          const int gi = bs + k;
          const int64_t ro = (int64_t)gi * B;
          T vv[NCM], acc[NCM];
#pragma unroll
          for (int cc = 0; cc < NCM; cc++) vv[cc] = acc[cc] = (T)0;
          if (a.v) {  // one uniform branch: the row's loads issued together
#pragma unroll
            for (int cc = 0; cc < NCM; cc++) vv[cc] = a.v[ro + jc[cc]];
          }
          if (a.x) {
            RowRange rr;
            rr.kb = rr.sp = a.split[gi];
            rr.ke = a.rp[gi + 1];
            rr.len = rr.ke - rr.kb;
            row_gather<T, CW, 1, VAL, NCM>(a, rr, 0, cl, NC, acc);
          }
#pragma unroll
          for (int cc = 0; cc < NCM; cc++) u[k][cc] = a.cu * acc[cc] + a.cv * vv[cc];
        } else {
#pragma unroll
          for (int cc = 0; cc < NCM; cc++) u[k][cc] = (T)0;
        }
      }
#pragma unroll
      for (int i = 0; i < S; i++) {
        if (i < bsz) {
          // row i of the inverse: every load issued (index clamped into the
          // row), entries past the block masked to 0
          T m[S];
#pragma unroll
          for (int k = 0; k < S; k++) m[k] = mi[i * bsz + (k < bsz ? k : bsz - 1)];
#pragma unroll
          for (int k = 0; k < S; k++) m[k] = k < bsz ? m[k] : (T)0;
          const int64_t ro = (int64_t)(bs + i) * B;
#pragma unroll
          for (int cc = 0; cc < NCM; cc++) {
            T o = m[0] * u[0][cc];
#pragma unroll
            for (int k = 1; k < S; k++) o += m[k] * u[k][cc];
            if (jok[cc]) a.out[ro + cl + CW * cc] = o;
          }
        }
      }
    }
  }
}

// z = G r with the dense symmetric G = M22^{-1} (L = chol(M22)).
template <typename T>
__global__ __launch_bounds__(WG) void k_dense_apply(int m, int B, const T* g, const T* r, T* z,
                                                    const int* n_active) {
  if (n_active && *n_active == 0) return;
  const int64_t P = (int64_t)m * B;
  for (int64_t p = blockIdx.x * (int64_t)WG + threadIdx.x; p < P; p += (int64_t)gridDim.x * WG) {
    const int i = (int)(p / B), j = (int)(p - (int64_t)i * B);
    T s = (T)0;
    for (int k = 0; k < m; k++) s += g[(int64_t)k * m + i] * r[(int64_t)k * B + j];
    z[p] = s;
  }
}

// --------------------------------------------------- low-rank correction
// V is stored column-major (V[k * m + i]), so lanes over rows read it
// coalesced.  W = V^T r (rank x B) is split over row chunks; the last
// workgroup forms DW = D o W.
//   small rank*B (<= 64): each thread owns rows and keeps all rank*B sums in
//   registers, reduced over the workgroup by wave shuffles and LDS;
//   otherwise lanes over (k, j) pairs loop over the rows.
template <typename T, typename TV>
__global__ __launch_bounds__(WG) void k_vt(int64_t m, int B, int rank, const TV* V, const T* r, int rows_per_wg,
                                           double* partials, const int* n_active) {
  if (n_active && *n_active == 0) return;
  __shared__ double sh[WG];
  const int P = rank * B;
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg, r1 = min<int64_t>(m, r0 + rows_per_wg);
  {
    int G = 1;
    while (G * 2 * P <= WG) G <<= 1;
    for (int pb = 0; pb < P; pb += WG / G) {
      const int pw = min(WG / G, P - pb);
      const int pl = tid % (WG / G), g = tid / (WG / G);
      double acc = 0.0;
      if (pl < pw) {
        const int p = pb + pl, k = p / B, j = p - k * B;
        for (int64_t i = r0 + g; i < r1; i += G) acc += to_d(V[(int64_t)k * m + i]) * (double)r[i * B + j];
      }
      __syncthreads();
      sh[tid] = acc;
      __syncthreads();
      if (g == 0 && pl < pw) {
        double s = 0.0;
        for (int gg = 0; gg < G; gg++) s += sh[gg * (WG / G) + pl];
        partials[(int64_t)blockIdx.x * P + pb + pl] = s;
      }
    }
  }
}

// W = V^T r for one column (B = 1): each thread owns rows and keeps the rank
// sums in registers (compile-time indexed), reduced by wave shuffles and LDS.
// VR: V is the row-major BF16 copy with exactly RMAX columns (rank == RMAX),
// read one 16-byte vector at a time instead of one 2-byte load per column.
template <typename T, typename TV, int RMAX, bool VR = false>
__global__ __launch_bounds__(WG) void k_vt1(int64_t m, int rank, const TV* V, const T* r, int rows_per_wg,
                                            double* partials, const int* n_active) {
  if (n_active && *n_active == 0) return;
  __shared__ double sh[(WG / 64) * RMAX];
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg, r1 = min<int64_t>(m, r0 + rows_per_wg);
  double acc[RMAX];
#pragma unroll
  for (int k = 0; k < RMAX; k++) acc[k] = 0.0;
  for (int64_t i = r0 + tid; i < r1; i += WG) {
    // all factor loads first, unconditionally (columns past the rank repeat
    // the last one and their sums are never used), so they are in flight
    // together instead of one latency each
    double vd[RMAX];
    if constexpr (VR) {
      float vf[RMAX];
      load_vrow<RMAX>((const bf16*)V, i, vf);
#pragma unroll
      for (int k = 0; k < RMAX; k++) vd[k] = (double)vf[k];
    } else {
      TV vv[RMAX];
#pragma unroll
      for (int k = 0; k < RMAX; k++) vv[k] = V[(int64_t)(k < rank ? k : rank - 1) * m + i];
#pragma unroll
      for (int k = 0; k < RMAX; k++) vd[k] = to_d(vv[k]);
    }
    const double rv = (double)r[i];
    __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the FMAs
#pragma unroll
    for (int k = 0; k < RMAX; k++) acc[k] += vd[k] * rv;
  }
  const int wave = tid / 64, lane = tid % 64;
  wave_sum_spread<RMAX, RMAX>(acc, lane);  // sums past the rank are never read
  if (lane % (64 / RMAX) == 0) sh[wave * RMAX + lane / (64 / RMAX)] = acc[0];
  __syncthreads();
  if (tid < rank) {
    double s = 0.0;
    for (int wv = 0; wv < WG / 64; wv++) s += sh[wv * RMAX + tid];
    partials[(int64_t)blockIdx.x * rank + tid] = s;
  }
}

// z = base + V DW with base = r (L = I) or the already stored z (L = chol),
// then <r, z> per column (EP_RZ_INIT: rz = <r,z>; EP_RZ: bcg = <r,z>_new / rz).
template <typename T, typename TV>
__global__ __launch_bounds__(WG) void k_lowrank(int64_t m, int B, int rank, const TV* V, const double* DW,
                                                const T* r, T* z, int z_has_base, int rows_per_wg,
                                                const int* n_active, double* partials) {
  if (n_active && *n_active == 0) return;
  const ColMap cm = colmap(B);
  const int tid = threadIdx.x, cl = tid % cm.CL, rg = tid / cm.CL;
  double dacc[2] = {0.0, 0.0};
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg, r1 = min<int64_t>(m, r0 + rows_per_wg);
  for (int64_t i = r0 + rg; i < r1; i += cm.RG)
    for (int c = 0; c < cm.NCL; c++) {
      const int j = cl + cm.CL * c;
      if (j >= B) continue;
      const int64_t o = i * B + j;
      double s = z_has_base ? (double)z[o] : (double)r[o];
      for (int k = 0; k < rank; k++) s += to_d(V[(int64_t)k * m + i]) * DW[k * B + j];
      T zv = (T)s;
      z[o] = zv;
      dacc[c] += (double)r[o] * (double)zv;
    }
  wg_colsum(cm, B, dacc, partials);
}

// One column (B = 1) of k_lowrank with the rank known at compile time (<=
// RMAX): DW in registers (0 past the rank) and all factor loads of a row
// issued together.  Same sums, same order.
// PUPD: z is not stored; the search direction is updated in place instead,
// z[i] <- z_new + b z[i] (z holds p; b = bcg, 0 at init), when the column is
// active, and no partials are written.
template <typename T, typename TV, int RMAX, bool PUPD = false, bool VR = false>
__global__ __launch_bounds__(WG) void k_lowrank1(int64_t m, int rank, const TV* V, const double* DW, const T* r,
                                                 T* z, int z_has_base, int rows_per_wg, const int* n_active,
                                                 double* partials, const double* bcg = nullptr,
                                                 const int* active = nullptr, int init = 0) {
  if (n_active && *n_active == 0) return;
  if (PUPD && !active[0]) return;
  const double b = PUPD && !init ? bcg[0] : 0.0;
  double dw[RMAX];
#pragma unroll
  for (int k = 0; k < RMAX; k++) dw[k] = k < rank ? DW[k] : 0.0;
  double dacc[1] = {0.0};
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg, r1 = min<int64_t>(m, r0 + rows_per_wg);
  for (int64_t i = r0 + threadIdx.x; i < r1; i += WG) {
    double vd[RMAX];
    if constexpr (VR) {
      float vf[RMAX];
      load_vrow<RMAX>((const bf16*)V, i, vf);
#pragma unroll
      for (int k = 0; k < RMAX; k++) vd[k] = (double)vf[k];
    } else {
      TV vv[RMAX];
#pragma unroll
      for (int k = 0; k < RMAX; k++) vv[k] = V[(int64_t)(k < rank ? k : rank - 1) * m + i];
#pragma unroll
      for (int k = 0; k < RMAX; k++) vd[k] = to_d(vv[k]);
    }
    const double rv = (double)r[i];
    const double pv = PUPD && !init ? (double)z[i] : 0.0;
    double s = !PUPD && z_has_base ? (double)z[i] : rv;
#pragma unroll
    for (int k = 0; k < RMAX; k++) s += vd[k] * dw[k];
    if (PUPD) {
      z[i] = (T)(s + b * pv);
    } else {
      const T zv = (T)s;
      z[i] = zv;
      dacc[0] += rv * (double)zv;
    }
  }
  if (!PUPD) wg_colsum(colmap(1), 1, dacc, partials);
}

// ------------------------------------- low-rank products for B >= 2 columns
// Both kernels give thread t of a workgroup one panel column,
// j = blockIdx.y * JW + t % JW (JW: a power of two <= 256 covering B, or 256),
// and WG / JW row groups; blockIdx.x is a chunk of rpc rows.  In the staged
// form (16 columns and more) the rows of V (column-major n2 x rank) of a
// 64-row block are staged in LDS as a row-major tile (stride RMAX + 2
// doubles: rows of different row groups fall in different banks), so each
// panel element is read once and each V value once per workgroup.  Ranks
// above `rank` (up to RMAX) are staged as 0.  Narrower batches take the
// unstaged form (DIRECT below).
constexpr int kVRows = 64;

template <typename TV, int RMAX>
__device__ inline void stage_v(double* sV, const TV* V, int64_t m, int rank, int64_t b0, int nb) {
  constexpr int LD = RMAX + 2;
  for (int e = threadIdx.x; e < kVRows * RMAX; e += WG) {
    const int k = e / kVRows, ii = e % kVRows;  // consecutive threads: consecutive rows of one column
    sV[ii * LD + k] = (k < rank && ii < nb) ? to_d(V[(int64_t)k * m + b0 + ii]) : 0.0;
  }
}

// W partials: partials[blockIdx.x * rank * B + k * B + j] = sum over the
// chunk's rows i of V[i][k] r[i][j] (FP64 sums).
// DIRECT (narrow batches, JW <= 8): no LDS tile; each thread issues all the
// factor loads of its row at once (columns past the rank repeat the last
// one, their sums unused), so many loads are in flight per wave instead of
// one block's staging per barrier pair.  A thread visits rows r0 + rg,
// r0 + rg + NR, ... as the staged form does when NR divides the block height.
// VR (DIRECT only): V is the row-major BF16 copy with rank == RMAX.
template <typename T, typename TV, int RMAX, bool DIRECT = false, bool VR = false>
__global__ __launch_bounds__(WG) void k_vt_rows(int64_t m, int B, int rank, int JW, const TV* V, const T* r,
                                                int64_t rpc, double* partials, const int* n_active) {
  if (n_active && *n_active == 0) return;
  constexpr int LD = RMAX + 2;
  __shared__ double sV[kVRows * LD];
  const int tid = threadIdx.x, jl = tid % JW, rg = tid / JW, NR = WG / JW;
  const int j = blockIdx.y * JW + jl;
  const bool col_ok = j < B;
  const int64_t r0 = (int64_t)blockIdx.x * rpc, r1 = min<int64_t>(m, r0 + rpc);
  double acc[RMAX];
#pragma unroll
  for (int k = 0; k < RMAX; k++) acc[k] = 0.0;
  if (DIRECT) {
    if (col_ok) {
      for (int64_t i = r0 + rg; i < r1; i += NR) {
        double vd[RMAX];
        if constexpr (VR) {
          float vf[RMAX];
          load_vrow<RMAX>((const bf16*)V, i, vf);
#pragma unroll
          for (int k = 0; k < RMAX; k++) vd[k] = (double)vf[k];
        } else {
          TV vv[RMAX];
#pragma unroll
          for (int k = 0; k < RMAX; k++) vv[k] = V[(int64_t)(k < rank ? k : rank - 1) * m + i];
#pragma unroll
          for (int k = 0; k < RMAX; k++) vd[k] = to_d(vv[k]);
        }
        const double x = (double)r[i * B + j];
        __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the FMAs
#pragma unroll
        for (int k = 0; k < RMAX; k++) acc[k] += vd[k] * x;
      }
    }
  } else {
    for (int64_t b0 = r0; b0 < r1; b0 += kVRows) {
      const int nb = (int)min<int64_t>(kVRows, r1 - b0);
      __syncthreads();
      stage_v<TV, RMAX>(sV, V, m, rank, b0, nb);
      __syncthreads();
      if (col_ok) {
        for (int ii = rg; ii < nb; ii += NR) {
          const double x = (double)r[(b0 + ii) * B + j];
          const double* vr = sV + ii * LD;
#pragma unroll
          for (int k = 0; k < RMAX; k++) acc[k] += vr[k] * x;
        }
      }
    }
  }
  const int64_t nv = (int64_t)rank * B;
  double* out = partials + (int64_t)blockIdx.x * nv;
  if (JW <= 8) {
    // the lanes of one column in a wave differ in bits 3-5 and in the bits
    // [log2 JW, 3): halving exchanges over bits 5, 4, 3, butterflies over
    // the others; then the wave sums in order through LDS
    const int lane = tid % 64, wave = tid / 64;
    wave_halve<RMAX, RMAX, 32, 8>(acc, lane);
    constexpr int C8 = RMAX / 8;
    for (int off = 4; off >= JW; off >>= 1) {
#pragma unroll
      for (int c = 0; c < C8; c++) acc[c] += __shfl_xor(acc[c], off, 64);
    }
    __syncthreads();  // sV is free (the staged path's last reads are done)
    if ((lane & 7) < JW) {
      const int base = ((lane >> 5) & 1) * (RMAX / 2) + ((lane >> 4) & 1) * (RMAX / 4) + ((lane >> 3) & 1) * C8;
#pragma unroll
      for (int c = 0; c < C8; c++) sV[(wave * RMAX + base + c) * JW + jl] = acc[c];
    }
    __syncthreads();
    for (int t = tid; t < rank * JW; t += WG) {
      const int k = t / JW, jj = t % JW, j2 = blockIdx.y * JW + jj;
      if (j2 < B) {
        double sum = 0.0;
        for (int wv = 0; wv < WG / 64; wv++) sum += sV[(wv * RMAX + k) * JW + jj];
        out[(int64_t)k * B + j2] = sum;
      }
    }
    return;
  }
  if (NR == 1) {
#pragma unroll
    for (int k = 0; k < RMAX; k++)
      if (k < rank && col_ok) out[(int64_t)k * B + j] = acc[k];
    return;
  }
  // sum over the row groups in a fixed tree order
#pragma unroll
  for (int k = 0; k < RMAX; k++) {
    if (k < rank) {
      __syncthreads();
      sV[tid] = acc[k];
      __syncthreads();
      for (int off = NR / 2; off > 0; off >>= 1) {
        if (rg < off) sV[tid] += sV[tid + off * JW];
        __syncthreads();
      }
      if (rg == 0 && col_ok) out[(int64_t)k * B + j] = sV[tid];
    }
  }
}

// DW[v] = D[v / B] * sum over chunks c of partials[c * nv + v], nv = rank * B
// (D NULL: the plain sums): 64 values per workgroup, its four waves taking
// every fourth chunk, combined in a fixed order (deterministic).
__global__ __launch_bounds__(WG) void k_vt_reduce(const double* partials, int nchunk, int64_t nv, int B,
                                                  const double* Dg, double* DW, const int* n_active,
                                                  double* DW2 = nullptr) {
  if (n_active && *n_active == 0) return;
  __shared__ double sh[WG];
  const int tid = threadIdx.x, lane = tid % 64, wv = tid / 64;
  const int64_t v = (int64_t)blockIdx.x * 64 + lane;
  double s0 = 0.0, s1 = 0.0;
  if (v < nv) {
    int c = wv;
    for (; c + 4 < nchunk; c += 8) {
      s0 += partials[(int64_t)c * nv + v];
      s1 += partials[(int64_t)(c + 4) * nv + v];
    }
    for (; c < nchunk; c += 4) s0 += partials[(int64_t)c * nv + v];
  }
  sh[tid] = s0 + s1;
  __syncthreads();
  if (wv == 0 && v < nv) {
    const double sw = (sh[lane] + sh[64 + lane]) + (sh[128 + lane] + sh[192 + lane]);
    const double d = Dg ? Dg[v / B] : 1.0;
    DW[v] = d * sw;
    if (DW2) DW2[v] = d * sw * sw;  // this (k, j)'s term of <r, z>
  }
}

// z = base + V DW (base = r, or the z already stored when L = chol), then
// the per-column <r, z> partials[blockIdx.x * B + j] over the chunk's rows.
// PUPD: as in k_lowrank1, z holds the search direction p, updated in place
// (p <- z_new + bcg p, p <- z_new at init) for the active columns, no partials.
// DIRECT: as in k_vt_rows (factor loads of a row issued together, no LDS
// tile); the same value per element (DW is 0 past the rank).
// PUPD with XUP (never at init): also xk += alpha p with the old p on the
// columns whose step this iteration set (fresh), active or just converged.
template <typename T, typename TV, int RMAX, bool PUPD = false, bool DIRECT = false, bool VR = false,
          bool XUP = false>
__global__ __launch_bounds__(WG) void k_lowrank_rows(int64_t m, int B, int rank, int JW, const TV* V,
                                                     const double* DW, const T* __restrict__ r, T* __restrict__ z,
                                                     int z_has_base, int64_t rpc, const int* n_active,
                                                     double* partials, const double* bcg = nullptr,
                                                     const int* active = nullptr, int init = 0,
                                                     T* __restrict__ xk = nullptr, const double* alpha = nullptr,
                                                     const int* fresh = nullptr) {
  if (!XUP && n_active && *n_active == 0) return;
  constexpr int LD = RMAX + 2;
  __shared__ double sV[kVRows * LD];
  const int tid = threadIdx.x, jl = tid % JW, rg = tid / JW, NR = WG / JW;
  const int j = blockIdx.y * JW + jl;
  const bool col_ok = j < B && (!PUPD || active[j]);
  constexpr bool xu = PUPD && XUP;  // XUP: never at init
  const bool xf = xu && j < B && fresh[j];
  const T xal = xf ? (T)alpha[j] : (T)0;
  const double b = PUPD && !init && col_ok ? bcg[j] : 0.0;
  const int64_t r0 = (int64_t)blockIdx.x * rpc, r1 = min<int64_t>(m, r0 + rpc);
  double dw[RMAX];
#pragma unroll
  for (int k = 0; k < RMAX; k++) dw[k] = (col_ok && k < rank) ? DW[(int64_t)k * B + j] : 0.0;
  double dacc = 0.0;
  if (DIRECT) {
    if (col_ok || xf) {
      for (int64_t i = r0 + rg; i < r1; i += NR) {
        double vd[RMAX];
        if constexpr (VR) {
          float vf[RMAX];
          load_vrow<RMAX>((const bf16*)V, i, vf);
#pragma unroll
          for (int k = 0; k < RMAX; k++) vd[k] = (double)vf[k];
        } else {
          TV vv[RMAX];
#pragma unroll
          for (int k = 0; k < RMAX; k++) vv[k] = V[(int64_t)(k < rank ? k : rank - 1) * m + i];
#pragma unroll
          for (int k = 0; k < RMAX; k++) vd[k] = to_d(vv[k]);
        }
        const int64_t o = i * B + j;
        const double rv = (double)r[o];
        const T po = PUPD && !init ? z[o] : (T)0;
        const double pv = (double)po;
        double sum = !PUPD && z_has_base ? (double)z[o] : rv;
        __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the FMAs
#pragma unroll
        for (int k = 0; k < RMAX; k++) sum += vd[k] * dw[k];
        if (PUPD) {
          // a just-converged column (xf, not col_ok) gets z = r: its p is
          // not read again
          if constexpr (xu) xk[o] += xal * po;
          z[o] = (T)(sum + b * pv);
        } else {
          const T zv = (T)sum;
          z[o] = zv;
          dacc += rv * (double)zv;
        }
      }
    }
  } else {
    for (int64_t b0 = r0; b0 < r1; b0 += kVRows) {
      const int nb = (int)min<int64_t>(kVRows, r1 - b0);
      __syncthreads();
      stage_v<TV, RMAX>(sV, V, m, rank, b0, nb);
      __syncthreads();
      if (col_ok || xf) {
        for (int ii = rg; ii < nb; ii += NR) {
          const int64_t o = (b0 + ii) * B + j;
          const double rv = (double)r[o];
          const T po = PUPD && !init ? z[o] : (T)0;
          const double pv = (double)po;
          double sum = !PUPD && z_has_base ? (double)z[o] : rv;
          const double* vr = sV + ii * LD;
#pragma unroll
          for (int k = 0; k < RMAX; k++) sum += vr[k] * dw[k];
          if (PUPD) {
            if constexpr (xu) xk[o] += xal * po;
            z[o] = (T)(sum + b * pv);
          } else {
            const T zv = (T)sum;
            z[o] = zv;
            dacc += rv * (double)zv;
          }
        }
      }
    }
  }
  if (PUPD) return;
  __syncthreads();
  sV[tid] = dacc;
  __syncthreads();
  for (int off = NR / 2; off > 0; off >>= 1) {
    if (rg < off) sV[tid] += sV[tid + off * JW];
    __syncthreads();
  }
  if (rg == 0 && col_ok) partials[(int64_t)blockIdx.x * B + j] = sV[tid];
}

// ------------------------------------------- low-rank GEMMs on MFMA (bf16)
// FP32 panels, BF16 V: v_mfma_f32_16x16x32_bf16 with FP32 accumulation.  The
// FP32 panel operand is split into bf16 hi + lo parts (two MFMAs), so the
// product keeps ~16 mantissa bits; V itself is stored in BF16.
// Operand lanes (16x16x32): a[t] = A[l % 16][8 (l / 16) + t],
// b[t] = B[8 (l / 16) + t][l % 16]; result d[t] = D[4 (l / 16) + t][l % 16].
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ inline void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

// W partials: workgroup (jt, kt, s) computes the 32 (k) x 64 (j) tile of
// V^T r over row chunk s; wave w owns columns j0 + 16 w and both k halves.
// V16: column-major n2 x rank (bf16); r: m x B FP32.
__global__ __launch_bounds__(WG) void k_vt_mfma(int64_t m, int B, int rank, const bf16* V16, const float* r,
                                                int64_t rows_per_chunk, double* partials, const int* n_active) {
  if (n_active && *n_active == 0) return;
  const int wave = threadIdx.x / 64, l = threadIdx.x % 64;
  const int j0 = blockIdx.x * 64 + wave * 16;
  const int k0 = blockIdx.y * 32;
  const int64_t i_beg = (int64_t)blockIdx.z * rows_per_chunk;
  const int64_t i_end = min<int64_t>(m, i_beg + rows_per_chunk);
  const int jn = j0 + (l % 16);
  const bool jok = jn < B;
  const __bf16* Vb = reinterpret_cast<const __bf16*>(V16);
  floatx4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
  for (int64_t i0 = i_beg; i0 < i_end; i0 += 32) {
    bf16x8 bh, bl, a0, a1;
#pragma unroll
    for (int t = 0; t < 8; t++) {
      const int64_t i = i0 + 8 * (l / 16) + t;
      const bool iok = i < i_end;
      const float x = (iok && jok) ? r[i * B + jn] : 0.0f;
      __bf16 h, lo;
      split_bf16(x, h, lo);
      bh[t] = h;
      bl[t] = lo;
      const int ka = k0 + (l % 16), kb = k0 + 16 + (l % 16);
      a0[t] = (iok && ka < rank) ? Vb[(int64_t)ka * m + i] : (__bf16)0.0f;
      a1[t] = (iok && kb < rank) ? Vb[(int64_t)kb * m + i] : (__bf16)0.0f;
    }
    acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, bh, acc0, 0, 0, 0);
    acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, bl, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bh, acc1, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bl, acc1, 0, 0, 0);
  }
  // d[t] = W[k0 + 4 (l / 16) + t][jn] (acc0), W[k0 + 16 + 4 (l / 16) + t][jn] (acc1)
  const int64_t P = (int64_t)rank * B;
  double* out = partials + (int64_t)blockIdx.z * P;
  if (jok) {
#pragma unroll
    for (int t = 0; t < 4; t++) {
      const int ka = k0 + 4 * (l / 16) + t, kb = k0 + 16 + 4 * (l / 16) + t;
      if (ka < rank) out[(int64_t)ka * B + jn] = (double)acc0[t];
      if (kb < rank) out[(int64_t)kb * B + jn] = (double)acc1[t];
    }
  }
}

// z = base + V DW for 64-row x 64-column tiles (grid-stride over row tiles),
// base = r or the stored z; plus per-column partial dots <r, z>.
// V16r: row-major n2 x rank (bf16); DW: rank x B (FP64, split to bf16 hi/lo in LDS).
__global__ __launch_bounds__(WG) void k_lowrank_mfma(int64_t m, int B, int rank, const bf16* V16r, const double* DW,
                                                     const float* r, float* z, int z_has_base, double* partials,
                                                     const int* n_active) {
  if (n_active && *n_active == 0) return;
  extern __shared__ unsigned char smem_lr[];
  const int KP = (rank + 31) / 32 * 32;             // rank padded to the MFMA depth
  __bf16* dh = reinterpret_cast<__bf16*>(smem_lr);  // [KP][64]
  __bf16* dl = dh + KP * 64;
  double* red = reinterpret_cast<double*>(dl + KP * 64);  // [4 waves][64]
  const int wave = threadIdx.x / 64, l = threadIdx.x % 64;
  const int jb = blockIdx.y * 64;
  for (int e = threadIdx.x; e < KP * 64; e += WG) {
    const int k = e / 64, jj = e % 64;
    const float v = (k < rank && jb + jj < B) ? (float)DW[(int64_t)k * B + jb + jj] : 0.0f;
    __bf16 h, lo;
    split_bf16(v, h, lo);
    dh[e] = h;
    dl[e] = lo;
  }
  __syncthreads();
  const __bf16* Vb = reinterpret_cast<const __bf16*>(V16r);
  double dacc[4] = {0.0, 0.0, 0.0, 0.0};  // column jb + 16 c + l % 16
  const int64_t ntile = (m + 63) / 64;
  for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    const int64_t i0 = tile * 64 + wave * 16;  // this wave's 16 rows
    floatx4 acc[4];
#pragma unroll
    for (int c = 0; c < 4; c++) acc[c] = (floatx4){0, 0, 0, 0};
    for (int k0 = 0; k0 < KP; k0 += 32) {
      bf16x8 a;
      const int64_t ia = i0 + (l % 16);
#pragma unroll
      for (int t = 0; t < 8; t++) {
        const int k = k0 + 8 * (l / 16) + t;
        a[t] = (ia < m && k < rank) ? Vb[ia * rank + k] : (__bf16)0.0f;
      }
#pragma unroll
      for (int c = 0; c < 4; c++) {
        bf16x8 bh, bl;
#pragma unroll
        for (int t = 0; t < 8; t++) {
          const int e = (k0 + 8 * (l / 16) + t) * 64 + 16 * c + (l % 16);
          bh[t] = dh[e];
          bl[t] = dl[e];
        }
        acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bh, acc[c], 0, 0, 0);
        acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bl, acc[c], 0, 0, 0);
      }
    }
#pragma unroll
    for (int c = 0; c < 4; c++) {
      const int j = jb + 16 * c + (l % 16);
      if (j >= B) continue;
#pragma unroll
      for (int t = 0; t < 4; t++) {
        const int64_t i = i0 + 4 * (l / 16) + t;
        if (i >= m) continue;
        const int64_t o = i * B + j;
        const float base = z_has_base ? z[o] : r[o];
        const float zv = base + acc[c][t];
        z[o] = zv;
        dacc[c] += (double)r[o] * (double)zv;
      }
    }
  }
  // per-column sums: the 4 lanes l, l^16, l^32, l^48 share a column in a wave
#pragma unroll
  for (int c = 0; c < 4; c++) {
    double v = dacc[c];
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    if (l < 16) red[wave * 64 + 16 * c + l] = v;
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    const int j = jb + threadIdx.x;
    if (j < B) {
      double sum = 0.0;
      for (int wv = 0; wv < WG / 64; wv++) sum += red[wv * 64 + threadIdx.x];
      partials[(int64_t)blockIdx.x * B + j] = sum;
    }
  }
}

// One workgroup: reduces the producer's per-workgroup partials (fixed order)
// and applies the step's per-column logic.
//   EP_PQ: pq, alpha = rz / pq, breakdown test     EP_RES / EP_NORM: out = sum
//   EP_RR_INIT: rr, solve start                    EP_RR: rr, convergence / cap
//   EP_RR_CG: as EP_RR plus bcg = rr_new / rz      EP_VT: DW = D o W
//   EP_RZ_INIT: rz                                  EP_RZ: bcg = rz_new / rz
// First stage of a reduction over many partial rows: segment y of `seg`
// consecutive rows of partials[rows x nv] (the last one shorter), summed per
// value in row order by four row lanes combined in a fixed order, into
// out[y * nv + v].  Grid: (ceil(nv / 64), number of segments).
__global__ __launch_bounds__(WG) void k_seg_reduce(const double* partials, int64_t rows, int64_t nv, int64_t seg,
                                                   double* out, const int* n_active) {
  if (n_active && *n_active == 0) return;
  __shared__ double sh[WG];
  const int tid = threadIdx.x, lane = tid % 64, q = tid / 64;
  const int64_t v = (int64_t)blockIdx.x * 64 + lane;
  const int64_t r0 = (int64_t)blockIdx.y * seg, r1 = min<int64_t>(rows, r0 + seg);
  double s0 = 0.0, s1 = 0.0;
  if (v < nv) {
    int64_t r = r0 + q;
    for (; r + 4 < r1; r += 8) {
      s0 += partials[r * nv + v];
      s1 += partials[(r + 4) * nv + v];
    }
    for (; r < r1; r += 4) s0 += partials[r * nv + v];
  }
  sh[tid] = s0 + s1;
  __syncthreads();
  if (q == 0 && v < nv) out[(int64_t)blockIdx.y * nv + v] = (sh[lane] + sh[64 + lane]) + (sh[128 + lane] + sh[192 + lane]);
}

// One workgroup of kFinWG threads: the partials are read kFinWG wide (fewer
// dependent rounds than a 256-thread workgroup).
constexpr int kFinWG = 1024;
// <r, z> = <r, r> + sum_k DW2[k][j] (the terms D_k W_kj^2 of z = r + V (D o W),
// summed in a fixed order) and the PCG step: init sets rz for the masked
// columns, an iteration sets bcg = rz_new / rz_old for the active ones.
__device__ inline void rz_from_terms(int rank, int B, const double* DW2, int init, const ColState& cs) {
  for (int j = threadIdx.x; j < B; j += blockDim.x) {
    if (init ? !cs.mask[j] : !cs.active[j]) continue;
    double s = cs.rr[j];
    for (int k = 0; k < rank; k++) s += DW2[(int64_t)k * B + j];
    if (!init) cs.bcg[j] = s / cs.rz[j];
    cs.rz[j] = s;
  }
}

__global__ __launch_bounds__(kFinWG) void k_finalize(const double* partials, int nwg, int nv, int ep, ColState cs,
                                                     int B, double* out, const double* D, const int* n_active,
                                                     double* out2, int rz_mode, int* fresh) {
  if (n_active && *n_active == 0) return;
  final_reduce<kFinWG>(partials, nwg, nv, [&](int j, double s) {
    switch (ep) {
      case EP_RES:
      case EP_NORM:
        out[j] = s;
        break;
      case EP_VT:
        out[j] = D[j / B] * s;
        if (out2) out2[j] = D[j / B] * s * s;
        break;
      case EP_PQ:
        if (cs.active[j]) {
          cs.pq[j] = s;
          if (!finite_pos(s)) {
            cs.status[j] = 1;
            cs.active[j] = 0;
          } else {
            cs.alpha[j] = cs.rz[j] / s;
            if (fresh) fresh[j] = 1;
          }
        }
        break;
      case EP_RR_INIT:
        cs.rr[j] = s;
        cs.iters[j] = 0;
        cs.status[j] = 0;
        cs.active[j] = (cs.mask[j] && s > cs.thr[j]) ? 1 : 0;
        break;
      case EP_RR_VT:
        if (j < nv - 1) {
          out[j] = D[j] * s;  // DW (one column)
          if (out2) out2[j] = D[j] * s * s;
          break;
        }
        j = 0;  // the last value is <r, r> of column 0
        // fall through
      case EP_RR:
      case EP_RR_CG: {
        if (!cs.active[j]) break;
        cs.rr[j] = s;
        const int it = ++cs.iters[j];
        if (ep == EP_RR_CG) {
          cs.bcg[j] = s / cs.rz[j];
          cs.rz[j] = s;
        }
        if (!(s == s)) {
          cs.status[j] = 1;
          cs.active[j] = 0;
        } else if (s <= cs.thr[j]) {
          cs.active[j] = 0;
        } else if (it >= cs.max_iter) {
          cs.status[j] = 2;
          cs.active[j] = 0;
        }
        break;
      }
      case EP_RZ_INIT:
        if (cs.mask[j]) cs.rz[j] = s;
        break;
      case EP_RZ:
        if (cs.active[j]) {
          cs.bcg[j] = s / cs.rz[j];
          cs.rz[j] = s;
        }
        break;
      default:
        break;
    }
  });
  if (ep == EP_PQ || ep == EP_RR_INIT || ep == EP_RR || ep == EP_RR_CG || ep == EP_RR_VT) recount_active(cs, B);
  if (ep == EP_VT && rz_mode) {
    // the <r, z> terms just written by this workgroup (out2), then the PCG
    // step: 1 = iteration, 2 = initial step
    __syncthreads();
    rz_from_terms(nv / B, B, out2, rz_mode == 2, cs);
  }
  if (ep == EP_RR_VT && rz_mode) {
    // one column: the same from <r, r> (just stored) and the rank terms
    __syncthreads();
    rz_from_terms(nv - 1, 1, out2, 0, cs);
  }
}

// <r, z> of the preconditioned residual z = r + V (D o W), W = V^T r, without
// forming z: <r, r> + sum_k D_k W_k^2 (exact for the stored V; DW2 holds the
// terms D_k W_kj^2, rank x B), summed in a fixed order; then the PCG step
// logic of EP_RZ_INIT / EP_RZ (rz, and bcg = rz_new / rz_old).
__global__ void k_rz_lowrank(int rank, int B, const double* DW2, int init, ColState cs, const int* n_active) {
  if (!init && n_active && *n_active == 0) return;
  rz_from_terms(rank, B, DW2, init, cs);
}

// Start of a batch: stop thresholds on the recurrence residual and the first
// sweep's column mask (columns with b = 0 are done: k = 0).
__global__ void k_cols_setup(int B, const double* bn2, double scale, double* thr, int* mask) {
  for (int j = threadIdx.x; j < B; j += blockDim.x) {
    thr[j] = scale * bn2[j];
    mask[j] = bn2[j] > 0.0 ? 1 : 0;
  }
}

// Precision form, per sweep: the FP64 right-hand side is scaled to unit norm
// per column for the FP32 inner solve (inv), the correction is scaled back
// (fwd), and the inner stop threshold is the larger of the FP32 floor and half
// the outer tolerance relative to this right-hand side.
__global__ void k_mixed_scales(int B, const double* rn2, const double* bn2, double tol, double eps,
                               double* inv, double* fwd, double* thr) {
  for (int j = threadIdx.x; j < B; j += blockDim.x) {
    const double rn = sqrt(rn2[j]);
    inv[j] = rn > 0.0 ? 1.0 / rn : 0.0;
    fwd[j] = rn;
    const double t = rn > 0.0 ? fmax(eps, 0.5 * tol * sqrt(bn2[j]) / rn) : 1.0;
    thr[j] = t * t;
  }
}

// Plain-CG start: rz = rr, active = mask && rr > thr.
__global__ void k_cg_init(int B, ColState cs) {
  for (int j = threadIdx.x; j < B; j += blockDim.x) {
    cs.rz[j] = cs.rr[j];
    cs.iters[j] = 0;
    cs.status[j] = 0;
    cs.active[j] = (cs.mask[j] && cs.rr[j] > cs.thr[j]) ? 1 : 0;
  }
  recount_active(cs, B);
}

// scores[j * n + v] = K[perm[v] * B + j]
// out[t] = K[row[t]][col[t]] of the permuted n x B panel (pair queries).
__global__ void k_pair_gather(int np, int B, const double* K, const int32_t* row, const int32_t* col,
                              double* out) {
  const int t = blockIdx.x * WG + threadIdx.x;
  if (t < np) out[t] = K[(int64_t)row[t] * B + col[t]];
}

template <typename T>
__global__ void k_unpermute(int n, int B, const T* K, const int32_t* perm, double* out) {
  const int j = blockIdx.y;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
    out[(int64_t)j * n + v] = (double)K[(int64_t)perm[v] * B + j];
}

// The same for wide batches, as a tiled transpose: a workgroup moves 64
// nodes x 64 columns, reading 64 contiguous values of each node's (permuted)
// row and writing 64 consecutive nodes of each column, through LDS (rows
// padded by one element against bank conflicts).
template <typename T>
__global__ __launch_bounds__(WG) void k_unpermute_tiled(int n, int B, const T* K, const int32_t* perm,
                                                        double* out) {
  constexpr int TV = 64, TJ = 64, RS = WG / 64;
  __shared__ double tile[TV][TJ + 1];
  const int v0 = blockIdx.x * TV, j0 = blockIdx.y * TJ;
  const int tx = (int)threadIdx.x % 64, ty = (int)threadIdx.x / 64;
  for (int r = ty; r < TV; r += RS) {
    const int v = v0 + r, j = j0 + tx;
    if (v < n && j < B) tile[r][tx] = (double)K[(int64_t)perm[v] * B + j];
  }
  __syncthreads();
  for (int c = ty; c < TJ; c += RS) {
    const int j = j0 + c, v = v0 + tx;
    if (v < n && j < B) out[(int64_t)j * n + v] = tile[tx][c];
  }
}


// ============================================================== profiling
// Optional per-kernel timing: HIP events around each launch of the hot
// kernels on the solve stream, harvested at the solver's host sync points,
// plus the algorithmic bytes each launch moves (formulas next to the launches).
enum ProfKind { PK_SPMM_SEP = 0, PK_SPMM_FULL, PK_M11, PK_VT, PK_LOWRANK, PK_UPDATE_R, PK_UPDATE_P, PK_TOPK,
                PK_OTHER, PK_SPMM_RHS, PK_M11_BIG, PK_COUNT };
static const char* kProfNames[PK_COUNT] = {"spmm_separator_rows", "spmm_all_rows", "m11_block_apply",
                                           "lowrank_vt", "lowrank_apply", "update_r", "update_p", "topk_select",
                                           "other", "spmm_schur_rhs", "m11_big_blocks"};
struct ProfTable {
  std::mutex mu;
  int64_t launches[PK_COUNT] = {};
  double ms[PK_COUNT] = {};
  double bytes[PK_COUNT] = {};
};
static ProfTable g_prof;
static std::atomic<int> g_prof_on{0};

struct ProfEvents {
  std::vector<hipEvent_t> ev;  // pairs
  std::vector<int> kind;
  std::vector<double> bytes;
  size_t used = 0;
  void begin(int k, double b, hipStream_t st) {
    if (used == kind.size()) {
      std::lock_guard<std::recursive_mutex> g(hip_global_mu());
      hipEvent_t a, c;
      HIPCHECK(hipEventCreate(&a));
      HIPCHECK(hipEventCreate(&c));
      ev.push_back(a);
      ev.push_back(c);
      kind.push_back(0);
      bytes.push_back(0);
    }
    kind[used] = k;
    bytes[used] = b;
    HIPCHECK(hipEventRecord(ev[2 * used], st));
  }
  void end(hipStream_t st) {
    HIPCHECK(hipEventRecord(ev[2 * used + 1], st));
    used++;
  }
  // call after the stream was synchronized
  void harvest() {
    if (!used) return;
    std::lock_guard<std::mutex> g(g_prof.mu);
    for (size_t i = 0; i < used; i++) {
      float ms = 0;
      if (hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]) == hipSuccess) {
        g_prof.launches[kind[i]]++;
        g_prof.ms[kind[i]] += ms;
        g_prof.bytes[kind[i]] += bytes[i];
      }
    }
    used = 0;
  }
  ~ProfEvents() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
};

// ================================================================== tuning
// Launch shapes (overridable from the environment for tuning sweeps).  Every
// partials buffer is sized from these limits.
struct Tuning {
  int ts1;          // lanes per row of the one-column SpMM (4, 8, 16, 32)
  int spmm_nwg;     // max short-row workgroups of the SpMM
  int rows_team;    // target rows per team of the SpMM (0: 2 for one column, else 1)
  int ew_nwg;       // max workgroups of the row-parallel reduction kernels
  int ew_rows;      // target rows per workgroup of those kernels
  int xcd;          // XCD-slab chunk order for the gathering kernels
  int graphs;       // replay captured iteration chunks as HIP graphs
  int precapture;   // one column: capture every chunk length up to 8 at a kind's first capture
  int fuse;         // one-column residual update fused with V^T r
  int lr_nwg;       // max workgroups of the one-column low-rank kernels
  int vrow;         // one-column low-rank kernels read the row-major BF16 factor
  int m11_bpt;      // blocks per team and chunk of the batched small-block solve
  int autotune;     // tune the SpMM chunk walk per index (off when pinned by the environment)
  int m11_sub1;     // lanes per row of the A12 gather in the 1-3 column block solve
  int m11_tile;     // rows per tile of the block solve for 2-15 columns
  int defer_x;      // batched LRC: x += alpha p with the search-direction update
  int sparse_rhs;   // one-column Schur right-hand side from the rows b reaches
  int rec_res;      // precision form: residual updated by M d (FP32 d) per sweep
  int m11_small_min;  // narrowest batch taking the register block solve (5..513; default 16)
  int lr_direct;    // widest column group (JW) of the unstaged narrow low-rank kernels (0: never)
  int spmm_slice;   // SpMM column-slice width for wider batches (0: one launch over all columns)
};
static int env_int(const char* name, int dflt, int lo, int hi) {
  const char* e = getenv(name);
  int v = e ? atoi(e) : dflt;
  return (v >= lo && v <= hi) ? v : dflt;
}
static const Tuning& tuning() {
  static const Tuning t = [] {
    Tuning u;
    u.ts1 = env_int("KATZ_SPMM_TS1", 8, 4, 32);
    if (u.ts1 != 4 && u.ts1 != 8 && u.ts1 != 16 && u.ts1 != 32) u.ts1 = 8;
    u.spmm_nwg = env_int("KATZ_SPMM_NWG", 8192, 64, 65536);
    u.rows_team = env_int("KATZ_SPMM_ROWS_PER_TEAM", 0, 0, 64);
    u.ew_nwg = env_int("KATZ_EW_NWG", 1024, 64, 65536);
    u.ew_rows = env_int("KATZ_EW_ROWS", 256, 16, 65536);
    u.xcd = env_int("KATZ_XCD_SLAB", 0, 0, 1);
    u.graphs = env_int("KATZ_GRAPHS", 1, 0, 1);
    u.precapture = env_int("KATZ_PRECAPTURE", 1, 0, 1);
    u.fuse = env_int("KATZ_FUSE", 1, 0, 1);
    u.lr_nwg = env_int("KATZ_LR_NWG", 512, 64, 65536);
    u.vrow = env_int("KATZ_VROW", 1, 0, 1);
    u.m11_bpt = env_int("KATZ_M11_BLOCKS_PER_TEAM", 1, 1, 64);
    u.autotune = env_int("KATZ_AUTOTUNE", 1, 0, 1) && !getenv("KATZ_XCD_SLAB") && !getenv("KATZ_SPMM_NWG");
    u.m11_sub1 = env_int("KATZ_M11_SUB", 4, 1, 16);
    u.m11_tile = env_int("KATZ_M11_TILE", 64, 16, 256);
    u.defer_x = env_int("KATZ_DEFER_X", 1, 0, 1);
    u.sparse_rhs = env_int("KATZ_SPARSE_RHS", 1, 0, 1);
    u.rec_res = env_int("KATZ_REC_RES", 1, 0, 1);
    u.m11_small_min = env_int("KATZ_M11_SMALL_MIN", 16, 5, 513);
    u.lr_direct = env_int("KATZ_LR_DIRECT_MAX", 8, 0, 16);
    u.spmm_slice = env_int("KATZ_SPMM_SLICE", 0, 0, 512);
    if (u.m11_sub1 & (u.m11_sub1 - 1)) u.m11_sub1 = 4;  // a power of two (shuffle reduction)
    return u;
  }();
  return t;
}

// SpMM chunk walk, packed as xcd << 24 | workgroups (at most 65536).
inline int32_t walk_pack(int xcd, int nwg) { return (int32_t)((xcd ? 1 : 0) << 24 | (nwg & 0xffffff)); }
inline int walk_xcd(int32_t w) { return (w >> 24) & 1; }
inline int walk_nwg(int32_t w) { return w & 0xffffff; }
// SpMM variants x panel precisions x weights (Launcher::spmm_variant).
constexpr int kWalkSlots = 13 * 2 * 2;
// Tuned walks of this process by graph shape (n, nnz, n1) and variant slot.
struct WalkKey {
  int64_t n, nnz, n1;
  int slot;
  bool operator<(const WalkKey& o) const {
    return std::tie(n, nnz, n1, slot) < std::tie(o.n, o.nnz, o.n1, o.slot);
  }
};
static std::map<WalkKey, int32_t>& walk_cache() {
  static std::map<WalkKey, int32_t> m;
  return m;
}
// Held while tuning; taken before hip_global_mu, never while holding it.
static std::mutex& walk_mu() {
  static std::mutex m;
  return m;
}

// ============================================================= device index
struct Workspace {
  int B = 0;  // capacity in columns (a call may use any width <= B)
  int64_t n = 0, n2 = 0;
  // FP64: Rhs (b, then each sweep's residual), K (accumulated solution).
  // Solve panels in the precision of the inner solves (FP64, or FP32 for
  // the precision form; typed at the point of use): Dx, X (n rows), Y, W
  // (n rows for CG, n2 used by LRC), Z (n2 rows).
  double *Rhs = nullptr, *K = nullptr;
  void *Dx = nullptr, *X = nullptr, *Y = nullptr, *W = nullptr, *Z = nullptr;
  double* partials = nullptr;
  size_t partials_cap = 0;
  double* seg = nullptr;  // first-stage sums of a reduction over many partial rows (kSegValues)
  double* DW = nullptr;
  double* DW2 = nullptr;  // terms D_k W_kj^2 of <r, z> (rank x B)
  double *rz, *pq, *alpha, *bcg, *rr, *thr, *bn2, *res2, *colscale, *rn2, *inv, *fwd;
  float* Rf = nullptr;             // scaled FP32 right-hand side (precision form)
  int *active, *status, *iters, *n_active, *mask;
  // batched LRC: columns whose step alpha was set by this iteration's S p
  // (their x += alpha p rides on the search-direction update)
  int* fresh = nullptr;
  int32_t* qpos = nullptr;
  char* tk_scratch = nullptr;    // top-K selection state and winners
  size_t tk_cap = 0;
  int32_t* tk_ids = nullptr;     // staging for host top-K output
  int32_t *pr_rows = nullptr, *pr_cols = nullptr;  // pair queries: rows, columns, values
  double* pr_out = nullptr;
  int64_t pr_cap = 0;
  double* tk_sc = nullptr;
  int64_t tk_out_cap = 0;
  void* hpin = nullptr;          // pinned host staging for small scalars
  std::vector<void*> allocs;
  int device = 0;
  ProfEvents prof;
  hipStream_t stream = nullptr;          // the workspace's own stream (default priority)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  // captured iteration chunks: solve kind, width, chunk length, iteration cap
  struct ChunkGraph { int kind, B, len, max_iter; hipGraphExec_t ex; };
  std::vector<ChunkGraph> graphs;
  // carved from caller-independent scratch (katz_query_noalloc): owns no
  // memory, stream or events; runs without graphs, profiling or autotuning
  bool external = false;
  // PCGNR ablation only (allocated on its first use): an n-row panel [t1 | r]
  // and an n2-row panel s = S r
  void *ab1 = nullptr, *ab2 = nullptr;
  ~Workspace();
};

struct DeviceIndex {
  int device = 0;
  int32_t n = 0, n1 = 0, n2 = 0, rank = 0, nblocks = 0, ntiles = 0, max_tile_rows = 0;
  int64_t nnz = 0;
  double beta = 0, c = 0;
  int l_kind = KATZ_L_IDENTITY;
  int precision = KATZ_PREC_FP64;
  int32_t *rp = nullptr, *col = nullptr, *split = nullptr, *perm = nullptr, *iperm = nullptr;
  double* val = nullptr;
  int32_t *tile_row0 = nullptr, *row_blk = nullptr, *blk_start = nullptr;
  // finer tiles (whole blocks, at most m11_tile rows unless one block is
  // larger) for the block solve of 2-15 columns
  int32_t* ntile_row0 = nullptr;
  int n_ntiles = 0, max_ntile_rows = 0;
  int64_t* blk_off = nullptr;
  // blocks with more than kSmallBlock rows: one tile each, [big_row0, big_row1)
  int32_t *big_row0 = nullptr, *big_row1 = nullptr;
  int n_big = 0, max_big_rows = 0;
  int64_t big_rows = 0;
  double* minv = nullptr;
  double* ginv = nullptr;
  double* V = nullptr;
  double* D = nullptr;
  // precision form: FP32 block inverses and G, BF16 low-rank factor
  float* minv32 = nullptr;
  float* ginv32 = nullptr;
  bf16* V16 = nullptr;      // column-major n2 x r
  bf16* V16r = nullptr;     // row-major n2 x r (MFMA operand layout)
  float* V32 = nullptr;     // column-major n2 x r, FP32 storage for the FP64 path
  int64_t bytes = 0, factor_bytes = 0;
  std::vector<void*> allocs;
  std::mutex mu;
  std::vector<std::unique_ptr<Workspace>> pool;
  double avg_deg = 0;
  // sizes for the algorithmic-byte formulas
  int64_t nnz_sep = 0, nnz_sep_left = 0, nnz_a12 = 0, cols_sep = 0, cols_sep_left = 0, cols_a12 = 0,
          cols_all = 0, minv_elems = 0;
  // hub rows (more than kLongRow entries) of the separator range and of all rows
  int32_t *long_sep = nullptr, *long_all = nullptr;
  int n_long_sep = 0, n_long_all = 0;
  // autotuned SpMM chunk walk per variant (-1: not tuned, the default applies)
  std::atomic<int32_t> walk[kWalkSlots];
  // iterations the last solve of each kind needed (method x precision x first
  // or later sweep; 0: none yet), the first poll of the adaptive schedule
  std::atomic<int32_t> iter_hint[8];
  // workgroups of the unstaged narrow V^T r kernel resident at once, per
  // panel precision (FP64, FP32; 0: not sized, the default grid applies)
  std::atomic<int32_t> lr_resident[2];
  // device buffers reused by calls that need scratch beyond a workspace
  // (Sparse-Katz's gathered K_T and lists): taken and returned under aux_mu
  std::mutex aux_mu;
  std::vector<std::pair<void*, size_t>> aux_free;
};
constexpr int kLongRow = 256;
// HIP graphs of iteration chunks kept per workspace.
constexpr size_t kMaxGraphs = 128;
// Partial sums (rows x values) above which finalize reduces in two stages,
// and the size of the first stage's output.
constexpr int64_t kFinTwoStage = 1 << 20;
constexpr int64_t kSegValues = 1 << 16;
// Bound on an SpMM launch's chunk partials (chunks x batch width): wider
// batches take more rows per chunk.
constexpr int64_t kSpmmPartials = (int64_t)1 << 26;
// Batched block solves keep a block's rows in registers up to this size.
constexpr int kSmallBlock = 4;

namespace {

template <typename T>
T* dalloc(std::vector<void*>& list, int64_t count, int64_t* bytes = nullptr) {
  std::lock_guard<std::recursive_mutex> g(hip_global_mu());
  if (count <= 0) count = 1;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, (size_t)count * sizeof(T));
  if (e != hipSuccess) fail(e == hipErrorOutOfMemory ? KATZ_ENOMEM : KATZ_EDEVICE,
                            std::string("hipMalloc: ") + hipGetErrorString(e));
  list.push_back(p);
  if (bytes) *bytes += count * (int64_t)sizeof(T);
  return (T*)p;
}

// Grows a workspace buffer: *p (allocated from `list`, or null) is replaced
// by an allocation of `count` T and the old one freed.  Callers grow only
// between uses: a workspace serves one call at a time, and every use before
// the growth has been waited for (each batch of a call ends with a stream
// synchronisation).
template <typename T>
void dregrow(std::vector<void*>& list, T*& p, int64_t count) {
  std::lock_guard<std::recursive_mutex> g(hip_global_mu());
  if (p) {
    auto it = std::find(list.begin(), list.end(), (void*)p);
    if (it != list.end()) list.erase(it);
    (void)hipFree(p);
    p = nullptr;
  }
  p = dalloc<T>(list, count);
}

template <typename T>
T* upload(std::vector<void*>& list, const std::vector<T>& h, int64_t* bytes) {
  std::lock_guard<std::recursive_mutex> g(hip_global_mu());
  T* d = dalloc<T>(list, (int64_t)h.size(), bytes);
  if (!h.empty()) HIPCHECK(hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return d;
}

// float -> bfloat16 bits, round to nearest even (NaN kept quiet)
uint16_t bf16_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) return (uint16_t)((u >> 16) | 0x40);
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7FFFu + lsb;
  return (uint16_t)(u >> 16);
}

int grid_for(int64_t work, int per) {
  int64_t g = (work + per - 1) / per;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, 65535));
}

}  // namespace

// The low-rank factor's device copies (in the storage the index's precision
// and u_precision call for) and D.
static void upload_factors(const HostIndex& H, DeviceIndex* D) {
  D->rank = H.rank;
  if (H.rank <= 0) return;
  int64_t* by = &D->bytes;
  std::vector<double> vc((size_t)H.n2 * H.rank);  // column-major copy
  for (int64_t i = 0; i < H.n2; i++)
    for (int k = 0; k < H.rank; k++) vc[(size_t)k * H.n2 + i] = H.V[(size_t)i * H.rank + k];
  if (H.precision == KATZ_PREC_FP64 && H.u_precision == 2) {
    std::vector<float> v32(vc.begin(), vc.end());
    D->V32 = upload(D->allocs, v32, by);
  } else if (H.precision == KATZ_PREC_FP64 && H.u_precision == 3) {
    std::vector<uint16_t> vb(vc.size());
    for (size_t t = 0; t < vc.size(); t++) vb[t] = bf16_bits((float)vc[t]);
    D->V16 = (bf16*)upload(D->allocs, vb, by);
    // the row-major copy for the one-column kernels (16-byte row loads)
    if (H.rank == 8 || H.rank == 16 || H.rank == 32 || H.rank == 64) {
      std::vector<uint16_t> vr(vc.size());
      for (size_t t = 0; t < vc.size(); t++) vr[t] = bf16_bits((float)H.V[t]);
      D->V16r = (bf16*)upload(D->allocs, vr, by);
    }
  } else if (H.precision == KATZ_PREC_FP64) {
    D->V = upload(D->allocs, vc, by);
  }
  D->D = upload(D->allocs, H.D, by);
  if (H.precision == KATZ_PREC_MIXED) {
    std::vector<uint16_t> vb(vc.size()), vr(vc.size());
    for (size_t t = 0; t < vc.size(); t++) vb[t] = bf16_bits((float)vc[t]);
    for (int64_t i = 0; i < H.n2; i++)
      for (int k = 0; k < H.rank; k++) vr[(size_t)i * H.rank + k] = bf16_bits((float)H.V[(size_t)i * H.rank + k]);
    D->V16 = (bf16*)upload(D->allocs, vb, by);
    D->V16r = (bf16*)upload(D->allocs, vr, by);
  }
}

DeviceIndex* device_upload(const HostIndex& H, int device) {
  std::lock_guard<std::recursive_mutex> lk(hip_global_mu());
  HIPCHECK(hipSetDevice(device));
  auto D = new DeviceIndex();
  for (auto& x : D->walk) x.store(-1);
  for (auto& x : D->iter_hint) x.store(0);
  for (auto& x : D->lr_resident) x.store(0);
  try {
    D->device = device;
    D->n = H.n;
    D->n1 = H.n1;
    D->n2 = H.n2;
    D->nnz = H.nnz;
    D->beta = H.beta;
    D->c = H.c;
    D->l_kind = H.l_kind;
    D->precision = H.precision;
    D->rank = H.rank;
    D->avg_deg = H.n ? (double)H.nnz / H.n : 0;
    {
      // distinct columns touched by each row range (each gathered panel row is
      // counted once in the algorithmic bytes) and entry counts
      std::vector<char> seen(H.n, 0), seenl(H.n, 0), seena(H.n, 0), seenall(H.n, 0);
      for (int32_t i = 0; i < H.n; i++)
        for (int32_t k = H.rp[i]; k < H.rp[i + 1]; k++) {
          int32_t c = H.col[k];
          seenall[c] = 1;
          if (i >= H.n1) {
            D->nnz_sep++;
            seen[c] = 1;
            if (k < H.split[i]) { D->nnz_sep_left++; seenl[c] = 1; }
          } else if (k >= H.split[i]) {
            D->nnz_a12++;
            seena[c] = 1;
          }
        }
      for (int32_t c = 0; c < H.n; c++) {
        D->cols_sep += seen[c];
        D->cols_sep_left += seenl[c];
        D->cols_a12 += seena[c];
        D->cols_all += seenall[c];
      }
      D->minv_elems = (int64_t)H.minv.size();
      std::vector<int32_t> ls, la;
      for (int32_t i = 0; i < H.n; i++)
        if (H.rp[i + 1] - H.rp[i] > kLongRow) {
          la.push_back(i);
          if (i >= H.n1) ls.push_back(i);
        }
      D->n_long_sep = (int)ls.size();
      D->n_long_all = (int)la.size();
      D->long_sep = upload(D->allocs, ls, &D->bytes);
      D->long_all = upload(D->allocs, la, &D->bytes);
    }
    int64_t* by = &D->bytes;
    D->rp = upload(D->allocs, H.rp, by);
    D->col = upload(D->allocs, H.col, by);
    D->split = upload(D->allocs, H.split, by);
    D->perm = upload(D->allocs, H.perm, by);
    D->iperm = upload(D->allocs, H.iperm, by);
    if (H.weighted) D->val = upload(D->allocs, H.val, by);
    // tiles of consecutive blocks with at most 256 rows (a larger block is a
    // tile of its own)
    const int nb = (int)H.blk_start.size() - 1;
    D->nblocks = nb;
    std::vector<int32_t> tiles{0}, row_blk(std::max(1, H.n1));
    int32_t cur = 0;
    int max_rows = 0;
    for (int b = 0; b < nb; b++) {
      int32_t s = H.blk_start[b], e = H.blk_start[b + 1];
      for (int32_t i = s; i < e; i++) row_blk[i] = b;
      if (e - tiles.back() > WG && s > tiles.back()) {
        tiles.push_back(s);
      }
      cur = e;
      (void)cur;
    }
    if (tiles.back() != H.n1) tiles.push_back(H.n1);
    if (H.n1 == 0) tiles.assign(1, 0);
    for (size_t t = 0; t + 1 < tiles.size(); t++) max_rows = std::max(max_rows, tiles[t + 1] - tiles[t]);
    D->ntiles = (int)tiles.size() - 1;
    D->max_tile_rows = max_rows;
    D->tile_row0 = upload(D->allocs, tiles, by);
    {
      const int target = tuning().m11_tile;
      std::vector<int32_t> nt{0};
      for (int b = 0; b < nb; b++) {
        const int32_t s = H.blk_start[b], e = H.blk_start[b + 1];
        if (e - nt.back() > target && s > nt.back()) nt.push_back(s);
      }
      if (nt.back() != H.n1) nt.push_back(H.n1);
      if (H.n1 == 0) nt.assign(1, 0);
      int mr = 0;
      for (size_t t = 0; t + 1 < nt.size(); t++) mr = std::max(mr, nt[t + 1] - nt[t]);
      D->n_ntiles = (int)nt.size() - 1;
      D->max_ntile_rows = mr;
      D->ntile_row0 = upload(D->allocs, nt, by);
    }
    D->row_blk = upload(D->allocs, row_blk, by);
    D->blk_start = upload(D->allocs, H.blk_start, by);
    D->blk_off = upload(D->allocs, H.blk_off, by);
    {
      std::vector<int32_t> b0, b1;
      for (int b = 0; b < nb; b++) {
        const int32_t sz = H.blk_start[b + 1] - H.blk_start[b];
        if (sz <= kSmallBlock) continue;
        b0.push_back(H.blk_start[b]);
        b1.push_back(H.blk_start[b + 1]);
        D->max_big_rows = std::max(D->max_big_rows, (int)sz);
        D->big_rows += sz;
      }
      D->n_big = (int)b0.size();
      if (D->n_big) {
        D->big_row0 = upload(D->allocs, b0, by);
        D->big_row1 = upload(D->allocs, b1, by);
      }
    }
    int64_t fb0 = D->bytes;
    D->minv = upload(D->allocs, H.minv, by);
    D->factor_bytes = D->bytes - fb0;
    if (H.l_kind != KATZ_L_IDENTITY && H.n2 > 0) D->ginv = upload(D->allocs, H.ginv, by);
    if (H.precision == KATZ_PREC_MIXED) {
      std::vector<float> m32(H.minv.begin(), H.minv.end());
      D->minv32 = upload(D->allocs, m32, by);
      if (D->ginv) {
        std::vector<float> g32(H.ginv.begin(), H.ginv.end());
        D->ginv32 = upload(D->allocs, g32, by);
      }
    }
    upload_factors(H, D);
    HIPCHECK(hipDeviceSynchronize());
  } catch (...) {
    device_free(D);
    throw;
  }
  return D;
}

static void free_ws(Workspace* w) {
  std::lock_guard<std::recursive_mutex> lk(hip_global_mu());
  for (auto& g : w->graphs) (void)hipGraphExecDestroy(g.ex);
  w->graphs.clear();
  if (w->stream) (void)hipStreamDestroy(w->stream);
  if (w->ev_in) (void)hipEventDestroy(w->ev_in);
  if (w->ev_out) (void)hipEventDestroy(w->ev_out);
  w->stream = nullptr;
  w->ev_in = w->ev_out = nullptr;
  for (void* p : w->allocs) (void)hipFree(p);
  if (w->hpin && !w->external) (void)hipHostFree(w->hpin);
  w->hpin = nullptr;
  w->allocs.clear();
}
// Frees everything still held (also a workspace whose creation failed part
// way); free_ws is idempotent.
Workspace::~Workspace() { free_ws(this); }

void device_free(DeviceIndex* D) {
  if (!D) return;
  std::lock_guard<std::recursive_mutex> lk(hip_global_mu());
  (void)hipSetDevice(D->device);
  for (auto& w : D->pool) free_ws(w.get());
  for (void* p : D->allocs) (void)hipFree(p);
  for (auto& a : D->aux_free) (void)hipFree(a.first);
  delete D;
}
int64_t device_bytes(const DeviceIndex* D) { return D ? D->bytes : 0; }
int64_t device_factor_bytes(const DeviceIndex* D) { return D ? D->factor_bytes : 0; }

// Factor storage for a panel type: FP64 panels use the FP64 factors, FP32
// panels the FP32 block inverses and the BF16 low-rank factor.
template <typename T> struct Factors;
template <> struct Factors<double> {
  typedef double TV;
  static const double* minv(const DeviceIndex* D) { return D->minv; }
  static const double* ginv(const DeviceIndex* D) { return D->ginv; }
};
template <> struct Factors<float> {
  typedef bf16 TV;
  static const float* minv(const DeviceIndex* D) { return D->minv32; }
  static const float* ginv(const DeviceIndex* D) { return D->ginv32; }
};

constexpr size_t kPinFlagOff = 16384;  // pinned staging offset of the poll flag
constexpr size_t kPinProfOff = 28672;  // active-column count read for profiling

// ================================================================ workspace
// Element size of the inner-solve panels: FP32 for the precision form.
static int64_t solve_elem_bytes(const DeviceIndex* D) { return D->precision == KATZ_PREC_MIXED ? 4 : 8; }
// Partial sums per column: the largest producer is the SpMM (short + hub
// workgroups) or a row-parallel kernel, times max(1, rank) values.
static size_t partials_per_column(const DeviceIndex* D) {
  const Tuning& tu = tuning();
  size_t wgs = std::max<size_t>((size_t)tu.spmm_nwg + std::max(D->n_long_all, D->n_long_sep), (size_t)tu.ew_nwg);
  return wgs * (size_t)std::max(1, D->rank);
}
// Lanes per row (team size) of the SpMM for a launch of B columns.
static int spmm_team_size(int B) {
  if (B == 1) return tuning().ts1;
  if (B == 2) return 8;
  if (B <= 4) return 16;
  if (B <= 8) return 32;
  return 64;
}
// Rows per chunk of an SpMM launch of B columns over `rows` rows with n_long
// hub rows, whose partial rows are ld values apart: teams x rows_team, with
// rows_team raised until (n_long + chunks) x ld fits kSpmmPartials.
static int spmm_chunk_rows(int B, int ld, int64_t rows, int n_long) {
  const int64_t teams = WG / spmm_team_size(B);
  // one column: two rows per team (measured 2-3% faster than one, both
  // methods, over 4,096-16,384 workgroups on the 1M-node Chung-Lu graph)
  int64_t rt = tuning().rows_team > 0 ? tuning().rows_team : (B == 1 ? 2 : 1);
  const int64_t cap = std::max<int64_t>(1, kSpmmPartials / std::max(1, ld) - n_long);
  if ((rows + teams * rt - 1) / (teams * rt) > cap) rt = (rows + teams * cap - 1) / (teams * cap);
  return (int)(teams * rt);
}
// Partial sums a B-column workspace needs for its largest SpMM (all rows).
static size_t spmm_partials_need(const DeviceIndex* D, int B) {
  size_t need = 0;
  const int W = tuning().spmm_slice;
  for (int bw : {B, (W > 0 && B > W && B % W == 0) ? W : B}) {
    const int64_t cr = spmm_chunk_rows(bw, B, D->n, D->n_long_all);
    need = std::max(need, (size_t)(D->n_long_all + (D->n + cr - 1) / cr) * (size_t)B);
  }
  return need;
}
// First-stage sums of a two-stage reduction: at most kSegValues, or one row
// of nv values.
static size_t seg_values(const DeviceIndex* D, int B) {
  return std::max<size_t>({(size_t)kSegValues, (size_t)std::max(1, D->rank) * B, (size_t)B});
}
// Device bytes of a workspace per column of capacity (panels, FP32 copy of
// the right-hand side, partial sums, top-K scratch for K <= 4096).
int64_t ws_bytes_per_column(const DeviceIndex* D) {
  const int64_t n = D->n, n2 = std::max(1, D->n2), esz = solve_elem_bytes(D);
  int64_t b = 16 * n + esz * (4 * n + n2);
  if (D->precision == KATZ_PREC_MIXED) b += 4 * n;
  b += 8 * (int64_t)std::max(partials_per_column(D), spmm_partials_need(D, 1)) + 16 * std::max(1, D->rank);  // partials, DW, DW2
  b += 8 * (int64_t)std::max(1, D->rank) + 8;  // first-stage sums
  b += 64 + 1024 + 12 * 4096;
  return b;
}

static std::unique_ptr<Workspace> make_ws(DeviceIndex* D, int B) {
  std::lock_guard<std::recursive_mutex> lk(hip_global_mu());
  auto w = std::make_unique<Workspace>();
  w->B = B;
  w->n = D->n;
  w->n2 = D->n2;
  w->device = D->device;
  auto& L = w->allocs;
  const int64_t nB = (int64_t)D->n * B;
  const int64_t esz = solve_elem_bytes(D);
  w->Rhs = dalloc<double>(L, nB);
  w->K = dalloc<double>(L, nB);
  w->Dx = dalloc<char>(L, nB * esz);
  w->X = dalloc<char>(L, nB * esz);
  w->Y = dalloc<char>(L, nB * esz);
  w->W = dalloc<char>(L, nB * esz);
  w->Z = dalloc<char>(L, (int64_t)std::max(1, D->n2) * B * esz);
  w->partials_cap = std::max(partials_per_column(D) * (size_t)std::max(B, 1), spmm_partials_need(D, std::max(B, 1)));
  w->partials = dalloc<double>(L, (int64_t)w->partials_cap);
  w->seg = dalloc<double>(L, (int64_t)seg_values(D, std::max(B, 1)));
  w->DW = dalloc<double>(L, (int64_t)std::max(1, D->rank) * B);
  w->DW2 = dalloc<double>(L, (int64_t)std::max(1, D->rank) * B);
  double* s = dalloc<double>(L, 12 * (int64_t)B);
  w->rz = s; w->pq = s + B; w->alpha = s + 2 * B; w->bcg = s + 3 * B; w->rr = s + 4 * B;
  w->thr = s + 5 * B; w->bn2 = s + 6 * B; w->res2 = s + 7 * B; w->colscale = s + 8 * B;
  w->rn2 = s + 9 * B; w->inv = s + 10 * B; w->fwd = s + 11 * B;
  if (D->precision == KATZ_PREC_MIXED) w->Rf = dalloc<float>(L, nB);
  int* ip = dalloc<int>(L, 5 * (int64_t)B + 1);
  w->active = ip; w->status = ip + B; w->iters = ip + 2 * B; w->mask = ip + 3 * B; w->n_active = ip + 4 * B;
  w->fresh = ip + 4 * B + 1;
  w->qpos = dalloc<int32_t>(L, B);
  HIPCHECK(hipHostMalloc(&w->hpin, 64 * 1024, hipHostMallocDefault));
  HIPCHECK(hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking));
  HIPCHECK(hipEventCreateWithFlags(&w->ev_in, hipEventDisableTiming));
  HIPCHECK(hipEventCreateWithFlags(&w->ev_out, hipEventDisableTiming));
  // cleared on the workspace's own stream (not the legacy stream)
  HIPCHECK(hipMemsetAsync(s, 0, 12 * sizeof(double) * (size_t)B, w->stream));
  HIPCHECK(hipMemsetAsync(ip, 0, (4 * (size_t)B + 1) * sizeof(int), w->stream));
  HIPCHECK(hipStreamSynchronize(w->stream));
  return w;
}

// Takes the pooled workspace of the smallest capacity >= B (or makes one of
// capacity B) for the duration of a call, and returns it to the pool.
struct WsLease {
  DeviceIndex* D;
  std::unique_ptr<Workspace> w;
  WsLease(DeviceIndex* d, int B) : D(d) {
    {
      std::lock_guard<std::mutex> g(D->mu);
      int best = -1;
      for (size_t i = 0; i < D->pool.size(); i++)
        if (D->pool[i]->B >= B && (best < 0 || D->pool[i]->B < D->pool[best]->B)) best = (int)i;
      if (best >= 0) {
        w = std::move(D->pool[best]);
        D->pool.erase(D->pool.begin() + best);
      }
    }
    if (!w) w = make_ws(D, B);
  }
  ~WsLease() {
    std::lock_guard<std::mutex> g(D->mu);
    if (D->pool.size() >= 4) {
      free_ws(D->pool.front().get());
      D->pool.erase(D->pool.begin());
    }
    D->pool.push_back(std::move(w));
  }
};

// ============================================================ launch helpers
struct Launcher {
  DeviceIndex* D;
  Workspace* w;
  hipStream_t st;
  int B;
  int iter_hint = 0;  // first poll of the adaptive schedule (0: default)
  int* fresh_out = nullptr;  // EP_PQ finalizes flag the columns given a step here

  ColState cs(int max_iter) const {
    ColState c;
    c.rz = w->rz; c.pq = w->pq; c.alpha = w->alpha; c.bcg = w->bcg; c.rr = w->rr; c.thr = w->thr;
    c.active = w->active; c.status = w->status; c.iters = w->iters; c.n_active = w->n_active;
    c.mask = w->mask; c.max_iter = max_iter;
    return c;
  }

  // Runs launch(); with profiling on, brackets it with HIP events and books
  // `bytes` algorithmic bytes to `kind`.
  template <typename F>
  void timed(int kind, double bytes, F&& launch) {
    const bool on = g_prof_on.load(std::memory_order_relaxed) != 0 && !w->external;
    if (on) w->prof.begin(kind, bytes, st);
    launch();
    if (on) w->prof.end(st);
  }
  // As timed(), for kernels that touch only the active columns: with
  // profiling on, first reads the active-column count (a stream sync outside
  // the timed region) and books bytes_per_col for each active column.
  template <typename F>
  void timed_cols(int kind, double bytes_per_col, F&& launch) {
    double b = 0.0;
    if (g_prof_on.load(std::memory_order_relaxed) != 0 && !w->external) {
      int* h = (int*)((char*)w->hpin + kPinProfOff);
      HIPCHECK(hipMemcpyAsync(h, w->n_active, sizeof(int), hipMemcpyDeviceToHost, st));
      HIPCHECK(hipStreamSynchronize(st));
      b = bytes_per_col * (double)*h;
    }
    timed(kind, b, launch);
  }
  void sync() {
    HIPCHECK(hipStreamSynchronize(st));
    w->prof.harvest();
  }

  template <typename T>
  void fill(T* p, int64_t cnt, T v) {
    if (cnt <= 0) return;
    k_fill<T><<<grid_for(cnt, WG * 4), WG, 0, st>>>(p, cnt, v);
  }

  // Workgroups for the elementwise reduction kernels over m rows.
  int rows_per_wg(int64_t m) const {
    const Tuning& tu = tuning();
    int64_t nwg = std::min<int64_t>(tu.ew_nwg, std::max<int64_t>(1, (m + tu.ew_rows - 1) / tu.ew_rows));
    return (int)((m + nwg - 1) / nwg);
  }
  // Checked before every launch that writes nwg x nv partial sums.
  void need(int64_t nwg, int64_t nv) const {
    if ((size_t)(nwg * nv) > w->partials_cap) fail(KATZ_EDEVICE, "internal: partials buffer too small");
  }
  static int nwg_for(int64_t m, int rpw) { return (int)((m + rpw - 1) / rpw); }

  // Reduces nwg x nv partials and applies the epilogue `ep` (one workgroup).
  void finalize(int nwg, int nv, int ep, const ColState& cs, double* out, const int* nact,
                double* out2 = nullptr, int rz_mode = 0) {
    need(nwg, nv);
    const double* src = w->partials;
    if ((int64_t)nwg * nv > kFinTwoStage && nwg > 1) {
      // many partial rows: segments of consecutive rows summed in row order
      // by many workgroups into w->seg, then the one-workgroup step over the
      // segment sums (both stages in a fixed order)
      const int64_t nseg0 = std::max<int64_t>(1, std::min<int64_t>(1024, kSegValues / nv));
      const int64_t seg = (nwg + nseg0 - 1) / nseg0;
      const int64_t nseg = (nwg + seg - 1) / seg;
      k_seg_reduce<<<dim3((unsigned)((nv + 63) / 64), (unsigned)nseg), WG, 0, st>>>(w->partials, nwg, nv, seg,
                                                                                   w->seg, nact);
      src = w->seg;
      nwg = (int)nseg;
    }
    k_finalize<<<1, kFinWG, 0, st>>>(src, nwg, nv, ep, cs, B, out, D->D, nact, out2, rz_mode,
                                     ep == EP_PQ ? fresh_out : nullptr);
  }

  // SpMM kernel variant for this batch width: team size TS, column lanes CW,
  // compile-time column groups NCM and weights; `slot` numbers the variant
  // (with the panel precision) for the autotuned chunk walk.  FP32 x with
  // FP64 sums (TX = float, T = double) exists for 16 columns and more and
  // shares the FP64 variant's walk.
  template <typename T, typename TX = T>
  struct SpmmVariant {
    void (*fn)(SpmmArgs<T, TX>);
    int TS, CW, slot;
  };
  template <typename T, typename TX = T>
  SpmmVariant<T, TX> spmm_variant(bool weighted, int B) const {
    const Tuning& tu = tuning();
    (void)tu;
    const int TS = spmm_team_size(B);
    const int CW = B <= 1 ? 1 : (B <= 2 ? 2 : (B <= 4 ? 4 : (B <= 8 ? 8 : (B <= 16 ? 16 : (B <= 32 ? 32 : 64)))));
    if (B > MAXC * CW) fail(KATZ_EINVAL, "batch too wide for one launch");
    const int nc = (B + CW - 1) / CW;  // column groups per lane
    SpmmVariant<T, TX> v{nullptr, TS, CW, -1};
    int idx = 0;
#define KZ_SPMM_V(ts, cw, ncm)                                                              \
  if constexpr (std::is_same<T, TX>::value || cw >= 16) {                                   \
    if (!v.fn && TS == ts && CW == cw && nc <= ncm) {                                       \
      v.fn = weighted ? k_spmm<T, ts, cw, true, ncm, TX> : k_spmm<T, ts, cw, false, ncm, TX>; \
      v.slot = idx;                                                                         \
    }                                                                                       \
  }                                                                                         \
  idx++;
    KZ_SPMM_V(4, 1, 1) KZ_SPMM_V(8, 1, 1) KZ_SPMM_V(16, 1, 1) KZ_SPMM_V(32, 1, 1) KZ_SPMM_V(8, 2, 1)
    KZ_SPMM_V(16, 4, 1) KZ_SPMM_V(32, 8, 1) KZ_SPMM_V(64, 16, 1) KZ_SPMM_V(64, 32, 1)
    KZ_SPMM_V(64, 64, 1) KZ_SPMM_V(64, 64, 2) KZ_SPMM_V(64, 64, 4) KZ_SPMM_V(64, 64, 8)
#undef KZ_SPMM_V
    if (!v.fn) fail(KATZ_EDEVICE, "internal: no SpMM variant for this batch width");
    v.slot = (v.slot * 2 + (sizeof(T) == 8 ? 1 : 0)) * 2 + (weighted ? 1 : 0);
    return v;
  }

  // Fills in the launch shape of `a` (chunking, walk, hub rows, partials)
  // and returns the grid and LDS size.
  template <typename T, typename TX>
  void spmm_shape(SpmmArgs<T, TX>& a, const SpmmVariant<T, TX>& v, int32_t walk, dim3& g, size_t& shm) const {
    const int B = a.B;
    const Tuning& tu = tuning();
    const int64_t rows = a.row1 - a.row0;
    const int teams = WG / v.TS;
    (void)tu;
    a.partials = w->partials;
    a.long_thr = kLongRow;
    if (a.row0 == D->n1 && a.row1 == D->n) { a.long_rows = D->long_sep; a.n_long = D->n_long_sep; }
    else if (a.row0 == 0 && a.row1 == D->n) { a.long_rows = D->long_all; a.n_long = D->n_long_all; }
    else { a.long_rows = nullptr; a.n_long = 0; }
    if (a.n_long == 0) a.long_rows = nullptr;
    // chunks of teams x rows_team rows, walked contiguously or in XCD slabs;
    // chunk ch's dot terms are partial row n_long + ch
    a.rows_per_wg = spmm_chunk_rows(B, a.ld, rows, a.n_long);
    a.xcd = walk_xcd(walk);
    a.nchunks = (rows + a.rows_per_wg - 1) / a.rows_per_wg;
    const int64_t nwg = std::min<int64_t>(walk_nwg(walk), a.nchunks);
    g = dim3((unsigned)(nwg + a.n_long));
    shm = sizeof(double) * std::max<size_t>((size_t)teams * B, (size_t)(WG / 64) * MAXC * v.CW);
  }

  template <typename T, typename TX = T>
  void spmm(SpmmArgs<T, TX> a) {
    const int64_t rows = a.row1 - a.row0;
    if (rows <= 0) {
      if (a.ep != EP_NONE) fail(KATZ_EDEVICE, "internal: empty SpMM with a reduction");
      return;
    }
    // column slices: launches of W columns each over the same rows (every
    // slice has the same launch shape, so the partial sums line up for one
    // finalize over all B columns)
    const int W = tuning().spmm_slice;
    const int nsl = (W > 0 && B > W && B % W == 0) ? B / W : 1;
    const int bw = B / nsl;
    a.ld = B;
    a.B = bw;
    const SpmmVariant<T, TX> v = spmm_variant<T, TX>(a.val != nullptr, bw);
    dim3 g;
    size_t shm;
    spmm_shape(a, v, walk_for(v.slot), g, shm);
    const int prows = (int)(a.n_long + a.nchunks);  // partial rows (walk-independent)
    need(prows, B);
    // algorithmic bytes: row pointers and splits, the selected entries, each
    // gathered panel row once, the row-aligned panels read and y written
    const bool sep = a.row0 == D->n1 && a.row1 == D->n;
    int64_t nnz_sel, cols_sel;
    if (sep && a.parts == 1) { nnz_sel = D->nnz_sep_left; cols_sel = D->cols_sep_left; }
    else if (sep) { nnz_sel = D->nnz_sep; cols_sel = D->cols_sep; }
    else { nnz_sel = D->nnz; cols_sel = D->cols_all; }
    const double wb = (double)sizeof(T) * B, wbx = (double)sizeof(TX) * B;
    const int panels = 1 + (a.v ? 1 : 0) + ((a.dotv && a.dotv != a.v) ? 1 : 0);
    double bytes = 8.0 * rows + 4.0 + (4.0 + (a.val ? 8.0 : 0.0)) * nnz_sel + wbx * cols_sel + wb * rows * panels +
                   (a.w ? wbx * rows : 0.0);
    const int kind = sep ? (a.parts == 1 ? PK_SPMM_RHS : PK_SPMM_SEP) : PK_SPMM_FULL;
    timed(kind, bytes, [&] {
      for (int sl = 0; sl < nsl; sl++) {
        a.j0 = sl * bw;
        v.fn<<<g, WG, shm, st>>>(a);
      }
    });
    if (a.ep != EP_NONE) finalize(prows, B, a.ep, a.cs, a.out, a.n_active);
  }

  // Chunk walk of an SpMM variant: the one tuned for this index, else the
  // default (contiguous chunks over spmm_nwg workgroups, or as pinned by
  // KATZ_XCD_SLAB / KATZ_SPMM_NWG).
  int32_t walk_for(int slot) const {
    const int32_t t = D->walk[slot].load(std::memory_order_acquire);
    if (t >= 0) return t;
    const Tuning& tu = tuning();
    return walk_pack(tu.xcd, tu.spmm_nwg);
  }

  // Autotuner of the SpMM chunk walk (the launch shape that decides which
  // rows run together, and so how well the gathered panel rows are reused in
  // the L2 and the last-level cache).  Candidates: the default (contiguous
  // chunks over spmm_nwg workgroups, which balances power-law row lengths)
  // and XCD slabs over R/4, R/2, R and 2R workgroups, R the resident count
  // (each XCD walks its own slab in a narrow sliding window, which suits
  // community-ordered graphs).  Each is timed on the launch `a` describes (one warm-up and two
  // timed launches; `a.y` must be a panel the caller overwrites afterwards)
  // and the fastest kept, a non-default only when 3% faster.  The choice is
  // kept per index and variant, and per process for the graph's shape.  It
  // changes no result bit: the reductions are indexed by chunk, not by
  // workgroup.  Not run under HIP-graph capture or when the walk is pinned by
  // the environment.
  template <typename T>
  void tune_spmm(SpmmArgs<T> a) {
    const Tuning& tu = tuning();
    if (a.row1 <= a.row0) return;
    const int W = tu.spmm_slice;
    a.B = (W > 0 && B > W && B % W == 0) ? W : B;   // the launch width spmm() uses
    a.ld = B;
    a.j0 = 0;
    const SpmmVariant<T> v = spmm_variant<T>(a.val != nullptr, a.B);
    if (!tu.autotune || w->external || D->walk[v.slot].load(std::memory_order_acquire) >= 0) return;
    hipStreamCaptureStatus cst = hipStreamCaptureStatusNone;
    HIPCHECK(hipStreamIsCapturing(st, &cst));
    if (cst != hipStreamCaptureStatusNone) return;
    std::lock_guard<std::mutex> lk(walk_mu());
    if (D->walk[v.slot].load(std::memory_order_acquire) >= 0) return;
    // no other thread captures a graph or allocates while the candidates run
    std::lock_guard<std::recursive_mutex> lg(hip_global_mu());
    const WalkKey key{D->n, D->nnz, D->n1, v.slot};
    auto& cache = walk_cache();
    const auto it = cache.find(key);
    if (it != cache.end()) {
      D->walk[v.slot].store(it->second, std::memory_order_release);
      return;
    }
    a.ep = EP_NONE; a.v = nullptr; a.w = nullptr; a.dotv = nullptr; a.n_active = nullptr;
    dim3 g;
    size_t shm;
    spmm_shape(a, v, walk_pack(tu.xcd, tu.spmm_nwg), g, shm);
    int per_cu = 0, cus = 0;
    HIPCHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, v.fn, WG, shm));
    HIPCHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, D->device));
    const int R = std::max(1, per_cu) * std::max(1, cus);
    // XCD slabs over R/4 .. 2R workgroups: fewer workgroups per XCD narrow
    // the window of rows it works on at once (less reuse lost to eviction),
    // more of them keep more gathers in flight
    constexpr int kCand = 5;
    const int32_t cand[kCand] = {walk_pack(tu.xcd, tu.spmm_nwg), walk_pack(1, std::max(8, R / 4)),
                                 walk_pack(1, std::max(8, R / 2)), walk_pack(1, std::min(R, 65536)),
                                 walk_pack(1, std::min(2 * R, 65536))};
    float ms[kCand] = {0.f, 0.f, 0.f, 0.f, 0.f};
    hipEvent_t e0, e1;
    HIPCHECK(hipEventCreate(&e0));
    HIPCHECK(hipEventCreate(&e1));
    for (int c = 0; c < kCand; c++) {
      spmm_shape(a, v, cand[c], g, shm);
      v.fn<<<g, WG, shm, st>>>(a);
      HIPCHECK(hipEventRecord(e0, st));
      for (int r = 0; r < 2; r++) v.fn<<<g, WG, shm, st>>>(a);
      HIPCHECK(hipEventRecord(e1, st));
      HIPCHECK(hipEventSynchronize(e1));
      HIPCHECK(hipEventElapsedTime(&ms[c], e0, e1));
    }
    HIPCHECK(hipEventDestroy(e0));
    HIPCHECK(hipEventDestroy(e1));
    HIPCHECK(hipGetLastError());
    int best = 0;
    for (int c = 1; c < kCand; c++)
      if (ms[c] < 0.97f * ms[best]) best = c;
    if (best != 0) {
      // among the slab walks within 3% of the fastest, the one over the most
      // workgroups: back-to-back launches find the caches warm, which
      // flatters a narrow window; in the solve other kernels run between
      // (4M-node SBM at 256 columns: 1,024 workgroups beat 512 by 2% there)
      const float bms = ms[best];
      for (int c = 1; c < kCand; c++)
        if (ms[c] <= 1.03f * bms && walk_nwg(cand[c]) > walk_nwg(cand[best])) best = c;
    }
    if (getenv("KATZ_VERBOSE") && atoi(getenv("KATZ_VERBOSE")) > 0)
      fprintf(stderr, "[katz] SpMM walk, variant %d, rows %d..%d, B %d: default %.3f ms, xcd slabs x%d %.3f ms, "
                      "x%d %.3f ms, x%d %.3f ms, x%d %.3f ms -> candidate %d\n", v.slot, a.row0, a.row1, B,
              ms[0] / 2, walk_nwg(cand[1]), ms[1] / 2, walk_nwg(cand[2]), ms[2] / 2, walk_nwg(cand[3]), ms[3] / 2,
              walk_nwg(cand[4]), ms[4] / 2, best);
    cache[key] = cand[best];
    D->walk[v.slot].store(cand[best], std::memory_order_release);
  }

  // Runs one_iter() up to max_iter times in chunks, polling the active-column
  // count after each chunk.  check_every > 0: chunks of that length.
  // check_every == 0 (adaptive): the first chunk is iter_hint (what the last
  // solve of this kind needed; 8 if none), then 1, 1, 2, 2, 4, 4, 8, 8, ...:
  // iterations after convergence still launch every kernel (which exits at
  // once) and each poll is a host round trip, so the schedule keeps both few
  // when consecutive solves need similar counts.  A chunk is captured once per
  // workspace, solve kind, width, length and iteration cap into a HIP graph
  // and replayed (not while profiling; at most kMaxGraphs per workspace,
  // further lengths run eagerly).  One column: the first capture of a kind
  // also captures every length up to 8, so that a later solve needing one
  // iteration more or less than the last replays a graph instead of paying
  // for a capture in its own latency.
  template <typename F>
  void iterate(int kind, int max_iter, int check_every, F&& one_iter) {
    int* hflag = (int*)((char*)w->hpin + kPinFlagOff);
    const bool graphs = tuning().graphs && !g_prof_on.load(std::memory_order_relaxed) && !w->external;
    auto find = [&](int len) -> hipGraphExec_t {
      for (const auto& g : w->graphs)
        if (g.kind == kind && g.B == B && g.len == len && g.max_iter == max_iter) return g.ex;
      return nullptr;
    };
    auto capture = [&](int len) -> hipGraphExec_t {
      std::lock_guard<std::recursive_mutex> lk(hip_global_mu());
      hipGraph_t gr = nullptr;
      HIPCHECK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      try {
        for (int s2 = 0; s2 < len; s2++) one_iter();
      } catch (...) {
        (void)hipStreamEndCapture(st, &gr);
        if (gr) (void)hipGraphDestroy(gr);
        throw;
      }
      HIPCHECK(hipStreamEndCapture(st, &gr));
      hipGraphExec_t ex = nullptr;
      hipError_t e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
      (void)hipGraphDestroy(gr);
      if (e != hipSuccess) fail(KATZ_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
      w->graphs.push_back({kind, B, len, max_iter, ex});
      return ex;
    };
    int it = 0;
    for (int chunk = 0; it < max_iter; chunk++) {
      int want;
      if (check_every > 0) want = check_every;
      else if (chunk == 0) want = iter_hint > 0 ? iter_hint : 8;
      else want = std::min(8, 1 << ((chunk - 1) / 2));
      const int len = std::min(want, max_iter - it);
      hipGraphExec_t ex = nullptr;
      if (graphs) {
        ex = find(len);
        if (!ex && w->graphs.size() < kMaxGraphs) {
          bool first = true;
          for (const auto& g : w->graphs)
            if (g.kind == kind && g.B == B && g.max_iter == max_iter) first = false;
          ex = capture(len);
          if (first && B == 1 && check_every == 0 && tuning().precapture)
            for (int l = 1; l <= std::min(8, max_iter); l++)
              if (l != len && w->graphs.size() < kMaxGraphs) capture(l);
        }
      }
      if (ex)
        HIPCHECK(hipGraphLaunch(ex, st));
      else
        for (int s2 = 0; s2 < len; s2++) one_iter();
      it += len;
      HIPCHECK(hipMemcpyAsync(hflag, w->n_active, sizeof(int), hipMemcpyDeviceToHost, st));
      sync();
      if (*hflag == 0) break;
    }
  }

  // out[j] = sum of squares of column j of the m x B panel p
  template <typename T>
  void colnorm2(const T* p, int64_t m, double* out) {
    const int rpw = rows_per_wg(m), nwg = nwg_for(m, rpw);
    need(nwg, B);
    k_colnorm2<T><<<nwg, WG, WG * sizeof(double), st>>>(p, m, B, rpw, w->partials);
    finalize(nwg, B, EP_NORM, cs(0), out, nullptr);
  }
};

// Relative accuracy the FP32 inner solves are asked for (the FP64 sweeps do the rest).
constexpr double kInnerTolFP32 = 1e-5;

// Pinned host staging (w->hpin, 64 KiB), B <= 512:
constexpr size_t kPinQ = 0, kPinMask0 = 2048, kPinMask1 = 4096, kPinBn2 = 8192, kPinRes = 12288,
                 kPinFlag = kPinFlagOff, kPinStat0 = 20480, kPinIter0 = 22528, kPinStat1 = 24576, kPinIter1 = 26624;
// the row lists of the sparse one-column Schur right-hand side
constexpr size_t kPinList = 32768;
constexpr int kPinListCap = 8192;

// The structure of the sparse one-column Schur right-hand side for b =
// beta A e_qp (qp a permuted position), laid out in out[] as k_schur_rhs1
// reads it: the rows of the blocks holding a neighbour of qp (nt), the
// separator rows next to qp or to those rows, ascending (ns), per separator
// row the offsets (ns + 1) into the entry pairs, then the pairs' block rows
// and CSR entries (np each), sorted by (separator row, block row).  False
// when it takes more than cap values.
static bool sparse_rhs_rows(const HostIndex& H, int32_t qp, int32_t* out, int cap, int& nt, int& ns, int& np) {
  std::vector<int32_t> blocks;
  for (int32_t k = H.rp[qp]; k < H.split[qp]; k++)  // block columns (< n1) come first in a row
    blocks.push_back((int32_t)(std::upper_bound(H.blk_start.begin(), H.blk_start.end(), H.col[k]) -
                               H.blk_start.begin()) - 1);
  std::sort(blocks.begin(), blocks.end());
  blocks.erase(std::unique(blocks.begin(), blocks.end()), blocks.end());
  std::vector<int32_t> trow;
  for (int32_t b : blocks)
    for (int32_t r = H.blk_start[b]; r < H.blk_start[b + 1]; r++) trow.push_back(r);
  if ((int64_t)trow.size() > cap) return false;
  // (separator row, block row, entry) for every entry of the block rows
  // towards the separator; the block rows ascend, so a stable sort by the
  // separator row keeps each row's terms in block-row order
  struct Pair { int32_t i, j, k; };
  std::vector<Pair> pr;
  for (int32_t j : trow)
    for (int32_t k = H.split[j]; k < H.rp[j + 1]; k++) pr.push_back({H.col[k], j, k});
  if ((int64_t)trow.size() + 3 * (int64_t)pr.size() > cap) return false;
  std::stable_sort(pr.begin(), pr.end(), [](const Pair& x, const Pair& y) { return x.i < y.i; });
  std::vector<int32_t> srow(H.col.begin() + H.split[qp], H.col.begin() + H.rp[qp + 1]);
  for (const Pair& x : pr) srow.push_back(x.i);
  std::sort(srow.begin(), srow.end());
  srow.erase(std::unique(srow.begin(), srow.end()), srow.end());
  nt = (int)trow.size();
  ns = (int)srow.size();
  np = (int)pr.size();
  if ((int64_t)nt + ns + (ns + 1) + 2 * (int64_t)np > cap) return false;
  int32_t* o = out;
  o = std::copy(trow.begin(), trow.end(), o);
  o = std::copy(srow.begin(), srow.end(), o);
  int32_t* off = o;
  size_t p = 0;
  for (int s = 0; s < ns; s++) {
    off[s] = (int32_t)p;
    while (p < pr.size() && pr[p].i == srow[s]) p++;
  }
  off[ns] = (int32_t)p;
  o += ns + 1;
  for (int t = 0; t < np; t++) o[t] = pr[t].j;
  for (int t = 0; t < np; t++) o[np + t] = pr[t].k;
  return true;
}

// Rank-r preconditioner on MFMA for FP32 panels: DW = D o (V^T r) by split-K
// tiles + finalize; z = r + V DW with the <r, z> partials + finalize.
static void precond_mfma(Launcher& L, const float* R2, float* Z2, int ep, const ColState& cs, const int* nact) {
  DeviceIndex* D = L.D;
  Workspace* w = L.w;
  const int B = L.B, rank = D->rank;
  const int64_t m = D->n2;
  hipStream_t st = L.st;
  const int jt = (B + 63) / 64, kt = (rank + 31) / 32;
  int S = (int)std::max<int64_t>(1, std::min<int64_t>(512, 2048 / (jt * kt)));
  S = (int)std::min<int64_t>(S, (m + 31) / 32);
  int64_t rows_per_chunk = ((m + S - 1) / S + 31) / 32 * 32;
  S = (int)((m + rows_per_chunk - 1) / rows_per_chunk);
  L.need(S, (int64_t)rank * B);
  L.timed(PK_VT, 2.0 * m * rank + 4.0 * B * m, [&] {
    k_vt_mfma<<<dim3(jt, kt, S), WG, 0, st>>>(m, B, rank, D->V16, R2, rows_per_chunk, w->partials, nact);
  });
  L.finalize(S, rank * B, EP_VT, cs, w->DW, nact);
  const int64_t ntile = (m + 63) / 64;
  const int gx = (int)std::min<int64_t>(ntile, 1024);
  L.need(gx, B);
  const int KP = (rank + 31) / 32 * 32;
  const size_t shm = (size_t)KP * 64 * 2 * sizeof(uint16_t) + 4 * 64 * sizeof(double);
  if (shm > 65536) {  // rank > 224: ask for more than the default 64 KiB of LDS
    static std::mutex mu;
    static size_t granted = 65536;
    std::lock_guard<std::mutex> g(mu);
    if (shm > granted) {
      HIPCHECK(hipFuncSetAttribute((const void*)k_lowrank_mfma, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
      granted = shm;
    }
  }
  L.timed(PK_LOWRANK, 2.0 * m * rank + 4.0 * B * m * 2, [&] {
    k_lowrank_mfma<<<dim3(gx, jt), WG, shm, st>>>(m, B, rank, D->V16r, w->DW, R2, Z2, 0, w->partials, nact);
  });
  L.finalize(gx, B, ep, cs, nullptr, nact);
}

// Calls f(V) with the low-rank factor in the storage the index holds for
// panels of type T (FP32 panels: BF16; FP64 panels: BF16, FP32 or FP64).
template <typename T, typename F>
static void with_lowrank_factor(const DeviceIndex* D, F&& f) {
  if (std::is_same<T, float>::value || D->V16)
    f(D->V16);
  else if (D->V32)
    f(D->V32);
  else
    f(D->V);
}

// The row-blocked low-rank kernels for rank <= 64 (RMAX from the rank).
template <typename T, typename TV, bool DIRECT, bool VR = false>
static void launch_vt_rows(dim3 g, hipStream_t st, int64_t m, int B, int rk, int JW, const TV* V, const T* R2,
                           int64_t rpc, double* partials, const int* nact) {
  if (rk <= 8) k_vt_rows<T, TV, 8, DIRECT, VR><<<g, WG, 0, st>>>(m, B, rk, JW, V, R2, rpc, partials, nact);
  else if (rk <= 16) k_vt_rows<T, TV, 16, DIRECT, VR><<<g, WG, 0, st>>>(m, B, rk, JW, V, R2, rpc, partials, nact);
  else if (rk <= 32) k_vt_rows<T, TV, 32, DIRECT, VR><<<g, WG, 0, st>>>(m, B, rk, JW, V, R2, rpc, partials, nact);
  else k_vt_rows<T, TV, 64, DIRECT, VR><<<g, WG, 0, st>>>(m, B, rk, JW, V, R2, rpc, partials, nact);
}
// XU: the deferred x update of k_lowrank_rows (xk, alpha, fresh)
struct XU {
  void* xk = nullptr;
  const double* alpha = nullptr;
  const int* fresh = nullptr;
};
template <typename T, typename TV, bool PUPD, bool DIRECT, bool VR = false, bool XUP = false>
static void launch_lowrank_rows_x(dim3 g, hipStream_t st, int64_t m, int B, int rk, int JW, const TV* V,
                                  const double* DW, const T* R2, T* Z2, int has_base, int64_t rpc,
                                  const int* nact, double* partials, const double* bcg, const int* active, int init,
                                  XU xu) {
  T* xk = (T*)xu.xk;
  if (rk <= 8)
    k_lowrank_rows<T, TV, 8, PUPD, DIRECT, VR, XUP><<<g, WG, 0, st>>>(m, B, rk, JW, V, DW, R2, Z2, has_base, rpc,
                                                                      nact, partials, bcg, active, init, xk,
                                                                      xu.alpha, xu.fresh);
  else if (rk <= 16)
    k_lowrank_rows<T, TV, 16, PUPD, DIRECT, VR, XUP><<<g, WG, 0, st>>>(m, B, rk, JW, V, DW, R2, Z2, has_base, rpc,
                                                                       nact, partials, bcg, active, init, xk,
                                                                       xu.alpha, xu.fresh);
  else if (rk <= 32)
    k_lowrank_rows<T, TV, 32, PUPD, DIRECT, VR, XUP><<<g, WG, 0, st>>>(m, B, rk, JW, V, DW, R2, Z2, has_base, rpc,
                                                                       nact, partials, bcg, active, init, xk,
                                                                       xu.alpha, xu.fresh);
  else
    k_lowrank_rows<T, TV, 64, PUPD, DIRECT, VR, XUP><<<g, WG, 0, st>>>(m, B, rk, JW, V, DW, R2, Z2, has_base, rpc,
                                                                       nact, partials, bcg, active, init, xk,
                                                                       xu.alpha, xu.fresh);
}
// xu.xk set (PUPD, not at init): the variant that also takes x += alpha p
template <typename T, typename TV, bool PUPD, bool DIRECT, bool VR = false>
static void launch_lowrank_rows(dim3 g, hipStream_t st, int64_t m, int B, int rk, int JW, const TV* V,
                                const double* DW, const T* R2, T* Z2, int has_base, int64_t rpc, const int* nact,
                                double* partials, const double* bcg, const int* active, int init, XU xu = XU()) {
  if constexpr (PUPD) {
    if (xu.xk && !init) {
      launch_lowrank_rows_x<T, TV, PUPD, DIRECT, VR, true>(g, st, m, B, rk, JW, V, DW, R2, Z2, has_base, rpc, nact,
                                                           partials, bcg, active, init, xu);
      return;
    }
  }
  launch_lowrank_rows_x<T, TV, PUPD, DIRECT, VR, false>(g, st, m, B, rk, JW, V, DW, R2, Z2, has_base, rpc, nact,
                                                        partials, bcg, active, init, XU());
}
// Vr: the row-major BF16 factor (vrow_factor), read by the unstaged form.
template <typename T, typename TV>
static void vt_rows(bool direct, dim3 g, hipStream_t st, int64_t m, int B, int rk, int JW, const TV* V,
                    const T* R2, int64_t rpc, double* partials, const int* nact, const bf16* Vr = nullptr) {
  if (direct && Vr) launch_vt_rows<T, bf16, true, true>(g, st, m, B, rk, JW, Vr, R2, rpc, partials, nact);
  else if (direct) launch_vt_rows<T, TV, true>(g, st, m, B, rk, JW, V, R2, rpc, partials, nact);
  else launch_vt_rows<T, TV, false>(g, st, m, B, rk, JW, V, R2, rpc, partials, nact);
}
template <typename T, typename TV, bool PUPD>
static void lowrank_rows(bool direct, dim3 g, hipStream_t st, int64_t m, int B, int rk, int JW, const TV* V,
                         const double* DW, const T* R2, T* Z2, int has_base, int64_t rpc, const int* nact,
                         double* partials, const double* bcg = nullptr, const int* active = nullptr,
                         int init = 0, const bf16* Vr = nullptr, XU xu = XU()) {
  if (direct && Vr)
    launch_lowrank_rows<T, bf16, PUPD, true, true>(g, st, m, B, rk, JW, Vr, DW, R2, Z2, has_base, rpc, nact,
                                                   partials, bcg, active, init, xu);
  else if (direct)
    launch_lowrank_rows<T, TV, PUPD, true>(g, st, m, B, rk, JW, V, DW, R2, Z2, has_base, rpc, nact, partials, bcg,
                                           active, init, xu);
  else
    launch_lowrank_rows<T, TV, PUPD, false>(g, st, m, B, rk, JW, V, DW, R2, Z2, has_base, rpc, nact, partials,
                                            bcg, active, init, xu);
}

// Narrow batches run the unstaged kernels over one resident round of
// workgroups (so no chunk waits for a second round): the count is queried
// once per index and panel precision, outside HIP-graph capture, at the start
// of a solve; until then the default grid applies.
template <typename T, typename TV>
static const void* vt_rows_direct_fn(int rk) {
  if (rk <= 8) return (const void*)k_vt_rows<T, TV, 8, true>;
  if (rk <= 16) return (const void*)k_vt_rows<T, TV, 16, true>;
  if (rk <= 32) return (const void*)k_vt_rows<T, TV, 32, true>;
  return (const void*)k_vt_rows<T, TV, 64, true>;
}
template <typename T>
static void size_lowrank_rows(DeviceIndex* D, hipStream_t st) {
  const int slot = std::is_same<T, float>::value ? 1 : 0;
  if (!tuning().lr_direct || D->rank <= 0 || D->rank > 64) return;
  if (D->lr_resident[slot].load(std::memory_order_acquire) > 0) return;
  hipStreamCaptureStatus cst = hipStreamCaptureStatusNone;
  HIPCHECK(hipStreamIsCapturing(st, &cst));
  if (cst != hipStreamCaptureStatusNone) return;
  with_lowrank_factor<T>(D, [&](auto* V) {
    typedef typename std::remove_cv<typename std::remove_pointer<decltype(V)>::type>::type TV;
    int per_cu = 0, cus = 0;
    HIPCHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, vt_rows_direct_fn<T, TV>(D->rank), WG, 0));
    HIPCHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, D->device));
    D->lr_resident[slot].store(std::min(4096, std::max(1, per_cu) * std::max(1, cus)), std::memory_order_release);
  });
}
// Rows per chunk of the row-blocked low-rank kernels: 1024 chunks, or one
// resident round for the unstaged form once sized.
template <typename T>
static int64_t lowrank_rows_rpc(const DeviceIndex* D, int64_t m, bool direct) {
  int64_t chunks = 1024;
  if (direct) {
    const int res = D->lr_resident[std::is_same<T, float>::value ? 1 : 0].load(std::memory_order_acquire);
    if (res > 0) chunks = res;
  }
  return std::max<int64_t>(kVRows, (m + chunks - 1) / chunks);
}

// Rank-r preconditioner with the row-parallel kernels (any B, V of type TV):
// DW = D o (V^T r), then z = G r + V DW (G = M22^{-1} or I) with <r, z>.
// Preconditioner for B >= 2 columns and rank <= 64 with the row-blocked
// kernels: DW = D o (V^T r) (chunk partials, then a many-workgroup fixed-order
// reduction), then z = base + V DW with the <r, z> partials and finalize.
// The row-major BF16 factor for the one-column kernels, when V is the BF16
// factor and the index holds a row-major copy of it (rank 8, 16, 32 or 64).
template <typename TV>
static const bf16* vrow_factor(const DeviceIndex* D, const TV* V) {
  if (!std::is_same<TV, bf16>::value || !tuning().vrow || !D->V16r || (const void*)V != (const void*)D->V16)
    return nullptr;
  const int rk = D->rank;
  return (rk == 8 || rk == 16 || rk == 32 || rk == 64) ? D->V16r : nullptr;
}

// k_vt1 / k_lowrank1 over the row-major BF16 factor (RMAX = rank).
template <typename T>
static void vt1_vrow(hipStream_t st, int nwg, int64_t m, int rk, const bf16* Vr, const T* R2, int rpw,
                     double* partials, const int* nact) {
  switch (rk) {
    case 8: k_vt1<T, bf16, 8, true><<<nwg, WG, 0, st>>>(m, rk, Vr, R2, rpw, partials, nact); break;
    case 16: k_vt1<T, bf16, 16, true><<<nwg, WG, 0, st>>>(m, rk, Vr, R2, rpw, partials, nact); break;
    case 32: k_vt1<T, bf16, 32, true><<<nwg, WG, 0, st>>>(m, rk, Vr, R2, rpw, partials, nact); break;
    default: k_vt1<T, bf16, 64, true><<<nwg, WG, 0, st>>>(m, rk, Vr, R2, rpw, partials, nact); break;
  }
}
template <typename T, bool PUPD>
static void lowrank1_vrow(hipStream_t st, int nwg, size_t shm, int64_t m, int rk, const bf16* Vr, const double* DW,
                          const T* R2, T* Z2, int has_base, int rpw, const int* nact, double* partials,
                          const double* bcg, const int* active, int init) {
  switch (rk) {
    case 8:
      k_lowrank1<T, bf16, 8, PUPD, true><<<nwg, WG, shm, st>>>(m, rk, Vr, DW, R2, Z2, has_base, rpw, nact,
                                                               partials, bcg, active, init);
      break;
    case 16:
      k_lowrank1<T, bf16, 16, PUPD, true><<<nwg, WG, shm, st>>>(m, rk, Vr, DW, R2, Z2, has_base, rpw, nact,
                                                                partials, bcg, active, init);
      break;
    case 32:
      k_lowrank1<T, bf16, 32, PUPD, true><<<nwg, WG, shm, st>>>(m, rk, Vr, DW, R2, Z2, has_base, rpw, nact,
                                                                partials, bcg, active, init);
      break;
    default:
      k_lowrank1<T, bf16, 64, PUPD, true><<<nwg, WG, shm, st>>>(m, rk, Vr, DW, R2, Z2, has_base, rpw, nact,
                                                                partials, bcg, active, init);
      break;
  }
}

template <typename T, typename TV>
static void precond_rows(Launcher& L, const TV* V, const T* R2, T* Z2, int ep, const ColState& cs,
                         const int* nact) {
  DeviceIndex* D = L.D;
  Workspace* w = L.w;
  const int B = L.B, rk = D->rank;
  const int64_t m = D->n2;
  hipStream_t st = L.st;
  int JW = 1;
  while (JW < B && JW < WG) JW <<= 1;
  const int njt = (B + JW - 1) / JW;
  const bool direct = JW <= tuning().lr_direct;
  const bf16* vr = direct ? vrow_factor(D, V) : nullptr;
  const int64_t rpc = lowrank_rows_rpc<T>(D, m, direct);
  const int nchunk = (int)((m + rpc - 1) / rpc);
  const int64_t nv = (int64_t)rk * B;
  dim3 g((unsigned)nchunk, (unsigned)njt);
  L.need(nchunk, nv);
  L.timed(PK_VT, (double)sizeof(TV) * m * rk + (double)sizeof(T) * B * m, [&] {
    vt_rows<T, TV>(direct, g, st, m, B, rk, JW, V, R2, rpc, w->partials, nact, vr);
  });
  k_vt_reduce<<<(unsigned)((nv + 63) / 64), WG, 0, st>>>(w->partials, nchunk, nv, B, D->D, w->DW, nact);
  int has_base = 0;
  if (Factors<T>::ginv(D)) {
    L.timed(PK_OTHER, (double)sizeof(T) * (m * m + 2 * m * B), [&] {
      k_dense_apply<T><<<grid_for(m * B, WG), WG, 0, st>>>((int)m, B, Factors<T>::ginv(D), R2, Z2, nact);
    });
    has_base = 1;
  }
  L.need(nchunk, B);
  L.timed(PK_LOWRANK, (double)sizeof(TV) * m * rk + (double)sizeof(T) * B * m * (2 + has_base), [&] {
    lowrank_rows<T, TV, false>(direct, g, st, m, B, rk, JW, V, w->DW, R2, Z2, has_base, rpc, nact, w->partials,
                               nullptr, nullptr, 0, vr);
  });
  L.finalize(nchunk, B, ep, cs, nullptr, nact);
}

template <typename T, typename TV>
static void precond_simple(Launcher& L, const TV* V, const T* R2, T* Z2, int ep, const ColState& cs,
                           const int* nact, int rpw, int nwg) {
  DeviceIndex* D = L.D;
  Workspace* w = L.w;
  const int B = L.B, rk = D->rank;
  const int64_t m = D->n2;
  hipStream_t st = L.st;
  if (B >= 2 && rk > 0 && rk <= 64) {
    precond_rows<T, TV>(L, V, R2, Z2, ep, cs, nact);
    return;
  }
  if (B == 1) {
    // the one-column low-rank kernels amortize their per-workgroup rank-wide
    // reduction over more rows than the update kernels do
    const int64_t want = std::max<int64_t>(1, std::min<int64_t>(tuning().lr_nwg, (m + 63) / 64));
    rpw = (int)((m + want - 1) / want);
    nwg = Launcher::nwg_for(m, rpw);
    L.need(nwg, std::max(1, rk));
  }
  const bf16* Vr = B == 1 ? vrow_factor(D, V) : nullptr;
  if (rk > 0) {
    L.timed(PK_VT, (double)sizeof(TV) * m * rk + (double)sizeof(T) * B * m, [&] {
      if (Vr) vt1_vrow<T>(st, nwg, m, rk, Vr, R2, rpw, w->partials, nact);
      else if (B == 1 && rk <= 8) k_vt1<T, TV, 8><<<nwg, WG, 0, st>>>(m, rk, V, R2, rpw, w->partials, nact);
      else if (B == 1 && rk <= 16) k_vt1<T, TV, 16><<<nwg, WG, 0, st>>>(m, rk, V, R2, rpw, w->partials, nact);
      else if (B == 1 && rk <= 32) k_vt1<T, TV, 32><<<nwg, WG, 0, st>>>(m, rk, V, R2, rpw, w->partials, nact);
      else if (B == 1 && rk <= 64) k_vt1<T, TV, 64><<<nwg, WG, 0, st>>>(m, rk, V, R2, rpw, w->partials, nact);
      else k_vt<T, TV><<<nwg, WG, 0, st>>>(m, B, rk, V, R2, rpw, w->partials, nact);
    });
    L.finalize(nwg, rk * B, EP_VT, cs, w->DW, nact);
  }
  int has_base = 0;
  if (Factors<T>::ginv(D)) {
    L.timed(PK_OTHER, (double)sizeof(T) * (m * m + 2 * m * B), [&] {
      k_dense_apply<T><<<grid_for(m * B, WG), WG, 0, st>>>((int)m, B, Factors<T>::ginv(D), R2, Z2, nact);
    });
    has_base = 1;
  }
  L.timed(PK_LOWRANK, (double)sizeof(TV) * m * rk + (double)sizeof(T) * B * m * (2 + has_base), [&] {
    const size_t shm = WG * sizeof(double);
    if (Vr)
      lowrank1_vrow<T, false>(st, nwg, shm, m, rk, Vr, w->DW, R2, Z2, has_base, rpw, nact, w->partials, nullptr,
                              nullptr, 0);
    else if (B == 1 && rk >= 1 && rk <= 8)
      k_lowrank1<T, TV, 8><<<nwg, WG, shm, st>>>(m, rk, V, w->DW, R2, Z2, has_base, rpw, nact, w->partials);
    else if (B == 1 && rk >= 1 && rk <= 16)
      k_lowrank1<T, TV, 16><<<nwg, WG, shm, st>>>(m, rk, V, w->DW, R2, Z2, has_base, rpw, nact, w->partials);
    else if (B == 1 && rk >= 1 && rk <= 32)
      k_lowrank1<T, TV, 32><<<nwg, WG, shm, st>>>(m, rk, V, w->DW, R2, Z2, has_base, rpw, nact, w->partials);
    else if (B == 1 && rk >= 1 && rk <= 64)
      k_lowrank1<T, TV, 64><<<nwg, WG, shm, st>>>(m, rk, V, w->DW, R2, Z2, has_base, rpw, nact, w->partials);
    else
      k_lowrank<T, TV><<<nwg, WG, shm, st>>>(m, B, rk, V, w->DW, R2, Z2, has_base, rpw, nact, w->partials);
  });
  L.finalize(nwg, B, ep, cs, nullptr, nact);
}

// Preconditioner and search-direction update in one pass (L = I, 1 <= rank
// <= 64): W = V^T r and DW = D o W as in precond_rows / precond_simple, then
// <r, z> = <r, r> + sum_k D_k W_k^2 gives bcg before z exists (k_rz_lowrank),
// and one pass writes p = r + V DW + bcg p (init: p = r + V DW) for the
// active columns.  Saves writing and re-reading z and one launch per
// iteration.
template <typename T, typename TV>
static void precond_fused(Launcher& L, const TV* V, const T* R2, T* P2, int init, const ColState& cs,
                          const int* nact, T* xk = nullptr) {
  DeviceIndex* D = L.D;
  Workspace* w = L.w;
  const int B = L.B, rk = D->rank;
  const int64_t m = D->n2;
  hipStream_t st = L.st;
  const double pbytes = (double)sizeof(TV) * m * rk + (double)sizeof(T) * B * m * (init ? 2 : 3);
  if (B == 1) {
    const int64_t want = std::max<int64_t>(1, std::min<int64_t>(tuning().lr_nwg, (m + 63) / 64));
    const int rpw = (int)((m + want - 1) / want), nwg = Launcher::nwg_for(m, rpw);
    L.need(nwg, rk);
    const bf16* Vr = vrow_factor(D, V);
    L.timed(PK_VT, (double)sizeof(TV) * m * rk + (double)sizeof(T) * m, [&] {
      if (Vr) vt1_vrow<T>(st, nwg, m, rk, Vr, R2, rpw, w->partials, nact);
      else if (rk <= 8) k_vt1<T, TV, 8><<<nwg, WG, 0, st>>>(m, rk, V, R2, rpw, w->partials, nact);
      else if (rk <= 16) k_vt1<T, TV, 16><<<nwg, WG, 0, st>>>(m, rk, V, R2, rpw, w->partials, nact);
      else if (rk <= 32) k_vt1<T, TV, 32><<<nwg, WG, 0, st>>>(m, rk, V, R2, rpw, w->partials, nact);
      else k_vt1<T, TV, 64><<<nwg, WG, 0, st>>>(m, rk, V, R2, rpw, w->partials, nact);
    });
    L.finalize(nwg, rk, EP_VT, cs, w->DW, nact, w->DW2, init ? 2 : 1);  // with <r, z> and the step
    L.timed(PK_LOWRANK, pbytes, [&] {
      if (Vr)
        lowrank1_vrow<T, true>(st, nwg, 0, m, rk, Vr, w->DW, R2, P2, 0, rpw, nact, nullptr, cs.bcg, cs.active, init);
      else if (rk <= 8)
        k_lowrank1<T, TV, 8, true><<<nwg, WG, 0, st>>>(m, rk, V, w->DW, R2, P2, 0, rpw, nact, nullptr, cs.bcg,
                                                         cs.active, init);
      else if (rk <= 16)
        k_lowrank1<T, TV, 16, true><<<nwg, WG, 0, st>>>(m, rk, V, w->DW, R2, P2, 0, rpw, nact, nullptr, cs.bcg,
                                                          cs.active, init);
      else if (rk <= 32)
        k_lowrank1<T, TV, 32, true><<<nwg, WG, 0, st>>>(m, rk, V, w->DW, R2, P2, 0, rpw, nact, nullptr, cs.bcg,
                                                          cs.active, init);
      else
        k_lowrank1<T, TV, 64, true><<<nwg, WG, 0, st>>>(m, rk, V, w->DW, R2, P2, 0, rpw, nact, nullptr, cs.bcg,
                                                          cs.active, init);
    });
    return;
  }
  int JW = 1;
  while (JW < B && JW < WG) JW <<= 1;
  const int njt = (B + JW - 1) / JW;
  const bool direct = JW <= tuning().lr_direct;
  const bf16* vr = direct ? vrow_factor(D, V) : nullptr;
  const int64_t rpc = lowrank_rows_rpc<T>(D, m, direct);
  const int nchunk = (int)((m + rpc - 1) / rpc);
  const int64_t nv = (int64_t)rk * B;
  dim3 g((unsigned)nchunk, (unsigned)njt);
  L.need(nchunk, nv);
  L.timed(PK_VT, (double)sizeof(TV) * m * rk + (double)sizeof(T) * B * m, [&] {
    vt_rows<T, TV>(direct, g, st, m, B, rk, JW, V, R2, rpc, w->partials, nact, vr);
  });
  k_vt_reduce<<<(unsigned)((nv + 63) / 64), WG, 0, st>>>(w->partials, nchunk, nv, B, D->D, w->DW, nact, w->DW2);
  k_rz_lowrank<<<1, WG, 0, st>>>(rk, B, w->DW2, init, cs, nact);
  L.timed(PK_LOWRANK, pbytes, [&] {
    XU xu;
    xu.xk = xk; xu.alpha = cs.alpha; xu.fresh = w->fresh;
    lowrank_rows<T, TV, true>(direct, g, st, m, B, rk, JW, V, w->DW, R2, P2, 0, rpc, nact, nullptr, cs.bcg,
                              cs.active, init, vr, xk ? xu : XU());
  });
}

// One column, L = I, rank <= 64: x += alpha p; r -= alpha q with W = V^T r
// and <r, r> in one pass; one finalize gives DW = D o W, the convergence test
// and the PCG step (<r, z> = <r, r> + sum_k D_k W_k^2, bcg); then p = r +
// V DW + bcg p in one pass.  Two launches and one finalize per iteration
// fewer than update, V^T r and the fused apply as separate passes.
template <typename T, typename TV>
static void update_r_precond1(Launcher& L, const TV* V, T* x, T* p, T* r, const T* q, const ColState& cs) {
  DeviceIndex* D = L.D;
  Workspace* w = L.w;
  const int rk = D->rank;
  const int64_t m = D->n2;
  hipStream_t st = L.st;
  const int64_t want = std::max<int64_t>(1, std::min<int64_t>(tuning().lr_nwg, (m + 63) / 64));
  const int rpw = (int)((m + want - 1) / want), nwg = Launcher::nwg_for(m, rpw);
  L.need(nwg, rk + 1);
  const bf16* Vr = vrow_factor(D, V);
  L.timed(PK_UPDATE_R, 6.0 * sizeof(T) * m + (double)sizeof(TV) * m * rk, [&] {
    if (Vr) {
      switch (rk) {
        case 8: k_update_r_vt1<T, bf16, 8, true><<<nwg, WG, 0, st>>>(m, rpw, x, p, r, q, rk, Vr, cs, w->partials); break;
        case 16: k_update_r_vt1<T, bf16, 16, true><<<nwg, WG, 0, st>>>(m, rpw, x, p, r, q, rk, Vr, cs, w->partials); break;
        case 32: k_update_r_vt1<T, bf16, 32, true><<<nwg, WG, 0, st>>>(m, rpw, x, p, r, q, rk, Vr, cs, w->partials); break;
        default: k_update_r_vt1<T, bf16, 64, true><<<nwg, WG, 0, st>>>(m, rpw, x, p, r, q, rk, Vr, cs, w->partials); break;
      }
    } else if (rk <= 8) {
      k_update_r_vt1<T, TV, 8><<<nwg, WG, 0, st>>>(m, rpw, x, p, r, q, rk, V, cs, w->partials);
    } else if (rk <= 16) {
      k_update_r_vt1<T, TV, 16><<<nwg, WG, 0, st>>>(m, rpw, x, p, r, q, rk, V, cs, w->partials);
    } else if (rk <= 32) {
      k_update_r_vt1<T, TV, 32><<<nwg, WG, 0, st>>>(m, rpw, x, p, r, q, rk, V, cs, w->partials);
    } else {
      k_update_r_vt1<T, TV, 64><<<nwg, WG, 0, st>>>(m, rpw, x, p, r, q, rk, V, cs, w->partials);
    }
  });
  L.finalize(nwg, rk + 1, EP_RR_VT, cs, w->DW, w->n_active, w->DW2, 1);
  L.timed(PK_LOWRANK, (double)sizeof(TV) * m * rk + 3.0 * sizeof(T) * m, [&] {
    if (Vr)
      lowrank1_vrow<T, true>(st, nwg, 0, m, rk, Vr, w->DW, r, p, 0, rpw, w->n_active, nullptr, cs.bcg, cs.active, 0);
    else if (rk <= 8)
      k_lowrank1<T, TV, 8, true><<<nwg, WG, 0, st>>>(m, rk, V, w->DW, r, p, 0, rpw, w->n_active, nullptr, cs.bcg,
                                                       cs.active, 0);
    else if (rk <= 16)
      k_lowrank1<T, TV, 16, true><<<nwg, WG, 0, st>>>(m, rk, V, w->DW, r, p, 0, rpw, w->n_active, nullptr, cs.bcg,
                                                        cs.active, 0);
    else if (rk <= 32)
      k_lowrank1<T, TV, 32, true><<<nwg, WG, 0, st>>>(m, rk, V, w->DW, r, p, 0, rpw, w->n_active, nullptr, cs.bcg,
                                                        cs.active, 0);
    else
      k_lowrank1<T, TV, 64, true><<<nwg, WG, 0, st>>>(m, rk, V, w->DW, r, p, 0, rpw, w->n_active, nullptr, cs.bcg,
                                                        cs.active, 0);
  });
}

// ============================================================ solve sweeps
// One correction solve M d = rhs for the columns in w->mask; d is left in
// w->Dx (all n rows), per-column outcome in w->iters / w->status.
template <typename T>
// sp_rows (host, one column, first sweep): the rows b reaches (sparse_rhs_rows),
// for the sparse Schur right-hand side; nullptr: the dense one.
static void solve_lrc(Launcher& L, const T* rhs, int max_iter, int check_every, bool pcgnr = false,
                      const int32_t* sp_rows = nullptr, int sp_nt = 0, int sp_ns = 0, int sp_np = 0) {
  DeviceIndex* D = L.D;
  Workspace* w = L.w;
  const int B = L.B;
  const int n = D->n, n1 = D->n1, n2 = D->n2;
  const T beta = (T)D->beta;
  hipStream_t st = L.st;
  ColState cs = L.cs(max_iter);
  T* X = (T*)w->X;      // rows < n1: block-solve output; rows >= n1: p2
  T* P2 = X + (int64_t)n1 * B;
  T* R2 = (T*)w->Y;     // n2 x B
  T* Q2 = (T*)w->W;     // n2 x B
  T* Z2 = (T*)w->Z;     // n2 x B
  T* Dx = (T*)w->Dx;
  T* K2 = Dx + (int64_t)n1 * B;

  auto m11 = [&](const T* v, T cv, const T* x2, T ca, T* out, const int* nact) {
    if (n1 == 0) return;
    M11Args<T> a;
    a.tile_row0 = D->tile_row0; a.row_blk = D->row_blk; a.blk_start = D->blk_start; a.blk_off = D->blk_off;
    a.minv = Factors<T>::minv(D); a.rp = D->rp; a.col = D->col; a.split = D->split; a.val = D->val; a.n1 = n1;
    a.v = v; a.cv = cv; a.x2 = x2; a.ca = ca; a.out = out; a.B = B; a.n_active = nact;
    a.xcd = tuning().xcd;
    a.tile_row1 = nullptr;
    // k_m11_apply for 2-15 columns: the finer tiles (more workgroups, fewer
    // sequential passes each); one column keeps the 256-row tiles (measured
    // faster there)
    const bool fine = B >= 2 && B < 16;
    if (fine) a.tile_row0 = D->ntile_row0;
    const int tile_rows = fine ? D->max_ntile_rows : D->max_tile_rows;
    int cb = std::max(1, std::min(B, (int)(32768 / sizeof(T) / std::max(1, tile_rows))));
    a.CB = cb;
    a.sub = cb >= 16 ? 1 : (cb >= 4 ? 2 : tuning().m11_sub1);
    size_t shm = (size_t)tile_rows * cb * sizeof(T);
    const double wb = (double)sizeof(T) * B;
    double bytes = (double)sizeof(T) * D->minv_elems + 4.0 * n1 + wb * n1 + (v ? wb * n1 : 0.0) +
                   (x2 ? 8.0 * n1 + 4.0 * D->nnz_a12 + wb * D->cols_a12 : 0.0);
    if (B >= tuning().m11_small_min) {
      if (B > 512) fail(KATZ_EINVAL, "batch too wide for one launch");
      // blocks of <= kSmallBlock rows in registers, a team of CW lanes per
      // block; larger ones by the tile kernel below (bytes split by row share)
      const int cw = B <= 8 ? 8 : (B <= 16 ? 16 : (B <= 32 ? 32 : 64));
      const Tuning& tu = tuning();
      M11SmallArgs<T> s;
      s.blk_start = D->blk_start; s.blk_off = D->blk_off; s.minv = a.minv;
      s.rp = D->rp; s.col = D->col; s.split = D->split; s.val = D->val;
      s.x = x2 ? x2 - (int64_t)n1 * B : nullptr;  // x2 is rows >= n1 of a full panel
      s.ca = (T)0; s.cb = (T)1; s.cu = ca; s.v = v; s.cv = cv; s.out = out;
      s.B = B; s.nblocks = D->nblocks; s.blocks_per_chunk = (WG / cw) * tu.m11_bpt; s.xcd = tu.xcd;
      s.ld = B; s.j0 = 0;
      s.nchunks = (D->nblocks + s.blocks_per_chunk - 1) / s.blocks_per_chunk;
      s.n_active = nact;
      const dim3 g((unsigned)std::min<int64_t>(tu.spmm_nwg, s.nchunks));
      const double fb = n1 > 0 ? (double)D->big_rows / n1 : 0.0;
      L.timed(PK_M11, bytes * (1.0 - fb), [&] {
        const bool wv = s.val != nullptr;
#define KZ_M11S(cw, ncm)                                                                    \
  if (wv) k_m11_small<T, cw, ncm, kSmallBlock, true><<<g, WG, 0, st>>>(s);                  \
  else k_m11_small<T, cw, ncm, kSmallBlock, false><<<g, WG, 0, st>>>(s);
        if (cw == 8) { KZ_M11S(8, 1) } else if (cw == 16) { KZ_M11S(16, 1) } else if (cw == 32) { KZ_M11S(32, 1) }
        else if (B <= 64) { KZ_M11S(64, 1) } else if (B <= 128) { KZ_M11S(64, 2) } else if (B <= 256) { KZ_M11S(64, 4) }
        else { KZ_M11S(64, 8) }
#undef KZ_M11S
      });
      if (D->n_big > 0) {
        a.tile_row0 = D->big_row0;
        a.tile_row1 = D->big_row1;
        const int cbw = B <= 16 ? 16 : ((B <= 32 || sizeof(T) == 8) ? 32 : 64);
        const size_t shm2 = (size_t)D->max_big_rows * cbw * sizeof(T);
        if (shm2 > 65536) fail(KATZ_EDEVICE, "internal: block too large for LDS");
        const dim3 gb((unsigned)D->n_big, (unsigned)((B + cbw - 1) / cbw));
        L.timed(PK_M11_BIG, bytes * fb, [&] {
          const bool wv = a.val != nullptr;
          if (cbw == 16) {
            if (wv) k_m11_cols<T, 16, true><<<gb, WG, shm2, st>>>(a); else k_m11_cols<T, 16, false><<<gb, WG, shm2, st>>>(a);
          } else if (cbw == 32) {
            if (wv) k_m11_cols<T, 32, true><<<gb, WG, shm2, st>>>(a); else k_m11_cols<T, 32, false><<<gb, WG, shm2, st>>>(a);
          } else {
            if (wv) k_m11_cols<T, 64, true><<<gb, WG, shm2, st>>>(a); else k_m11_cols<T, 64, false><<<gb, WG, shm2, st>>>(a);
          }
        });
      }
    } else if (B >= 16) {
      // column-chunked kernel: 64 KB of LDS per workgroup at most
      const int cbw = sizeof(T) == 8 ? (B <= 16 ? 16 : 32) : (B <= 16 ? 16 : (B <= 32 ? 32 : 64));
      const size_t shm2 = (size_t)D->max_tile_rows * cbw * sizeof(T);
      if (shm2 > 65536) fail(KATZ_EDEVICE, "internal: block tile too large for LDS");
      dim3 g((unsigned)D->ntiles, (unsigned)((B + cbw - 1) / cbw));
      L.timed(PK_M11, bytes, [&] {
        const bool wv = a.val != nullptr;
        if (cbw == 16) {
          if (wv) k_m11_cols<T, 16, true><<<g, WG, shm2, st>>>(a); else k_m11_cols<T, 16, false><<<g, WG, shm2, st>>>(a);
        } else if (cbw == 32) {
          if (wv) k_m11_cols<T, 32, true><<<g, WG, shm2, st>>>(a); else k_m11_cols<T, 32, false><<<g, WG, shm2, st>>>(a);
        } else {
          if (wv) k_m11_cols<T, 64, true><<<g, WG, shm2, st>>>(a); else k_m11_cols<T, 64, false><<<g, WG, shm2, st>>>(a);
        }
      });
    } else {
      L.timed(PK_M11, bytes, [&] { k_m11_apply<T><<<fine ? D->n_ntiles : D->ntiles, WG, shm, st>>>(a); });
    }
  };
  // z2 = G r2 + V (D o (V^T r2)), then <r2, z2> (EP_RZ_INIT / EP_RZ)
  auto precond = [&](int ep) {
    const int64_t m = n2;
    const int rpw = L.rows_per_wg(m), nwg = Launcher::nwg_for(m, rpw);
    const int* nact = ep == EP_RZ ? w->n_active : nullptr;
    if (std::is_same<T, float>::value && B >= 16 && D->rank > 0 && !D->ginv) {
      precond_mfma(L, (const float*)R2, (float*)Z2, ep, cs, nact);
      return;
    }
    L.need(nwg, (int64_t)std::max(1, D->rank) * B);
    with_lowrank_factor<T>(D, [&](auto* V) {
      typedef typename std::remove_cv<typename std::remove_pointer<decltype(V)>::type>::type TV;
      precond_simple<T, TV>(L, V, R2, Z2, ep, cs, nact, rpw, nwg);
    });
  };

  // z = S~^{-1} r2 and p2 = z + bcg p2 (init: p2 = z).  With L = I and a
  // rank of at most 64 (or none), precond_fused updates p2 without forming z;
  // otherwise z is formed (with <r2, z>) and p2 updated after.
  const bool fuse_p = !D->ginv && D->rank <= 64 && !(std::is_same<T, float>::value && B >= 16 && D->rank > 0);
  // Two or more columns: x += alpha p is taken by the search-direction
  // update (which reads the old p anyway) instead of the residual update, on
  // the columns whose step this iteration's S p set (w->fresh), so one panel
  // pass fewer per iteration; same values, same bits.
  const bool defer_x = B >= 2 && tuning().defer_x;
  T* xd = defer_x ? K2 : nullptr;
  auto precond_p = [&](int init) {
    T* xk = init ? nullptr : xd;
    if (!fuse_p) {
      precond(init ? EP_RZ_INIT : EP_RZ);
      L.timed_cols(PK_UPDATE_P, (xk ? 5.0 : 3.0) * sizeof(T) * n2, [&] {
        k_update_p<T><<<grid_for((int64_t)n2, 64), WG, 0, st>>>(n2, B, Z2, P2, init, cs, xk, w->fresh);
      });
      return;
    }
    const int* nact = init ? nullptr : w->n_active;
    if (D->rank == 0) {
      // z = r: <r, z> = <r, r>
      k_rz_lowrank<<<1, WG, 0, st>>>(0, B, nullptr, init, cs, nact);
      L.timed_cols(PK_UPDATE_P, (xk ? 5.0 : 3.0) * sizeof(T) * n2, [&] {
        k_update_p<T><<<grid_for((int64_t)n2, 64), WG, 0, st>>>(n2, B, R2, P2, init, cs, xk, w->fresh);
      });
      return;
    }
    with_lowrank_factor<T>(D, [&](auto* V) {
      typedef typename std::remove_cv<typename std::remove_pointer<decltype(V)>::type>::type TV;
      precond_fused<T, TV>(L, V, R2, P2, init, cs, nact, xk);
    });
  };

  {
    // chunk walk of the iteration's S p launch, tuned before any SpMM of the
    // solve so that every launch of this variant uses the same walk (Q2 is
    // first written by the iterations)
    SpmmArgs<T> a{};
    a.row0 = n1; a.row1 = n; a.rp = D->rp; a.col = D->col; a.split = D->split; a.val = D->val;
    a.x = X; a.ca = -beta; a.cb = -beta; a.parts = 3; a.y = Q2; a.cs = cs;
    L.tune_spmm(a);
  }
  size_lowrank_rows<T>(D, st);  // grid of the narrow low-rank kernels, before their first launch

  if (pcgnr) {
    // Ablation: the recurrence of Algorithm 2 as printed, with the step
    // gamma = s^T (S~^{-1} s) for s = S r (the printed y^T s matches neither
    // PCG nor PCGNR and diverges): preconditioned CG on the normal equations
    // S^2 k2 = S f, two S-applies per iteration, k2 starting at 0.
    if (w->external) fail(KATZ_EINVAL, "the PCGNR ablation is not available without allocation");
    if (!w->ab1) {
      w->ab1 = dalloc<char>(w->allocs, (int64_t)n * w->B * (int64_t)sizeof(T));
      w->ab2 = dalloc<char>(w->allocs, (int64_t)std::max(1, n2) * w->B * (int64_t)sizeof(T));
    }
    T* RF = (T*)w->ab1;            // rows < n1: block-solve output; rows >= n1: r
    T* Rn = RF + (int64_t)n1 * B;  // r = f - S k2 (n2 x B)
    T* S2 = (T*)w->ab2;            // s = S r
    // out2 = S in2 with in2 the separator rows of the full panel `full`
    auto sapply = [&](T* full, T* in2, T* out2, int ep, const int* nact) {
      m11(nullptr, (T)0, in2, beta, full, nact);   // t1 = M11^{-1} (beta A12 in2)
      SpmmArgs<T> a{};
      a.row0 = n1; a.row1 = n; a.rp = D->rp; a.col = D->col; a.split = D->split; a.val = D->val;
      a.x = full; a.ca = -beta; a.cb = -beta; a.parts = 3;
      a.v = in2; a.cv = (T)1; a.w = nullptr; a.cw = (T)0; a.y = out2;
      a.ep = ep; a.dotv = nullptr; a.cs = cs; a.n_active = nact;  // EP_PQ: <q, q>
      L.spmm(a);
    };
    auto precond_in = [&](const T* in, int ep, const int* nact) {  // Z2 = S~^{-1} in, <in, Z2>
      const int rpw = L.rows_per_wg(n2), nwg = Launcher::nwg_for(n2, rpw);
      L.need(nwg, (int64_t)std::max(1, D->rank) * B);
      with_lowrank_factor<T>(D, [&](auto* V) {
        typedef typename std::remove_cv<typename std::remove_pointer<decltype(V)>::type>::type TV;
        precond_simple<T, TV>(L, V, in, Z2, ep, cs, nact, rpw, nwg);
      });
    };
    m11(rhs, (T)1, nullptr, (T)0, X, nullptr);
    {
      SpmmArgs<T> a{};
      a.row0 = n1; a.row1 = n; a.rp = D->rp; a.col = D->col; a.split = D->split; a.val = D->val;
      a.x = X; a.ca = beta; a.cb = (T)0; a.parts = 1;
      a.v = rhs + (int64_t)n1 * B; a.cv = (T)1; a.w = nullptr; a.cw = (T)0; a.y = Rn;
      a.ep = EP_RR_INIT; a.dotv = nullptr; a.cs = cs; a.n_active = nullptr;
      L.spmm(a);   // r = f, <r, r>, the active columns
    }
    L.fill<T>(K2, (int64_t)n2 * B, (T)0);
    sapply(RF, Rn, S2, EP_NONE, nullptr);          // s = S r
    precond_in(S2, EP_RZ_INIT, nullptr);           // w = S~^{-1} s, gamma = <s, w>
    k_update_p<T><<<grid_for((int64_t)n2, 64), WG, 0, st>>>(n2, B, Z2, P2, 1, cs);  // p = w
    const int rpw2 = L.rows_per_wg(n2), nwg2 = Launcher::nwg_for(n2, rpw2);
    L.need(nwg2, B);
    L.iterate(sizeof(T) == 8 ? 5 : 6, max_iter, check_every, [&] {
      sapply(X, P2, Q2, EP_PQ, w->n_active);      // q = S p; alpha = gamma / <q, q>
      L.timed_cols(PK_UPDATE_R, 6.0 * sizeof(T) * n2, [&] {
        k_update_r<T><<<nwg2, WG, WG * sizeof(double), st>>>(n2, B, rpw2, K2, P2, Rn, Q2, cs, w->partials);
      });
      L.finalize(nwg2, B, EP_RR, cs, nullptr, w->n_active);   // k2 += alpha p, r -= alpha q
      sapply(RF, Rn, S2, EP_NONE, w->n_active);   // s = S r
      precond_in(S2, EP_RZ, w->n_active);         // w, gamma', ratio gamma' / gamma
      L.timed_cols(PK_UPDATE_P, 3.0 * sizeof(T) * n2, [&] {
        k_update_p<T><<<grid_for((int64_t)n2, 64), WG, 0, st>>>(n2, B, Z2, P2, 0, cs);  // p = w + ratio p
      });
    });
    m11(rhs, (T)1, K2, beta, Dx, nullptr);
    return;
  }

  // ---- a2: t = M11^{-1} b1 -> X[0:n1]; f = b2 + beta A21 t -> R2; rr
  if (sp_rows) {
    // one column, b = beta A e_q: only the listed rows are nonzero.  The
    // lists go to w->seg (free until the next two-stage reduction).
    int32_t* dl = (int32_t*)w->seg;
    const size_t len = (size_t)sp_nt + 2 * (size_t)sp_ns + 1 + 2 * (size_t)sp_np;
    HIPCHECK(hipMemcpyAsync(dl, sp_rows, sizeof(int32_t) * len, hipMemcpyHostToDevice, st));
    L.fill<T>(X, (int64_t)n1, (T)0);
    L.fill<T>(R2, (int64_t)n2, (T)0);
    const int32_t* off = dl + sp_nt + sp_ns;
    k_schur_rhs1<T><<<1, WG, 0, st>>>(dl, sp_nt, sp_ns, off, off + sp_ns + 1, off + sp_ns + 1 + sp_np, rhs, n1,
                                      D->row_blk, D->blk_start, D->blk_off, Factors<T>::minv(D), D->val, beta, X,
                                      R2, cs);
  } else {
  m11(rhs, (T)1, nullptr, (T)0, X, nullptr);
  {
    SpmmArgs<T> a{};
    a.row0 = n1; a.row1 = n; a.rp = D->rp; a.col = D->col; a.split = D->split; a.val = D->val;
    a.x = X; a.ca = beta; a.cb = (T)0; a.parts = 1;
    a.v = rhs + (int64_t)n1 * B; a.cv = (T)1; a.w = nullptr; a.cw = (T)0; a.y = R2;
    a.ep = EP_RR_INIT; a.dotv = nullptr; a.cs = cs; a.n_active = nullptr;
    L.spmm(a);
  }
  }
  // x2 (rows >= n1 of Dx) starts at 0; rows < n1 are written whole by the
  // back-solve (a4) before anything reads them
  L.fill<T>(K2, (int64_t)n2 * B, (T)0);
  precond_p(1);

  // ---- a3: PCG iterations, polled every check_every
  const int rpw2 = L.rows_per_wg(n2), nwg2 = Launcher::nwg_for(n2, rpw2);
  L.need(nwg2, B);
  const bool fuse_vt = B == 1 && D->rank > 0 && D->rank <= 64 && !D->ginv && fuse_p && tuning().fuse;
  if (defer_x) {
    L.fill<int>(w->fresh, (int64_t)B, 0);
    L.fresh_out = w->fresh;  // the iterations' S p finalizes flag their columns
  }
  L.iterate(sizeof(T) == 8 ? 1 : 2, max_iter, check_every, [&] {
      m11(nullptr, (T)0, P2, beta, X, w->n_active);   // t1' = M11^{-1} (beta A12 p2)
      SpmmArgs<T> a{};
      a.row0 = n1; a.row1 = n; a.rp = D->rp; a.col = D->col; a.split = D->split; a.val = D->val;
      a.x = X; a.ca = -beta; a.cb = -beta; a.parts = 3;
      a.v = P2; a.cv = (T)1; a.w = nullptr; a.cw = (T)0; a.y = Q2;       // q2 = S p2
      a.ep = EP_PQ; a.dotv = P2; a.cs = cs; a.n_active = w->n_active;
      L.spmm(a);
      if (fuse_vt) {
        // one column: update and V^T r in one pass, then p = r + V DW + bcg p
        with_lowrank_factor<T>(D, [&](auto* V) {
          typedef typename std::remove_cv<typename std::remove_pointer<decltype(V)>::type>::type TV;
          update_r_precond1<T, TV>(L, V, K2, P2, R2, Q2, cs);
        });
        return;
      }
      L.timed_cols(PK_UPDATE_R, (defer_x ? 3.0 : 6.0) * sizeof(T) * n2, [&] {
        k_update_r<T><<<nwg2, WG, WG * sizeof(double), st>>>(n2, B, rpw2, defer_x ? nullptr : K2, P2, R2, Q2, cs,
                                                             w->partials);
      });
      L.finalize(nwg2, B, EP_RR, cs, nullptr, w->n_active);
      precond_p(0);
      if (defer_x) L.fill<int>(w->fresh, (int64_t)B, 0);
  });
  L.fresh_out = nullptr;
  // ---- a4: k1 = M11^{-1} (b1 + beta A12 k2) -> Dx[0:n1]
  m11(rhs, (T)1, K2, beta, Dx, nullptr);
}

template <typename T>
static void solve_cg(Launcher& L, const T* rhs, int max_iter, int check_every) {
  DeviceIndex* D = L.D;
  Workspace* w = L.w;
  const int B = L.B, n = D->n;
  const T beta = (T)D->beta;
  hipStream_t st = L.st;
  ColState cs = L.cs(max_iter);
  T* P = (T*)w->X;
  T* R = (T*)w->Y;
  T* Q = (T*)w->W;
  T* Dx = (T*)w->Dx;
  const int64_t m = n;
  const int rpw = L.rows_per_wg(m), nwg = Launcher::nwg_for(m, rpw);
  L.need(nwg, B);
  {
    // chunk walk of the iteration's A p launch (Q is first written by the
    // iterations)
    SpmmArgs<T> a{};
    a.row0 = 0; a.row1 = n; a.rp = D->rp; a.col = D->col; a.split = D->split; a.val = D->val;
    a.x = P; a.ca = -beta; a.cb = -beta; a.parts = 3; a.y = Q; a.cs = cs;
    L.tune_spmm(a);
  }
  // r = rhs, x = 0, p = r, rz = rr = <r, r>
  k_axpy_mask<T, T><<<grid_for(m, 64), WG, 0, st>>>(m, B, R, rhs, nullptr, nullptr, 0);
  L.fill<T>(Dx, m * B, (T)0);
  L.colnorm2<T>(R, m, w->rr);
  k_cg_init<<<1, WG, 0, st>>>(B, cs);
  k_update_p<T><<<grid_for(m, 64), WG, 0, st>>>(m, B, R, P, 1, cs);
  L.iterate(sizeof(T) == 8 ? 3 : 4, max_iter, check_every, [&] {
      SpmmArgs<T> a{};
      a.row0 = 0; a.row1 = n; a.rp = D->rp; a.col = D->col; a.split = D->split; a.val = D->val;
      a.x = P; a.ca = -beta; a.cb = -beta; a.parts = 3;
      a.v = P; a.cv = (T)1; a.w = nullptr; a.cw = (T)0; a.y = Q;
      a.ep = EP_PQ; a.dotv = P; a.cs = cs; a.n_active = w->n_active;
      L.spmm(a);
      L.timed_cols(PK_UPDATE_R, 6.0 * sizeof(T) * m, [&] {
        k_update_r<T><<<nwg, WG, WG * sizeof(double), st>>>(m, B, rpw, Dx, P, R, Q, cs, w->partials);
      });
      L.finalize(nwg, B, EP_RR_CG, cs, nullptr, w->n_active);
      L.timed_cols(PK_UPDATE_P, 3.0 * sizeof(T) * m, [&] {
        k_update_p<T><<<grid_for(m, 64), WG, 0, st>>>(m, B, R, P, 0, cs);
      });
  });
}

// ============================================================ batch driver
void device_topk(int n, int B, int K, double* Kp, const int32_t* qpos, const int32_t* rp, const int32_t* col,
                 const int32_t* iperm, void* scratch, size_t scratch_bytes, int32_t* ids, double* scores,
                 hipStream_t st);

namespace {

bool is_device_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t at;
  hipError_t e = hipPointerGetAttributes(&at, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return at.type == hipMemoryTypeDevice;
}

struct ColResult {
  int iters = 0, sweeps = 0, path = KATZ_PATH_LRC, status = KATZ_OK;
  double rel = 0, bn = 0;
  bool done = false, fallback = false;
};

}  // namespace

// Solves one batch of B <= 512 queries; leaves K (permuted, FP64) in w->K.

static void run_batch(const HostIndex& H, DeviceIndex* D, Workspace* w, hipStream_t st, const int32_t* q,
                      int B, const katz_query_opts& o, std::vector<ColResult>& res) {
  Launcher L{D, w, st, B};
  const int n = D->n;
  const int64_t nB = (int64_t)n * B;
  char* pin = (char*)w->hpin;
  // a1: right-hand side b = beta A e_q in the permuted order
  int32_t* hq = (int32_t*)(pin + kPinQ);
  for (int j = 0; j < B; j++) hq[j] = H.perm[q[j]];
  HIPCHECK(hipMemcpyAsync(w->qpos, hq, sizeof(int32_t) * B, hipMemcpyHostToDevice, st));
  // b is sparse (deg(q) entries per column) and is written into Rhs
  // afresh where it is needed, instead of being kept as a dense panel
  auto put_b = [&] {
    L.fill<double>(w->Rhs, nB, 0.0);
    k_rhs_scatter<double><<<B, WG, 0, st>>>(w->qpos, B, D->rp, D->col, D->val, D->beta, w->Rhs);
  };
  put_b();
  // K is not cleared: the first sweep writes it whole (below)
  k_rhs_norm2<<<B, 64, 0, st>>>(w->qpos, B, D->rp, D->val, D->beta, w->bn2);
  // thresholds and the first sweep's mask on the device (no host round trip)
  const double tol = o.rel_tol;
  k_cols_setup<<<1, WG, 0, st>>>(B, w->bn2, 0.25 * tol * tol, w->thr, w->mask);
  res.assign(B, ColResult());
  for (int j = 0; j < B; j++) res[j].path = o.method == KATZ_METHOD_CG ? KATZ_PATH_CG : KATZ_PATH_LRC;
  // one column: the rows b reaches, for the first sweep's sparse Schur
  // right-hand side (a dense one when they are many)
  int32_t* sp_rows = nullptr;
  int sp_nt = 0, sp_ns = 0, sp_np = 0;
  if (B == 1 && o.method == KATZ_METHOD_LRC && tuning().sparse_rhs && D->n2 > 0 &&
      sparse_rhs_rows(H, hq[0], (int32_t*)(pin + kPinList), kPinListCap, sp_nt, sp_ns, sp_np))
    sp_rows = (int32_t*)(pin + kPinList);
  double* hb = (double*)(pin + kPinBn2);
  double* hres = (double*)(pin + kPinRes);
  bool have_bn = false;
  // Precision form, 16 columns and more: each sweep's residual is the last
  // one minus M d for the sweep's FP32 correction d (half the gathered bytes
  // of b - M K with K in FP64); <r, r> per column into res2.
  const bool rec_res = D->precision == KATZ_PREC_MIXED && B >= 16 && tuning().rec_res;
  auto residual_update_f32 = [&] {
    SpmmArgs<double, float> a{};
    a.row0 = 0; a.row1 = n; a.rp = D->rp; a.col = D->col; a.split = D->split; a.val = D->val;
    a.x = (const float*)w->Dx; a.ca = D->beta; a.cb = D->beta; a.parts = 3;
    a.v = w->Rhs; a.cv = 1.0; a.w = (const float*)w->Dx; a.cw = -1.0; a.y = w->Rhs;
    a.ep = EP_RES; a.dotv = nullptr; a.out = w->res2; a.n_active = nullptr; a.cs = L.cs(0);
    L.spmm(a);
  };
  for (int sweep = 0; sweep < o.max_sweeps; sweep++) {
    bool any = false;
    for (int j = 0; j < B; j++) any |= !res[j].done;
    if (!any) break;
    const double* rhs = w->Rhs;  // b in the first sweep, then the residual
    // each column takes one path per sweep, chosen before the sweep starts
    int ran[2] = {0, 0};
    for (int pass = 0; pass < 2; pass++) {
      // pass 0: columns on the LRC path; pass 1: plain CG (requested or fallback)
      const bool cg_pass = pass == 1;
      int* hm = (int*)(pin + (pass ? kPinMask1 : kPinMask0));
      int cnt = 0;
      for (int j = 0; j < B; j++) {
        const bool on_cg = o.method == KATZ_METHOD_CG || res[j].fallback || D->n2 == 0;
        hm[j] = (!res[j].done && on_cg == cg_pass) ? 1 : 0;
        cnt += hm[j];
      }
      if (!cnt) continue;
      ran[pass] = 1;
      // sweep 0: the device mask (b != 0) is already in place
      if (sweep > 0) HIPCHECK(hipMemcpyAsync(w->mask, hm, sizeof(int) * B, hipMemcpyHostToDevice, st));
      const int iters = (!cg_pass && o.force_fallback) ? 1 : o.max_iter;
      const int hslot = (cg_pass ? 4 : 0) + (D->precision == KATZ_PREC_MIXED ? 2 : 0) + (sweep > 0 ? 1 : 0);
      L.iter_hint = D->iter_hint[hslot].load(std::memory_order_relaxed);
      if (D->precision == KATZ_PREC_MIXED) {
        // FP32 inner solve on the unit-norm right-hand side, FP64 accumulation
        L.colnorm2<double>(rhs, n, w->rn2);
        k_mixed_scales<<<1, WG, 0, st>>>(B, w->rn2, w->bn2, tol, kInnerTolFP32, w->inv, w->fwd, w->thr);
        k_axpy_mask<float, double><<<grid_for(n, 64), WG, 0, st>>>(n, B, w->Rf, rhs, nullptr, w->inv, 0);
        if (cg_pass)
          solve_cg<float>(L, w->Rf, iters, o.check_every);
        else
          solve_lrc<float>(L, w->Rf, iters, o.check_every, o.method == KATZ_METHOD_PCGNR, sweep == 0 ? sp_rows : nullptr,
                           sp_nt, sp_ns, sp_np);
        // first sweep (one path for all columns): K = correction for every
        // column (those outside the mask are exactly 0: each solve clears Dx
        // and never touches inactive columns); later sweeps add
        if (rec_res) {
          // the correction as FP32 values (0 off the sweep's columns) into
          // K, then r -= M d with d gathered in FP32 and summed in FP64
          k_take_correction<<<grid_for(n, 64), WG, 0, st>>>(n, B, (float*)w->Dx, w->K, sweep == 0 ? nullptr : w->mask,
                                                             w->fwd, sweep == 0 ? 0 : 1);
          residual_update_f32();
        } else if (sweep == 0) {
          k_axpy_mask<double, float><<<grid_for(n, 64), WG, 0, st>>>(n, B, w->K, (const float*)w->Dx, nullptr,
                                                                    w->fwd, 0);
        } else {
          k_axpy_mask<double, float><<<grid_for(n, 64), WG, 0, st>>>(n, B, w->K, (const float*)w->Dx, w->mask,
                                                                    w->fwd, 1);
        }
      } else {
        if (cg_pass)
          solve_cg<double>(L, rhs, iters, o.check_every);
        else
          solve_lrc<double>(L, rhs, iters, o.check_every, o.method == KATZ_METHOD_PCGNR,
                            sweep == 0 ? sp_rows : nullptr, sp_nt, sp_ns, sp_np);
        if (sweep == 0)
          k_axpy_mask<double, double><<<grid_for(n, 64), WG, 0, st>>>(n, B, w->K, (const double*)w->Dx, nullptr,
                                                                      nullptr, 0);
        else
          k_axpy_mask<double, double><<<grid_for(n, 64), WG, 0, st>>>(n, B, w->K, (const double*)w->Dx, w->mask,
                                                                      nullptr, 1);
      }
      HIPCHECK(hipMemcpyAsync(pin + (pass ? kPinStat1 : kPinStat0), w->status, sizeof(int) * B,
                              hipMemcpyDeviceToHost, st));
      HIPCHECK(hipMemcpyAsync(pin + (pass ? kPinIter1 : kPinIter0), w->iters, sizeof(int) * B,
                              hipMemcpyDeviceToHost, st));
    }
    // a6: true FP64 residual r = b - M k, which is the next sweep's right-hand
    // side: Rhs = b, then Rhs = Rhs + beta A k - k in place (each element is
    // read and written by the same lane).  The first sweep's solve only read
    // Rhs, which still holds b.  (The precision form at 16 columns and more
    // has updated Rhs -= M d after each pass instead.)
    if (!rec_res) {
      if (sweep > 0) put_b();
      SpmmArgs<double> a{};
      a.row0 = 0; a.row1 = n; a.rp = D->rp; a.col = D->col; a.split = D->split; a.val = D->val;
      a.x = w->K; a.ca = D->beta; a.cb = D->beta; a.parts = 3;
      a.v = w->Rhs; a.cv = 1.0; a.w = w->K; a.cw = -1.0; a.y = w->Rhs;
      a.ep = EP_RES; a.dotv = nullptr; a.out = w->res2; a.n_active = nullptr; a.cs = L.cs(0);
      L.spmm(a);
    }
    HIPCHECK(hipMemcpyAsync(hres, w->res2, sizeof(double) * B, hipMemcpyDeviceToHost, st));
    if (!have_bn) HIPCHECK(hipMemcpyAsync(hb, w->bn2, sizeof(double) * B, hipMemcpyDeviceToHost, st));
    L.sync();  // one host round trip per sweep
    if (!have_bn) {
      for (int j = 0; j < B; j++) {
        res[j].bn = std::sqrt(hb[j]);
        if (hb[j] == 0.0) {  // isolated query node: k = 0 exactly
          res[j].done = true;
          res[j].rel = 0.0;
        }
      }
      have_bn = true;
    }
    for (int pass = 0; pass < 2; pass++) {
      if (!ran[pass]) continue;
      const int* hm = (const int*)(pin + (pass ? kPinMask1 : kPinMask0));
      const int* hs = (const int*)(pin + (pass ? kPinStat1 : kPinStat0));
      const int* hi = (const int*)(pin + (pass ? kPinIter1 : kPinIter0));
      // the iterations this solve needed: the first poll of the next one
      int most = 0;
      for (int j = 0; j < B; j++)
        if (hm[j] && res[j].bn != 0.0) most = std::max(most, hi[j]);
      if (most > 0) {
        const int hslot = (pass ? 4 : 0) + (D->precision == KATZ_PREC_MIXED ? 2 : 0) + (sweep > 0 ? 1 : 0);
        D->iter_hint[hslot].store(most, std::memory_order_relaxed);
      }
      for (int j = 0; j < B; j++) {
        if (!hm[j] || res[j].bn == 0.0) continue;
        res[j].iters += hi[j];
        if (pass == 0 && (hs[j] != 0 || o.force_fallback)) {
          res[j].fallback = true;  // breakdown or cap on the LRC path
          res[j].path = KATZ_PATH_CG_FALLBACK;
        }
      }
    }
    for (int j = 0; j < B; j++) {
      if (res[j].done) continue;
      res[j].sweeps++;
      res[j].rel = std::sqrt(hres[j]) / res[j].bn;
      if (res[j].rel <= tol) res[j].done = true;
    }
  }
  for (int j = 0; j < B; j++)
    if (!res[j].done) res[j].status = KATZ_ENOCONV;
}

int device_query(const HostIndex& H, DeviceIndex* D, const QueryArgs& qa) { return device_query_ws(H, D, qa, nullptr); }

std::recursive_mutex& hip_global_mu() {
  static std::recursive_mutex m;
  return m;
}

void copy_to_caller(void* dst, const void* src, size_t bytes) {
  std::lock_guard<std::recursive_mutex> lk(hip_global_mu());
  if (is_device_ptr(dst))
    HIPCHECK(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
  else
    std::memcpy(dst, src, bytes);
}

Workspace* ws_create(DeviceIndex* D, int cap) {
  HIPCHECK(hipSetDevice(D->device));
  return make_ws(D, cap).release();
}
void ws_destroy(DeviceIndex* D, Workspace* w) {
  if (!w) return;
  (void)hipSetDevice(D->device);
  free_ws(w);
  delete w;
}
int ws_capacity(const Workspace* w) { return w ? w->B : 0; }

int device_query_ws(const HostIndex& H, DeviceIndex* D, const QueryArgs& qa, Workspace* fixed) {
  HIPCHECK(hipSetDevice(D->device));
  hipStream_t st = (hipStream_t)qa.stream;
  const int n = D->n;
  const int BMAX = fixed ? std::min(512, fixed->B) : 512;
  bool dev_scores = is_device_ptr(qa.scores);
  bool dev_ids = is_device_ptr(qa.ids);
  if (qa.topk > 0 && qa.topk_scores && is_device_ptr(qa.topk_scores) != dev_ids)
    fail(KATZ_EINVAL, "ids and scores must both be host or both be device buffers");
  int rc = KATZ_OK;
  for (int c0 = 0; c0 < qa.nq; c0 += BMAX) {
    const int B = std::min(BMAX, qa.nq - c0);
    std::unique_ptr<WsLease> lease;
    Workspace* w = fixed;
    if (!w || w->B < B) {
      lease.reset(new WsLease(D, B));
      w = lease->w.get();
    }
    // work runs on the workspace's stream, ordered after the caller's stream
    {
      std::unique_lock<std::recursive_mutex> lk(hip_global_mu(), std::defer_lock);
      if (!st) lk.lock();  // the legacy stream
      HIPCHECK(hipEventRecord(w->ev_in, st));
      HIPCHECK(hipStreamWaitEvent(w->stream, w->ev_in, 0));
    }
    hipStream_t caller = st;
    st = w->stream;
    std::vector<ColResult> res;
    run_batch(H, D, w, st, qa.q + c0, B, qa.opts, res);
    if (qa.npairs > 0) {
      // the pairs whose column lies in this chunk (sorted by column)
      const int32_t* pc = qa.pair_col;
      const int64_t p0 = std::lower_bound(pc, pc + qa.npairs, c0) - pc;
      const int64_t p1 = std::lower_bound(pc, pc + qa.npairs, c0 + B) - pc;
      const int64_t np = p1 - p0;
      if (np > 0) {
        if (w->pr_cap < np) {
          // geometric growth, the old buffers freed: a run of calls with a
          // slowly growing pair count stays within twice the largest need
          const int64_t cap = std::max<int64_t>(np, w->pr_cap + w->pr_cap / 2);
          dregrow(w->allocs, w->pr_rows, cap);
          dregrow(w->allocs, w->pr_cols, cap);
          dregrow(w->allocs, w->pr_out, cap);
          w->pr_cap = cap;
        }
        std::vector<int32_t> cols(qa.pair_col + p0, qa.pair_col + p1);
        for (auto& x : cols) x -= c0;
        HIPCHECK(hipMemcpyAsync(w->pr_rows, qa.pair_row + p0, sizeof(int32_t) * np, hipMemcpyHostToDevice, st));
        HIPCHECK(hipMemcpyAsync(w->pr_cols, cols.data(), sizeof(int32_t) * np, hipMemcpyHostToDevice, st));
        k_pair_gather<<<(unsigned)((np + WG - 1) / WG), WG, 0, st>>>((int)np, B, w->K, w->pr_rows, w->pr_cols,
                                                                    w->pr_out);
        HIPCHECK(hipMemcpyAsync(qa.pair_out + p0, w->pr_out, sizeof(double) * np, hipMemcpyDefault, st));
        HIPCHECK(hipStreamSynchronize(st));  // `cols` is pageable host memory
      }
    }
    if (qa.scores) {
      double* dst = qa.scores + (int64_t)c0 * n;
      double* out = dst;
      if (!dev_scores) out = w->Rhs;  // free once the batch is solved
      if (B >= 32) {
        dim3 g((unsigned)((n + 63) / 64), (unsigned)((B + 63) / 64));
        k_unpermute_tiled<double><<<g, WG, 0, st>>>(n, B, w->K, D->perm, out);
      } else {
        dim3 g(grid_for(n, WG * 4), B);
        k_unpermute<double><<<g, WG, 0, st>>>(n, B, w->K, D->perm, out);
      }
      if (!dev_scores)
        HIPCHECK(hipMemcpyAsync(dst, out, sizeof(double) * (size_t)n * B, hipMemcpyDeviceToHost, st));
    }
    // top-K last: the selection overwrites q and its neighbours in K with -inf,
    // after the pair gather and the score output have read K
    if (qa.topk > 0) {
      const int K = qa.topk;
      size_t need = 64 * (size_t)B + 1024 * (size_t)B + 12 * (size_t)K * B + 1024;
      if (w->tk_cap < need) {
        const size_t cap = std::max(need, w->tk_cap + w->tk_cap / 2);
        dregrow(w->allocs, w->tk_scratch, (int64_t)cap);
        w->tk_cap = cap;
      }
      int32_t* ids = qa.ids + (int64_t)c0 * K;
      double* sc = qa.topk_scores ? qa.topk_scores + (int64_t)c0 * K : nullptr;
      int32_t* dids = ids;
      double* dsc = sc;
      if (!dev_ids) {
        if (w->tk_out_cap < (int64_t)K * B) {
          const int64_t cap = std::max<int64_t>((int64_t)K * B, w->tk_out_cap + w->tk_out_cap / 2);
          dregrow(w->allocs, w->tk_ids, cap);
          dregrow(w->allocs, w->tk_sc, cap);
          w->tk_out_cap = cap;
        }
        dids = w->tk_ids;
        dsc = sc ? w->tk_sc : nullptr;
      }
      device_topk(n, B, K, w->K, w->qpos, D->rp, D->col, D->iperm, w->tk_scratch, w->tk_cap, dids, dsc, st);
      if (!dev_ids) {
        HIPCHECK(hipMemcpyAsync(ids, dids, sizeof(int32_t) * (size_t)K * B, hipMemcpyDeviceToHost, st));
        if (sc) HIPCHECK(hipMemcpyAsync(sc, dsc, sizeof(double) * (size_t)K * B, hipMemcpyDeviceToHost, st));
      }
    }
    HIPCHECK(hipStreamSynchronize(st));
    w->prof.harvest();
    HIPCHECK(hipEventRecord(w->ev_out, st));
    {
      std::unique_lock<std::recursive_mutex> lk(hip_global_mu(), std::defer_lock);
      if (!caller) lk.lock();  // the legacy stream
      HIPCHECK(hipStreamWaitEvent(caller, w->ev_out, 0));
    }
    st = caller;
    HIPCHECK(hipGetLastError());
    for (int j = 0; j < B; j++) {
      if (res[j].status != KATZ_OK) rc = KATZ_ENOCONV;
      if (qa.st) {
        katz_query_stats& s = qa.st[c0 + j];
        s.status = res[j].status;
        s.iters = res[j].iters;
        s.sweeps = res[j].sweeps;
        s.path = res[j].path;
        s.rel_residual = res[j].rel;
        s.err_bound = res[j].rel * (1.0 + D->c) / (1.0 - D->c);
      }
    }
  }
  return rc;
}

// ------------------------------------------------ Sparse-Katz re-ranking
// Algorithm 3, last step, one workgroup per query i: with K_T the Katz scores
// K[v, t] of the query (row r = 0) and its nc listed candidates (rows
// r = 1..nc) at its T modular nodes t, rho_j is the Pearson correlation of
// rows 0 and j + 1 over t (undefined when either row is constant); the list
// is re-ordered by rho descending, undefined correlations last, equal ones in
// the Katz order.  kt[inv[base_i + t (nc + 1) + r]] holds K_T[r][t].  Means
// and sums run in t order; the order is a bitonic sort in LDS.
constexpr int kRerankMax = 4096;
__device__ inline bool rerank_before(double ka, int32_t pa, double kb, int32_t pb) {
  const bool fa = ka == ka, fb = kb == kb;
  if (fa != fb) return fa;
  if (fa && ka != kb) return ka > kb;
  return pa < pb;
}
__global__ __launch_bounds__(WG) void k_sparse_rerank(const double* kt, const int32_t* inv, const int64_t* base,
                                                      const int32_t* ncand, const int32_t* nmod, const int32_t* cand,
                                                      int s, int32_t* ids, double* corr) {
  __shared__ double key[kRerankMax];
  __shared__ int32_t pos[kRerankMax];
  __shared__ double qs[2];
  const int i = blockIdx.x, tid = threadIdx.x;
  const int nc = ncand[i], T = nmod[i];
  const int64_t b0 = base[i];
  const double nan = __longlong_as_double(0x7ff8000000000000LL);
  if (tid == 0) {
    double mq = 0.0, sq = 0.0;
    if (T >= 2) {
      for (int t = 0; t < T; t++) mq += kt[inv[b0 + (int64_t)t * (nc + 1)]];
      mq /= T;
      for (int t = 0; t < T; t++) {
        const double d = kt[inv[b0 + (int64_t)t * (nc + 1)]] - mq;
        sq = __fma_rn(d, d, sq);
      }
    }
    qs[0] = mq;
    qs[1] = sq;
  }
  __syncthreads();
  int P = 1;
  while (P < nc) P <<= 1;
  for (int j = tid; j < P; j += WG) {
    double rho = nan;
    if (j < nc && T >= 2) {
      double mj = 0.0;
      for (int t = 0; t < T; t++) mj += kt[inv[b0 + (int64_t)t * (nc + 1) + 1 + j]];
      mj /= T;
      double sj = 0.0, cj = 0.0;
      for (int t = 0; t < T; t++) {
        const double dq = kt[inv[b0 + (int64_t)t * (nc + 1)]] - qs[0];
        const double dj = kt[inv[b0 + (int64_t)t * (nc + 1) + 1 + j]] - mj;
        sj = __fma_rn(dj, dj, sj);
        cj = __fma_rn(dq, dj, cj);
      }
      if (qs[1] > 0.0 && sj > 0.0) rho = cj / sqrt(qs[1] * sj);
    }
    key[j] = rho;
    pos[j] = j;  // padding (j >= nc) is undefined and sorts after every candidate
  }
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1) {
    for (int h = k >> 1; h > 0; h >>= 1) {
      for (int a = tid; a < P; a += WG) {
        const int b = a ^ h;
        if (b > a) {
          const bool up = (a & k) == 0;  // this pair's run ascends in the order
          const bool swap = up ? rerank_before(key[b], pos[b], key[a], pos[a])
                               : rerank_before(key[a], pos[a], key[b], pos[b]);
          if (swap) {
            const double tk = key[a]; key[a] = key[b]; key[b] = tk;
            const int32_t tp = pos[a]; pos[a] = pos[b]; pos[b] = tp;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int p = tid; p < s; p += WG) {
    const bool in = p < nc;
    ids[(int64_t)i * s + p] = in ? cand[(int64_t)i * s + pos[p]] : -1;
    corr[(int64_t)i * s + p] = in ? key[p] : nan;
  }
}

// Bump allocation over [base, base + cap) at 256-byte alignment; with
// base == nullptr it only counts.
struct Carve {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(int64_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? (T*)(base + off) : nullptr;
    off += (size_t)std::max<int64_t>(count, 1) * sizeof(T);
    return p;
  }
};

// A device buffer of at least `bytes` from the index's reusable pool (the
// smallest free one that fits, else a new one); give it back with aux_give.
static std::pair<void*, size_t> aux_take(DeviceIndex* D, size_t bytes) {
  {
    std::lock_guard<std::mutex> g(D->aux_mu);
    int best = -1;
    for (size_t i = 0; i < D->aux_free.size(); i++)
      if (D->aux_free[i].second >= bytes && (best < 0 || D->aux_free[i].second < D->aux_free[best].second))
        best = (int)i;
    if (best >= 0) {
      auto r = D->aux_free[best];
      D->aux_free.erase(D->aux_free.begin() + best);
      return r;
    }
  }
  std::lock_guard<std::recursive_mutex> lk(hip_global_mu());
  void* p = nullptr;
  const hipError_t e = hipMalloc(&p, std::max<size_t>(bytes, 256));
  if (e != hipSuccess) fail(e == hipErrorOutOfMemory ? KATZ_ENOMEM : KATZ_EDEVICE, std::string("hipMalloc: ") + hipGetErrorString(e));
  return {p, std::max<size_t>(bytes, 256)};
}
static void aux_give(DeviceIndex* D, std::pair<void*, size_t> b) {
  std::lock_guard<std::mutex> g(D->aux_mu);
  if (D->aux_free.size() >= 4) {
    // keep the pool small: drop the smallest buffer
    size_t small = 0;
    for (size_t i = 1; i < D->aux_free.size(); i++)
      if (D->aux_free[i].second < D->aux_free[small].second) small = i;
    if (D->aux_free[small].second < b.second) {
      std::lock_guard<std::recursive_mutex> lk(hip_global_mu());
      (void)hipFree(D->aux_free[small].first);
      D->aux_free[small] = b;
      return;
    }
    std::lock_guard<std::recursive_mutex> lk(hip_global_mu());
    (void)hipFree(b.first);
    return;
  }
  D->aux_free.push_back(b);
}

// Solves the modular nodes' Katz vectors (the distinct sources q_src, as one
// batched query with pair gathers K[row, q_src[col]] into a device buffer),
// then re-ranks on the device (k_sparse_rerank) and copies the lists to the
// caller.  The buffers come from the index's reusable pool.  Returns the
// status of the solves; pst receives their stats.
int device_sparse_katz(const HostIndex& H, DeviceIndex* D, const katz_query_opts& opts, void* stream,
                       const std::vector<int32_t>& q_src, const std::vector<int32_t>& pcol,
                       const std::vector<int32_t>& prow, const std::vector<int32_t>& inv,
                       const std::vector<int64_t>& base, const std::vector<int32_t>& ncand,
                       const std::vector<int32_t>& nmod, const std::vector<int32_t>& cand, int nq, int s,
                       katz_query_stats* pst, int32_t* ids, double* corr) {
  if (s > kRerankMax) fail(KATZ_EINVAL, "Sparse-Katz list longer than 4096");
  HIPCHECK(hipSetDevice(D->device));
  const int64_t np = (int64_t)pcol.size();
  // one buffer: K_T entries, their positions, per-request sizes, candidates, outputs
  Carve lay{nullptr};
  lay.take<double>(np);
  lay.take<int32_t>(np);
  lay.take<int64_t>(nq);
  lay.take<int32_t>(nq);
  lay.take<int32_t>(nq);
  lay.take<int32_t>((int64_t)nq * s);
  lay.take<int32_t>((int64_t)nq * s);
  lay.take<double>((int64_t)nq * s);
  hipStream_t st = (hipStream_t)stream;
  auto buf = aux_take(D, lay.off);
  // back to the pool once the stream is idle (also when a step below throws
  // with work still queued, so that no other call reuses it in flight)
  struct Give {
    DeviceIndex* D;
    std::pair<void*, size_t> b;
    hipStream_t st;
    ~Give() {
      (void)hipStreamSynchronize(st);
      aux_give(D, b);
    }
  } give{D, buf, st};
  Carve c{(char*)buf.first};
  double* kt = c.take<double>(np);
  int32_t* d_inv = c.take<int32_t>(np);
  int64_t* d_base = c.take<int64_t>(nq);
  int32_t* d_nc = c.take<int32_t>(nq);
  int32_t* d_nm = c.take<int32_t>(nq);
  int32_t* d_cand = c.take<int32_t>((int64_t)nq * s);
  int32_t* d_ids = c.take<int32_t>((int64_t)nq * s);
  double* d_corr = c.take<double>((int64_t)nq * s);
  int rc = KATZ_OK;
  if (np > 0) {
    QueryArgs a{};
    a.q = q_src.data(); a.nq = (int32_t)q_src.size(); a.opts = opts; a.scores = nullptr; a.topk = 0;
    a.st = pst; a.stream = stream;
    a.npairs = (int32_t)np; a.pair_col = pcol.data(); a.pair_row = prow.data(); a.pair_out = kt;
    rc = device_query(H, D, a);
  }
  auto up = [&](void* d, const void* h, size_t bytes) {
    if (bytes) HIPCHECK(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, st));
  };
  up(d_inv, inv.data(), sizeof(int32_t) * inv.size());
  up(d_base, base.data(), sizeof(int64_t) * base.size());
  up(d_nc, ncand.data(), sizeof(int32_t) * ncand.size());
  up(d_nm, nmod.data(), sizeof(int32_t) * nmod.size());
  up(d_cand, cand.data(), sizeof(int32_t) * cand.size());
  k_sparse_rerank<<<nq, WG, 0, st>>>(kt, d_inv, d_base, d_nc, d_nm, d_cand, s, d_ids, d_corr);
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipMemcpyAsync(ids, d_ids, sizeof(int32_t) * (size_t)nq * s, hipMemcpyDefault, st));
  if (corr) HIPCHECK(hipMemcpyAsync(corr, d_corr, sizeof(double) * (size_t)nq * s, hipMemcpyDefault, st));
  HIPCHECK(hipStreamSynchronize(st));
  return rc;
}

// ------------------------------------------------ queries without allocation
// Scratch of katz_query_noalloc: panels, partial sums and per-column state
// of the solve live in this file-scope device array (one copy on every GPU
// the library runs on, held until the process ends).  Host code never passes
// `scratch` itself to a kernel or copy: its name is a host-side stand-in, and
// the device address is taken once per device with hipGetSymbolAddress.
constexpr size_t kScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

constexpr size_t kNoAllocHostBytes = 64 * 1024;  // host staging, as the pinned staging of a workspace

struct NoAllocSlot {
  void* dev = nullptr;                 // device address of `scratch` on this device
  std::unique_ptr<char[]> host;        // host staging for query ids, masks and polled scalars
};

// Set-up, once per device and with that device current: the device address
// of the scratch array and the host staging.  Later calls only look up.
NoAllocSlot& noalloc_slot(int device) {
  static std::mutex mu;
  static std::map<int, NoAllocSlot> slots;
  std::lock_guard<std::mutex> g(mu);
  NoAllocSlot& sl = slots[device];
  if (!sl.dev) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      fail(KATZ_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    sl.host.reset(new char[kNoAllocHostBytes]);
    sl.dev = p;
  }
  return sl;
}

// Lays a B-column workspace (the buffers run_batch uses: panels, partial
// sums, low-rank terms, per-column scalars and state) over `base`; returns
// the bytes it takes.  Top-K and pair buffers are not laid out.
size_t carve_ws(const DeviceIndex* D, int B, char* base, Workspace* w) {
  Carve c{base};
  const int64_t nB = (int64_t)D->n * B;
  const int64_t esz = solve_elem_bytes(D);
  const int64_t rk = std::max(1, D->rank);
  double* Rhs = c.take<double>(nB);
  double* K = c.take<double>(nB);
  char* Dx = c.take<char>(nB * esz);
  char* X = c.take<char>(nB * esz);
  char* Y = c.take<char>(nB * esz);
  char* W = c.take<char>(nB * esz);
  char* Z = c.take<char>((int64_t)std::max(1, D->n2) * B * esz);
  const size_t pcap = std::max(partials_per_column(D) * (size_t)std::max(B, 1), spmm_partials_need(D, std::max(B, 1)));
  double* partials = c.take<double>((int64_t)pcap);
  double* seg = c.take<double>((int64_t)seg_values(D, std::max(B, 1)));
  double* DW = c.take<double>(rk * B);
  double* DW2 = c.take<double>(rk * B);
  double* sc = c.take<double>(12 * (int64_t)B);
  float* Rf = D->precision == KATZ_PREC_MIXED ? c.take<float>(nB) : nullptr;
  int* ip = c.take<int>(5 * (int64_t)B + 1);
  int32_t* qpos = c.take<int32_t>(B);
  if (w) {
    w->B = B; w->n = D->n; w->n2 = D->n2; w->device = D->device;
    w->Rhs = Rhs; w->K = K; w->Dx = Dx; w->X = X; w->Y = Y; w->W = W; w->Z = Z;
    w->partials = partials; w->partials_cap = pcap; w->seg = seg; w->DW = DW; w->DW2 = DW2;
    w->rz = sc; w->pq = sc + B; w->alpha = sc + 2 * B; w->bcg = sc + 3 * B; w->rr = sc + 4 * B;
    w->thr = sc + 5 * B; w->bn2 = sc + 6 * B; w->res2 = sc + 7 * B; w->colscale = sc + 8 * B;
    w->rn2 = sc + 9 * B; w->inv = sc + 10 * B; w->fwd = sc + 11 * B;
    w->Rf = Rf;
    w->active = ip; w->status = ip + B; w->iters = ip + 2 * B; w->mask = ip + 3 * B; w->n_active = ip + 4 * B;
    w->fresh = ip + 4 * B + 1;
    w->qpos = qpos;
  }
  return c.off;
}

}  // namespace

int device_query_noalloc(const HostIndex& H, DeviceIndex* D, const QueryArgs& qa) {
  if (qa.opts.method == KATZ_METHOD_PCGNR)
    fail(KATZ_EINVAL, "the PCGNR ablation is not available without allocation");
  HIPCHECK(hipSetDevice(D->device));
  NoAllocSlot& sl = noalloc_slot(D->device);
  // columns that fit: the layout is affine in B
  const size_t one = carve_ws(D, 1, nullptr, nullptr), two = carve_ws(D, 2, nullptr, nullptr);
  const size_t per = two - one, fixed = one - per;
  if (one > kScratchBytes)
    fail(KATZ_EINVAL, "index too large for the allocation-free query: one query column needs " +
                          std::to_string(one) + " bytes of scratch, the scratch holds " +
                          std::to_string(kScratchBytes));
  const int cap = (int)std::min<size_t>(512, (kScratchBytes - fixed) / per);
  hipStream_t st = (hipStream_t)qa.stream;
  const int n = D->n;
  const bool dev_scores = qa.scores && is_device_ptr(qa.scores);
  int rc = KATZ_OK;
  for (int c0 = 0; c0 < qa.nq; c0 += cap) {
    const int B = std::min(cap, qa.nq - c0);
    Workspace w;
    w.external = true;
    const size_t used = carve_ws(D, B, (char*)sl.dev, &w);
    if (used > kScratchBytes) fail(KATZ_EDEVICE, "internal: scratch layout exceeds the scratch");
    w.hpin = sl.host.get();
    // state that starts at zero (per-column scalars and flags), cleared by a
    // fill kernel on the caller's stream: the previous call's contents remain
    Launcher L0{D, &w, st, B};
    L0.fill<double>(w.rz, 12 * (int64_t)B, 0.0);
    L0.fill<int>(w.active, 5 * (int64_t)B + 1, 0);
    std::vector<ColResult> res;
    run_batch(H, D, &w, st, qa.q + c0, B, qa.opts, res);
    if (qa.scores) {
      double* dst = qa.scores + (int64_t)c0 * n;
      double* out = dev_scores ? dst : w.Rhs;  // Rhs is free once the batch is solved
      if (B >= 32) {
        dim3 g((unsigned)((n + 63) / 64), (unsigned)((B + 63) / 64));
        k_unpermute_tiled<double><<<g, WG, 0, st>>>(n, B, w.K, D->perm, out);
      } else {
        dim3 g(grid_for(n, WG * 4), B);
        k_unpermute<double><<<g, WG, 0, st>>>(n, B, w.K, D->perm, out);
      }
      if (!dev_scores)
        HIPCHECK(hipMemcpyAsync(dst, out, sizeof(double) * (size_t)n * B, hipMemcpyDeviceToHost, st));
    }
    HIPCHECK(hipStreamSynchronize(st));
    HIPCHECK(hipGetLastError());
    for (int j = 0; j < B; j++) {
      if (res[j].status != KATZ_OK) rc = KATZ_ENOCONV;
      if (qa.st) {
        katz_query_stats& s2 = qa.st[c0 + j];
        s2.status = res[j].status;
        s2.iters = res[j].iters;
        s2.sweeps = res[j].sweeps;
        s2.path = res[j].path;
        s2.rel_residual = res[j].rel;
        s2.err_bound = res[j].rel * (1.0 + D->c) / (1.0 - D->c);
      }
    }
  }
  return rc;
}

// ------------------------------------------------ Lanczos on R (device)
// The top eigenpairs of R = I - S (L = I) by Lanczos with full
// reorthogonalisation, as the host index build computes them (Algorithm 1,
// Lanczos step), with the basis Q (column-major n2 x m, FP64) in HBM.

// partials[blockIdx.x * nv + k] = sum over the chunk's rows i of Q[k][i] w[i]
// for k in the workgroup's tile of kQT vectors (blockIdx.y).
constexpr int kQT = 16;
__global__ __launch_bounds__(WG) void k_qtw(int64_t m, int nv, const double* Q, const double* w, int64_t rpc,
                                            double* partials) {
  __shared__ double sh[(WG / 64) * kQT];
  const int tid = threadIdx.x, k0 = blockIdx.y * kQT;
  const int64_t r0 = (int64_t)blockIdx.x * rpc, r1 = min<int64_t>(m, r0 + rpc);
  double acc[kQT];
#pragma unroll
  for (int t = 0; t < kQT; t++) acc[t] = 0.0;
  for (int64_t i = r0 + tid; i < r1; i += WG) {
    // unconditional loads (vectors past nv repeat the last; their sums are
    // never used), in flight together
    double qv[kQT];
#pragma unroll
    for (int t = 0; t < kQT; t++) qv[t] = Q[(int64_t)(k0 + t < nv ? k0 + t : nv - 1) * m + i];
    const double x = w[i];
#pragma unroll
    for (int t = 0; t < kQT; t++) acc[t] += qv[t] * x;
  }
  const int wave = tid / 64, lane = tid % 64;
#pragma unroll
  for (int t = 0; t < kQT; t++) {
    double v = acc[t];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) sh[wave * kQT + t] = v;
  }
  __syncthreads();
  if (tid < kQT && k0 + tid < nv) {
    double s = 0.0;
    for (int wv = 0; wv < WG / 64; wv++) s += sh[wv * kQT + tid];
    partials[(int64_t)blockIdx.x * nv + k0 + tid] = s;
  }
}

// w[i] -= sum_k Q[k][i] h[k], k < nv (h staged in LDS, nv <= kMaxBasis).
constexpr int kMaxBasis = 4096;
constexpr int kMaxRitzSteps = 512;  // k_ritz stages kQT x steps doubles in 64 KB of LDS
__global__ __launch_bounds__(WG) void k_sub_qh(int64_t m, int nv, const double* Q, const double* h, double* w) {
  __shared__ double hs[kMaxBasis];
  for (int k = threadIdx.x; k < nv; k += WG) hs[k] = h[k];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (i >= m) return;
  double s = 0.0;
  for (int k = 0; k < nv; k++) s += Q[(int64_t)k * m + i] * hs[k];
  w[i] -= s;
}

// dst[i] = a * src[i]
__global__ void k_scale(int64_t m, double a, const double* src, double* dst) {
  const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (i < m) dst[i] = a * src[i];
}

// U[i][t] (row-major m x r) = sum_k Q[k][i] Z[t * mm + k] for the tile of
// kQT Ritz vectors t (blockIdx.y); Z staged in LDS.
__global__ __launch_bounds__(WG) void k_ritz(int64_t m, int mm, int r, const double* Q, const double* Z, double* U) {
  extern __shared__ double zs[];  // kQT x mm
  const int t0 = blockIdx.y * kQT;
  for (int e = threadIdx.x; e < kQT * mm; e += WG) {
    const int t = e / mm, k = e % mm;
    zs[e] = t0 + t < r ? Z[(int64_t)(t0 + t) * mm + k] : 0.0;
  }
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (i >= m) return;
  double acc[kQT];
#pragma unroll
  for (int t = 0; t < kQT; t++) acc[t] = 0.0;
  for (int k = 0; k < mm; k++) {
    const double q = Q[(int64_t)k * m + i];
#pragma unroll
    for (int t = 0; t < kQT; t++) acc[t] += q * zs[t * mm + k];
  }
#pragma unroll
  for (int t = 0; t < kQT; t++)
    if (t0 + t < r) U[i * r + t0 + t] = acc[t];
}

// ------------------------------------------------ lambda_max (device)
// The vector work of the Lanczos iteration for lambda_max(A) on the caller's
// CSR (original order), for large graphs at index build.  Every sum is
// taken in a fixed order: kLamWG workgroups over contiguous row ranges, each
// reduced by a fixed tree, the per-workgroup values summed on the host in
// order.
constexpr int kLamWG = 2048;
constexpr int kLamTS = 8;  // lanes per row of the product

// y = A x (kLamTS lanes per row) and partials[bid] = sum over the
// workgroup's rows of x_i y_i.
__global__ __launch_bounds__(WG) void k_lam_spmv(int32_t n, int64_t rows_per_wg, const int32_t* rp,
                                                 const int32_t* col, const double* val, const double* x,
                                                 double* y, double* partials) {
  __shared__ double sh[WG / 64];
  const int tid = threadIdx.x, lane = tid % kLamTS, team = tid / kLamTS;
  constexpr int TEAMS = WG / kLamTS;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg, r1 = min<int64_t>(n, r0 + rows_per_wg);
  double acc = 0.0;
  for (int64_t i = r0 + team; i < r1; i += TEAMS) {
    double s = 0.0;
    for (int32_t k = rp[i] + lane; k < rp[i + 1]; k += kLamTS) s += (val ? val[k] : 1.0) * x[col[k]];
#pragma unroll
    for (int off = 1; off < kLamTS; off <<= 1) s += __shfl_xor(s, off, kLamTS);
    if (lane == 0) {
      y[i] = s;
      acc += x[i] * s;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (tid % 64 == 0) sh[tid / 64] = acc;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int wv = 0; wv < WG / 64; wv++) t += sh[wv];
    partials[blockIdx.x] = t;
  }
}

// w -= a q + b qp and partials[bid] = sum over the workgroup's rows of w_i^2.
__global__ __launch_bounds__(WG) void k_lam_update(int32_t n, int64_t rows_per_wg, double a, double b,
                                                   const double* q, const double* qp, double* w,
                                                   double* partials) {
  __shared__ double sh[WG / 64];
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg, r1 = min<int64_t>(n, r0 + rows_per_wg);
  double acc = 0.0;
  for (int64_t i = r0 + tid; i < r1; i += WG) {
    const double v = w[i] - (a * q[i] + b * qp[i]);
    w[i] = v;
    acc += v * v;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (tid % 64 == 0) sh[tid / 64] = acc;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int wv = 0; wv < WG / 64; wv++) t += sh[wv];
    partials[blockIdx.x] = t;
  }
}

// q = w / bj
__global__ __launch_bounds__(WG) void k_lam_scale(int32_t n, double bj, const double* w, double* q) {
  for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * WG) q[i] = w[i] / bj;
}

namespace {
struct DeviceLambdaOps : LambdaOps {
  int32_t n;
  int64_t rpw;
  const int32_t *rp, *col;
  const double* val;
  double *q, *qp, *w, *part;
  double* hpart;
  hipStream_t st;
  double host_sum() {
    HIPCHECK(hipMemcpyAsync(hpart, part, sizeof(double) * kLamWG, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    double s = 0.0;
    for (int b = 0; b < kLamWG; b++) s += hpart[b];
    return s;
  }
  void start(const double* q0) override {
    HIPCHECK(hipMemcpyAsync(q, q0, sizeof(double) * n, hipMemcpyHostToDevice, st));
    k_fill<double><<<grid_for(n, WG * 4), WG, 0, st>>>(qp, (int64_t)n, 0.0);
    HIPCHECK(hipStreamSynchronize(st));  // q0 is the caller's host memory
  }
  double apply_dot() override {
    k_lam_spmv<<<kLamWG, WG, 0, st>>>(n, rpw, rp, col, val, q, w, part);
    return host_sum();
  }
  double update_norm2(double a, double bprev) override {
    k_lam_update<<<kLamWG, WG, 0, st>>>(n, rpw, a, bprev, q, qp, w, part);
    return host_sum();
  }
  void advance(double bj) override {
    std::swap(q, qp);  // the previous vector; q = w / bj
    k_lam_scale<<<grid_for(n, WG * 4), WG, 0, st>>>(n, bj, w, q);
  }
};
}  // namespace

double device_lambda_max(int device, int32_t n, int64_t nnz, const int32_t* rp, const int32_t* col,
                         const double* val, uint64_t seed) {
  std::lock_guard<std::recursive_mutex> lk(hip_global_mu());
  HIPCHECK(hipSetDevice(device));
  std::vector<void*> tmp;
  hipStream_t st = nullptr;
  double* hpart = nullptr;
  struct Freer {
    std::vector<void*>& v;
    hipStream_t& st;
    double*& h;
    ~Freer() {
      for (void* p : v) (void)hipFree(p);
      if (h) (void)hipHostFree(h);
      if (st) (void)hipStreamDestroy(st);
    }
  } freer{tmp, st, hpart};
  HIPCHECK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  HIPCHECK(hipHostMalloc((void**)&hpart, sizeof(double) * kLamWG, hipHostMallocDefault));
  DeviceLambdaOps ops;
  ops.n = n;
  ops.rpw = ((int64_t)n + kLamWG - 1) / kLamWG;
  ops.st = st;
  ops.hpart = hpart;
  int32_t* drp = dalloc<int32_t>(tmp, (int64_t)n + 1);
  int32_t* dcol = dalloc<int32_t>(tmp, nnz);
  double* dval = val ? dalloc<double>(tmp, nnz) : nullptr;
  HIPCHECK(hipMemcpyAsync(drp, rp, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyHostToDevice, st));
  HIPCHECK(hipMemcpyAsync(dcol, col, sizeof(int32_t) * (size_t)nnz, hipMemcpyHostToDevice, st));
  if (val) HIPCHECK(hipMemcpyAsync(dval, val, sizeof(double) * (size_t)nnz, hipMemcpyHostToDevice, st));
  ops.rp = drp;
  ops.col = dcol;
  ops.val = dval;
  ops.q = dalloc<double>(tmp, n);
  ops.qp = dalloc<double>(tmp, n);
  ops.w = dalloc<double>(tmp, n);
  ops.part = dalloc<double>(tmp, kLamWG);
  const double lam = lambda_max_with(n, seed, ops);
  HIPCHECK(hipStreamSynchronize(st));
  HIPCHECK(hipGetLastError());
  return lam;
}

void device_lanczos_R(HostIndex& H, DeviceIndex* D) {
  auto t0 = std::chrono::steady_clock::now();
  HIPCHECK(hipSetDevice(D->device));
  const int32_t m2 = H.n2, n1 = H.n1, n = H.n;
  const int32_t r = std::min(H.lanczos_rank, m2);
  if (r <= 0 || H.l_kind != KATZ_L_IDENTITY) fail(KATZ_EDEVICE, "internal: device Lanczos needs L = I and r > 0");
  int32_t m = H.lanczos_steps_req > 0 ? H.lanczos_steps_req : std::max(2 * r, r + 20);
  m = std::min(m, m2);
  if (m > kMaxRitzSteps) fail(KATZ_EINVAL, "more than 512 Lanczos steps run on the host");
  std::unique_ptr<Workspace> wsp = make_ws(D, 1);
  Workspace* w = wsp.get();
  hipStream_t st = w->stream;
  Launcher L{D, w, st, 1};
  std::vector<void*> tmp;
  struct Freer {
    std::vector<void*>& v;
    ~Freer() {
      std::lock_guard<std::recursive_mutex> lk(hip_global_mu());
      for (void* p : v) (void)hipFree(p);
    }
  } freer{tmp};
  double* Q = dalloc<double>(tmp, (int64_t)m * m2);
  double* wv = dalloc<double>(tmp, m2);
  const int64_t rpc = std::max<int64_t>(WG * 4, (m2 + 1023) / 1024);
  const int nchunk = (int)((m2 + rpc - 1) / rpc);
  double* part = dalloc<double>(tmp, (int64_t)nchunk * kMaxBasis);
  double* hv = dalloc<double>(tmp, kMaxBasis);
  // rows < n1: t1 = M11^{-1} (beta A12 q); rows >= n1: q (its own FP64 buffer:
  // the workspace panels are FP32 for the precision form)
  double* X = dalloc<double>(tmp, n);
  std::vector<double> hh(kMaxBasis);
  const unsigned g1 = (unsigned)((m2 + WG - 1) / WG);

  // h[0..nv) = Q[:, 0..nv)^T x (device), and a copy on the host
  auto qtx = [&](const double* Qb, int nv, const double* x) {
    dim3 g((unsigned)nchunk, (unsigned)((nv + kQT - 1) / kQT));
    k_qtw<<<g, WG, 0, st>>>(m2, nv, Qb, x, rpc, part);
    k_vt_reduce<<<(unsigned)((nv + 63) / 64), WG, 0, st>>>(part, nchunk, nv, 1, nullptr, hv, nullptr);
    HIPCHECK(hipMemcpyAsync(hh.data(), hv, sizeof(double) * nv, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
  };
  auto norm = [&](const double* x) {
    qtx(x, 1, x);
    return std::sqrt(hh[0]);
  };
  // q_j <- random, orthogonal to q_0..q_{j-1} (two passes), unit norm
  uint64_t rs = H.lanczos_seed;
  std::vector<double> hq(m2);
  auto random_start = [&](int j) {
    lanczos_normals(rs, hq.data(), m2);
    double* qj = Q + (int64_t)j * m2;
    HIPCHECK(hipMemcpyAsync(qj, hq.data(), sizeof(double) * m2, hipMemcpyHostToDevice, st));
    for (int pass = 0; pass < 2 && j > 0; pass++) {
      qtx(Q, j, qj);
      k_sub_qh<<<g1, WG, 0, st>>>(m2, j, Q, hv, qj);
    }
    const double nn = norm(qj);
    k_scale<<<g1, WG, 0, st>>>(m2, 1.0 / nn, qj, qj);
  };
  // y = R q = beta (A21 t1 + A22 q), t1 = M11^{-1} (beta A12 q)
  auto applyR = [&](const double* q, double* y) {
    HIPCHECK(hipMemcpyAsync(X + n1, q, sizeof(double) * m2, hipMemcpyDeviceToDevice, st));
    if (n1 > 0) {
      M11Args<double> a;
      a.tile_row0 = D->tile_row0; a.row_blk = D->row_blk; a.blk_start = D->blk_start; a.blk_off = D->blk_off;
      a.minv = D->minv; a.rp = D->rp; a.col = D->col; a.split = D->split; a.val = D->val; a.n1 = n1;
      a.v = nullptr; a.cv = 0.0; a.x2 = X + n1; a.ca = D->beta; a.out = X; a.B = 1; a.n_active = nullptr;
      a.xcd = 0;
      a.CB = 1;
      a.sub = 4;
      a.tile_row1 = nullptr;
      const size_t shm = (size_t)D->max_tile_rows * sizeof(double);
      k_m11_apply<double><<<D->ntiles, WG, shm, st>>>(a);
    }
    SpmmArgs<double> s{};
    s.row0 = n1; s.row1 = n; s.rp = D->rp; s.col = D->col; s.split = D->split; s.val = D->val;
    s.x = X; s.ca = D->beta; s.cb = D->beta; s.parts = 3;
    s.v = nullptr; s.cv = 0.0; s.w = nullptr; s.cw = 0.0; s.y = y;
    s.ep = EP_NONE; s.dotv = nullptr; s.cs = L.cs(0); s.n_active = nullptr;
    L.spmm(s);
  };

  std::vector<double> al, be;
  random_start(0);
  double tnorm = 0.0;
  for (int j = 0; j < m; j++) {
    const double* qj = Q + (int64_t)j * m2;
    applyR(qj, wv);
    qtx(qj, 1, wv);
    const double a = hh[0];
    al.push_back(a);
    tnorm = std::max(tnorm, std::fabs(a));
    for (int pass = 0; pass < 2; pass++) {  // full reorthogonalisation
      qtx(Q, j + 1, wv);
      k_sub_qh<<<g1, WG, 0, st>>>(m2, j + 1, Q, hv, wv);
    }
    const double b = norm(wv);
    if (j + 1 == m) {
      be.push_back(b);
      break;
    }
    if (b <= 1e-12 * std::max(tnorm, 1e-300)) {
      be.push_back(0.0);  // invariant subspace: T decouples, restart
      random_start(j + 1);
    } else {
      be.push_back(b);
      k_scale<<<g1, WG, 0, st>>>(m2, 1.0 / b, wv, Q + (int64_t)(j + 1) * m2);
    }
    tnorm = std::max(tnorm, b);
  }
  const int32_t mm = (int32_t)al.size();
  const std::vector<double> z = lanczos_ritz(H, al, be, r);
  double* Zd = dalloc<double>(tmp, (int64_t)mm * r);
  double* Ud = dalloc<double>(tmp, (int64_t)m2 * r);
  HIPCHECK(hipMemcpyAsync(Zd, z.data(), sizeof(double) * z.size(), hipMemcpyHostToDevice, st));
  {
    dim3 g(g1, (unsigned)((r + kQT - 1) / kQT));
    const size_t shm = sizeof(double) * kQT * mm;
    if (shm > 65536) fail(KATZ_EINVAL, "lanczos_steps too large for the device Ritz step");
    k_ritz<<<g, WG, shm, st>>>(m2, mm, r, Q, Zd, Ud);
  }
  H.U.resize((size_t)m2 * r);
  HIPCHECK(hipMemcpyAsync(H.U.data(), Ud, sizeof(double) * H.U.size(), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
  HIPCHECK(hipGetLastError());
  H.V = H.U;  // L = I
  {
    std::lock_guard<std::recursive_mutex> lk(hip_global_mu());
    upload_factors(H, D);
    HIPCHECK(hipDeviceSynchronize());
  }
  H.phase_seconds[10] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  H.build_seconds += H.phase_seconds[10];
}

int profile_enable(int on) { return g_prof_on.exchange(on ? 1 : 0); }
void profile_reset() {
  std::lock_guard<std::mutex> g(g_prof.mu);
  for (int k = 0; k < PK_COUNT; k++) { g_prof.launches[k] = 0; g_prof.ms[k] = 0; g_prof.bytes[k] = 0; }
}
int profile_read(katz_kernel_stat* out, int max) {
  std::lock_guard<std::mutex> g(g_prof.mu);
  int c = 0;
  for (int k = 0; k < PK_COUNT && c < max; k++) {
    std::memset(&out[c], 0, sizeof(out[c]));
    std::strncpy(out[c].name, kProfNames[k], sizeof(out[c].name) - 1);
    out[c].launches = g_prof.launches[k];
    out[c].total_ms = g_prof.ms[k];
    out[c].alg_bytes = g_prof.bytes[k];
    c++;
  }
  return c;
}

}  // namespace katz
