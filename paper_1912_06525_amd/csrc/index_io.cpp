// Index files: the host index (the offline part of the method, Sec. 3.2
// steps 1-4 / Algorithm 1) written once and loaded by later processes that
// only run queries (Algorithm 2).
//
// Layout (little-endian): magic "KATZIDX\0", u32 version, u32 byte-order tag
// 0x01020304, the scalar fields in a fixed order, then every array as a u64
// element count followed by the raw elements.  A loaded index is validated
// in full before it is used: the device kernels index memory with its
// arrays, so every structural invariant they rely on is checked here.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "katz_internal.h"

namespace katz {
namespace {

constexpr char kMagic[8] = {'K', 'A', 'T', 'Z', 'I', 'D', 'X', '\0'};
constexpr uint32_t kVersion = 1;
constexpr uint32_t kOrderTag = 0x01020304u;
constexpr int kMaxBlockRows = 256;  // the block kernels' tile limit

struct File {
  FILE* f = nullptr;
  std::string path;
  File(const char* p, const char* mode) : path(p) {
    f = std::fopen(p, mode);
    if (!f) fail(KATZ_EIO, "cannot open " + path);
  }
  ~File() {
    if (f) std::fclose(f);
  }
  void write(const void* p, size_t bytes) {
    if (bytes && std::fwrite(p, 1, bytes, f) != bytes) fail(KATZ_EIO, "write failed: " + path);
  }
  void read(void* p, size_t bytes) {
    if (bytes && std::fread(p, 1, bytes, f) != bytes) fail(KATZ_EIO, "truncated or unreadable file: " + path);
  }
  void close() {
    if (f && std::fclose(f) != 0) {
      f = nullptr;
      fail(KATZ_EIO, "close failed: " + path);
    }
    f = nullptr;
  }
};

template <typename T>
void put(File& o, const T& v) { o.write(&v, sizeof(T)); }
template <typename T>
void put_vec(File& o, const std::vector<T>& v) {
  const uint64_t n = v.size();
  put(o, n);
  o.write(v.data(), n * sizeof(T));
}
template <typename T>
void get(File& in, T& v) { in.read(&v, sizeof(T)); }
template <typename T>
void get_vec(File& in, std::vector<T>& v, uint64_t max_count) {
  uint64_t n = 0;
  get(in, n);
  if (n > max_count) fail(KATZ_EINVAL, "index file: array larger than its header allows");
  v.resize(n);
  in.read(v.data(), n * sizeof(T));
}

void bad(const char* what) { fail(KATZ_EINVAL, std::string("index file: ") + what); }

// Every invariant of the host index that the device path relies on.
void validate_index(const HostIndex& H) {
  const int64_t n = H.n;
  if (n <= 0 || H.n1 < 0 || H.n2 < 0 || (int64_t)H.n1 + H.n2 != n) bad("node counts");
  if (H.nnz < 0 || H.nnz >= INT32_MAX) bad("entry count");
  if (!(H.beta > 0) || !(H.lambda_max >= 0) || !(H.c >= 0 && H.c < 1) || !std::isfinite(H.beta)) bad("beta");
  if ((int64_t)H.rp.size() != n + 1 || (int64_t)H.col.size() != H.nnz || (int64_t)H.split.size() != n)
    bad("CSR sizes");
  if (H.weighted ? (int64_t)H.val.size() != H.nnz : !H.val.empty()) bad("value array size");
  // row pointers non-decreasing from 0 to nnz (all of them before any row's
  // entries are read: a pointer past the entries with a smaller one after it
  // would otherwise be followed first)
  if (H.rp[0] != 0 || H.rp[n] != H.nnz) bad("row pointers");
  for (int64_t i = 0; i < n; i++)
    if (H.rp[i + 1] < H.rp[i]) bad("row pointers");
  for (int64_t i = 0; i < n; i++) {
    const int32_t s = H.rp[i], e = H.rp[i + 1];
    if (H.split[i] < s || H.split[i] > e) bad("split points");
    for (int32_t k = s; k < e; k++) {
      const int32_t c = H.col[k];
      if (c < 0 || c >= n || c == i) bad("column index");
      if (k > s && H.col[k - 1] >= c) bad("row not strictly increasing");
      if ((k < H.split[i]) != (c < H.n1)) bad("split point does not separate block and separator columns");
      if (H.weighted && !(H.val[k] >= 0 && std::isfinite(H.val[k]))) bad("weights");
    }
  }
  // symmetry: every (i, c) has its (c, i)
  for (int64_t i = 0; i < n; i++)
    for (int32_t k = H.rp[i]; k < H.rp[i + 1]; k++) {
      const int32_t c = H.col[k];
      const int32_t* b = H.col.data() + H.rp[c];
      const int32_t* e = H.col.data() + H.rp[c + 1];
      const int32_t* f = std::lower_bound(b, e, (int32_t)i);
      if (f == e || *f != i) bad("adjacency is not symmetric");
      if (H.weighted && H.val[f - H.col.data()] != H.val[k]) bad("weights are not symmetric");
    }
  if ((int64_t)H.perm.size() != n || (int64_t)H.iperm.size() != n) bad("permutation sizes");
  for (int64_t v = 0; v < n; v++) {
    const int32_t p = H.perm[v];
    if (p < 0 || p >= n || H.iperm[p] != v) bad("permutation");
  }
  // blocks: contiguous, at most kMaxBlockRows rows, covering [0, n1), no
  // entries between different blocks, inverses of b x b each
  // (block sizes first, so every block lies in [0, n1) before its rows are read)
  const size_t nb1 = H.blk_start.size();
  if (nb1 < 1 || H.blk_start[0] != 0 || H.blk_start[nb1 - 1] != H.n1) bad("block starts");
  if (H.blk_off.size() != nb1 || H.blk_off[0] != 0) bad("block offsets");
  for (size_t b = 0; b + 1 < nb1; b++) {
    const int64_t sz = (int64_t)H.blk_start[b + 1] - H.blk_start[b];
    if (sz < 1 || sz > kMaxBlockRows) bad("block size");
  }
  for (size_t b = 0; b + 1 < nb1; b++) {
    const int64_t sz = (int64_t)H.blk_start[b + 1] - H.blk_start[b];
    if (H.blk_off[b + 1] - H.blk_off[b] != sz * sz) bad("block offsets");
    for (int32_t i = H.blk_start[b]; i < H.blk_start[b + 1]; i++)
      for (int32_t k = H.rp[i]; k < H.split[i]; k++)
        if (H.col[k] < H.blk_start[b] || H.col[k] >= H.blk_start[b + 1]) bad("M11 is not block diagonal");
  }
  if ((int64_t)H.minv.size() != H.blk_off[nb1 - 1]) bad("block inverse size");
  for (double x : H.minv)
    if (!std::isfinite(x)) bad("block inverse values");
  const int64_t n2 = H.n2;
  if (H.l_kind == KATZ_L_CHOL || H.l_kind == KATZ_L_IC0) {
    if ((int64_t)H.ginv.size() != n2 * n2 || (int64_t)H.lchol.size() != n2 * n2) bad("M22 factor size");
  } else if (H.l_kind == KATZ_L_IDENTITY) {
    if (!H.ginv.empty() || !H.lchol.empty()) bad("M22 factor present with L = I");
  } else {
    bad("factor kind");
  }
  if (H.rank < 0 || H.rank > std::max<int64_t>(n2, 0)) bad("rank");
  const int64_t nr = n2 * H.rank;
  if ((int64_t)H.U.size() != nr || (int64_t)H.V.size() != nr || (int64_t)H.sigma.size() != H.rank ||
      (int64_t)H.D.size() != H.rank)
    bad("low-rank factor sizes");
  for (int32_t k = 0; k < H.rank; k++)
    if (!(H.sigma[k] < 1) || !std::isfinite(H.D[k])) bad("Ritz values");
  if (H.precision != KATZ_PREC_FP64 && H.precision != KATZ_PREC_MIXED) bad("precision");
  if (H.u_precision < 1 || H.u_precision > 3) bad("low-rank storage precision");
}

}  // namespace

void save_host_index(const HostIndex& H, const char* path) {
  File o(path, "wb");
  o.write(kMagic, sizeof(kMagic));
  put(o, kVersion);
  put(o, kOrderTag);
  put(o, H.n); put(o, H.n1); put(o, H.n2); put(o, H.nnz);
  put(o, H.beta); put(o, H.lambda_max); put(o, H.c);
  const int32_t w = H.weighted ? 1 : 0;
  put(o, w);
  put(o, H.l_kind); put(o, H.rank); put(o, H.sigma_next); put(o, H.lanczos_steps);
  put(o, H.precision); put(o, H.u_precision); put(o, H.build_seconds);
  put_vec(o, H.perm); put_vec(o, H.iperm);
  put_vec(o, H.rp); put_vec(o, H.col); put_vec(o, H.split); put_vec(o, H.val);
  put_vec(o, H.blk_start); put_vec(o, H.blk_off); put_vec(o, H.minv);
  put_vec(o, H.ginv); put_vec(o, H.lchol);
  put_vec(o, H.U); put_vec(o, H.V); put_vec(o, H.sigma); put_vec(o, H.D);
  o.close();
}

void load_host_index(const char* path, HostIndex& H) {
  File in(path, "rb");
  char magic[8];
  in.read(magic, sizeof(magic));
  if (std::memcmp(magic, kMagic, sizeof(kMagic)) != 0) bad("not a Katz index file");
  uint32_t ver = 0, tag = 0;
  get(in, ver);
  get(in, tag);
  if (tag != kOrderTag) bad("byte order differs from this host");
  if (ver != kVersion) bad("unsupported version");
  get(in, H.n); get(in, H.n1); get(in, H.n2); get(in, H.nnz);
  get(in, H.beta); get(in, H.lambda_max); get(in, H.c);
  int32_t w = 0;
  get(in, w);
  H.weighted = w != 0;
  get(in, H.l_kind); get(in, H.rank); get(in, H.sigma_next); get(in, H.lanczos_steps);
  get(in, H.precision); get(in, H.u_precision); get(in, H.build_seconds);
  if (H.n <= 0 || H.n2 < 0 || H.n2 > H.n || H.nnz < 0 || H.nnz >= INT32_MAX || H.rank < 0 || H.rank > H.n2)
    bad("header sizes");
  const uint64_t n = (uint64_t)H.n, nnz = (uint64_t)H.nnz, n2 = (uint64_t)H.n2, r = (uint64_t)H.rank;
  get_vec(in, H.perm, n); get_vec(in, H.iperm, n);
  get_vec(in, H.rp, n + 1); get_vec(in, H.col, nnz); get_vec(in, H.split, n); get_vec(in, H.val, nnz);
  get_vec(in, H.blk_start, n + 1); get_vec(in, H.blk_off, n + 1);
  get_vec(in, H.minv, (uint64_t)kMaxBlockRows * n);
  get_vec(in, H.ginv, n2 * n2); get_vec(in, H.lchol, n2 * n2);
  get_vec(in, H.U, n2 * r); get_vec(in, H.V, n2 * r); get_vec(in, H.sigma, r); get_vec(in, H.D, r);
  char extra;
  if (std::fread(&extra, 1, 1, in.f) != 0) bad("trailing bytes");
  validate_index(H);
}

}  // namespace katz
