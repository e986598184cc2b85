// Region tree, level lattice keys and prolongations on the device
// (arXiv 2505.09064, Section 3.1.1 Steps 1-4, Section 3.1.2, Section 3.2).
//
// The same tree decisions, keys, weights and CSR structure as the host build
// (setup.cpp), bit for bit:
//
//  * Tree. A vertex's path down the region tree does not depend on the node
//    counts: at every node it goes to the upper child along an axis iff its
//    coordinate is >= the node's midline m + (M - m) * ((lo + half) * 2^-47).
//    The counts only decide where the path stops: at the first node holding at
//    most `capacity` vertices. The build is level-synchronous. The vertices
//    still in nodes that split stay grouped by node; a round marks the groups of
//    at most `capacity` vertices as leaves and moves the others one level down,
//    re-grouped by a 32-bit radix sort on (group rank * 2^d + child index).
//  * Packed lattice keys. All region corners of a tree of depth D lie on the
//    lattice of side 2^(48-D) key units, so a key packs into one 64-bit word:
//    (k_z >> s) << 2B | (k_y >> s) << B | (k_x >> s), B = D bits per axis,
//    s = 48 - D. Integer order of packed keys is the canonical (z, y, x) order.
//    Trees deeper than 21 levels in 3D (32 in 2D) do not pack: the host
//    builds those.
//  * Level-1 regions (the non-empty leaves), the fine-to-level-1 prolongation
//    (multilinear interpolation in the leaf), and the merges of Section 3.1.2
//    (deepest regions into their parents; a next-level vertex is injected,
//    any other interpolated in its merged parent): radix sorts, unique passes
//    and binary searches over packed keys. Each prolongation is assembled from
//    (row, key, weight) triplets, 2^d slots per row, zero weights dropped,
//    columns the ranks of the distinct keys, ascending within a row.
//
// Compiled without floating-point contraction: midlines and weights follow the
// host's operations one by one.
#include <hip/hip_runtime.h>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/device/device_select.hpp>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "hierarchy.hpp"
#include "vasmg.h"

namespace vasmg {
namespace tree {

constexpr int kThreads = 256;
constexpr int kKeyBits = 48;             // depth-48 nodes have side 1 key unit
constexpr double kKeyScale = 0x1p-47;    // key K -> m + (M - m) * K * 2^-47

void check(hipError_t e, const char* what) {
  if (e != hipSuccess)
    throw Error{VASMG_EDEVICE, std::string("device tree build: ") + what + ": " + hipGetErrorString(e)};
}

unsigned grid_for(int64_t n) {
  return static_cast<unsigned>((std::max<int64_t>(n, 1) + kThreads - 1) / kThreads);
}

// Device memory of one build, ordered on its stream, released with the arena.
class Arena {
 public:
  explicit Arena(hipStream_t st) : st_(st) {}
  ~Arena() {
    for (void* p : owned_) (void)hipFreeAsync(p, st_);
  }
  Arena(const Arena&) = delete;
  Arena& operator=(const Arena&) = delete;
  template <typename T>
  T* get(int64_t n) {
    void* p = nullptr;
    check(hipMallocAsync(&p, static_cast<size_t>(std::max<int64_t>(n, 1)) * sizeof(T), st_),
          "allocation");
    owned_.push_back(p);
    return static_cast<T*>(p);
  }
  // temporary storage of the library primitives (grows, never shrinks)
  void* temp(size_t bytes) {
    if (bytes > temp_bytes_) {
      temp_ = get<unsigned char>(static_cast<int64_t>(bytes));
      temp_bytes_ = bytes;
    }
    return temp_;
  }
  hipStream_t stream() const { return st_; }
  template <typename T>
  T fetch(const T* p) {   // one value back to the host (synchronises the stream)
    T v{};
    check(hipMemcpyAsync(&v, p, sizeof(T), hipMemcpyDeviceToHost, st_), "copy");
    check(hipStreamSynchronize(st_), "synchronise");
    return v;
  }

 private:
  hipStream_t st_;
  std::vector<void*> owned_;
  void* temp_ = nullptr;
  size_t temp_bytes_ = 0;
};

// ---- library primitives (rocPRIM), on the arena's stream
template <typename K, typename V>
void sort_pairs(Arena& A, const K* kin, K* kout, const V* vin, V* vout, int64_t n, int bits) {
  if (n <= 0) return;
  bits = std::max(bits, 1);
  size_t bytes = 0;
  check(rocprim::radix_sort_pairs(nullptr, bytes, kin, kout, vin, vout, n, 0u, unsigned(bits),
                                  A.stream()), "sort");
  void* t = A.temp(bytes);
  check(rocprim::radix_sort_pairs(t, bytes, kin, kout, vin, vout, n, 0u, unsigned(bits), A.stream()),
        "sort");
}

template <typename K>
void sort_keys(Arena& A, const K* kin, K* kout, int64_t n, int bits) {
  if (n <= 0) return;
  bits = std::max(bits, 1);
  size_t bytes = 0;
  check(rocprim::radix_sort_keys(nullptr, bytes, kin, kout, n, 0u, unsigned(bits), A.stream()), "sort");
  void* t = A.temp(bytes);
  check(rocprim::radix_sort_keys(t, bytes, kin, kout, n, 0u, unsigned(bits), A.stream()), "sort");
}

// out = the entries of in whose flag is set (order kept); returns their count
template <typename T>
int64_t select_flagged(Arena& A, const T* in, const uint8_t* flags, T* out, int64_t n, int64_t* d_count) {
  if (n <= 0) return 0;
  size_t bytes = 0;
  check(rocprim::select(nullptr, bytes, in, flags, out, d_count, static_cast<size_t>(n), A.stream()),
        "select");
  void* t = A.temp(bytes);
  check(rocprim::select(t, bytes, in, flags, out, d_count, static_cast<size_t>(n), A.stream()), "select");
  return A.fetch(d_count);
}

// out = the first of each run of equal entries of the sorted in; returns their count
template <typename T>
int64_t unique_sorted(Arena& A, const T* in, T* out, int64_t n, int64_t* d_count) {
  if (n <= 0) return 0;
  size_t bytes = 0;
  check(rocprim::unique(nullptr, bytes, in, out, d_count, static_cast<size_t>(n), rocprim::equal_to<T>(),
                        A.stream()), "unique");
  void* t = A.temp(bytes);
  check(rocprim::unique(t, bytes, in, out, d_count, static_cast<size_t>(n), rocprim::equal_to<T>(),
                        A.stream()), "unique");
  return A.fetch(d_count);
}

template <typename T>
void inclusive_sum(Arena& A, const T* in, T* out, int64_t n) {
  if (n <= 0) return;
  size_t bytes = 0;
  check(rocprim::inclusive_scan(nullptr, bytes, in, out, static_cast<size_t>(n), rocprim::plus<T>(),
                                A.stream()), "scan");
  void* t = A.temp(bytes);
  check(rocprim::inclusive_scan(t, bytes, in, out, static_cast<size_t>(n), rocprim::plus<T>(), A.stream()),
        "scan");
}

// ---- packed lattice keys
__host__ __device__ inline uint64_t axis_of(uint64_t k, int a, int B) {
  return (k >> (a * B)) & ((uint64_t(1) << B) - 1);
}
// each axis rounded down to a multiple of q (a power of two)
template <int D>
__device__ inline uint64_t round_down(uint64_t k, uint64_t q, int B) {
  uint64_t r = 0;
#pragma unroll
  for (int a = 0; a < D; ++a) r |= (axis_of(k, a, B) & ~(q - 1)) << (a * B);
  return r;
}
template <typename K>
__device__ inline int64_t lower_bound(const K* v, int64_t n, K x) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (v[mid] < x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// ---- tree rounds
__global__ void k_iota(int64_t n, int32_t* v) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (i < n) v[i] = static_cast<int32_t>(i);
}

// head[i] = 1 where a group of equal keys starts
template <typename K>
__global__ void k_heads(int64_t n, const K* key, int32_t* head) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (i < n) head[i] = (i == 0 || key[i] != key[i - 1]) ? 1 : 0;
}

// start[g] = first position of group g (groups numbered by the inclusive scan of
// the heads, from 1); start[number of groups] = n
__global__ void k_group_starts(int64_t n, const int32_t* head, const int32_t* gid, int32_t* start) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (i >= n) return;
  if (head[i]) start[gid[i] - 1] = static_cast<int32_t>(i);
  if (i == n - 1) start[gid[i]] = static_cast<int32_t>(n);
}

// One round at `depth`: a vertex whose node holds at most cap vertices stays
// there (a leaf: its depth recorded, lo no longer changes); any other moves to
// its child (the host's midline comparison) and gets key (group << d) | child.
template <int D>
__global__ void k_split(int64_t n, int depth, int cap, int max_depth, double m, double S,
                        const double* __restrict__ xt, const int32_t* __restrict__ act,
                        const int32_t* __restrict__ gid, const int32_t* __restrict__ start,
                        uint64_t* __restrict__ lo, int32_t* __restrict__ leaf_depth,
                        uint8_t* __restrict__ keep, uint32_t* __restrict__ nkey, int* __restrict__ too_deep) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (i >= n) return;
  const int32_t t = act[i];
  const int32_t g = gid[i] - 1;
  const int32_t cnt = start[g + 1] - start[g];
  if (cnt <= cap) {
    leaf_depth[t] = depth;
    keep[i] = 0;
    return;
  }
  if (depth + 1 > max_depth) {   // deeper than packed keys allow: the host builds this tree
    *too_deep = 1;
    keep[i] = 0;
    return;
  }
  const uint64_t half = uint64_t(1) << (kKeyBits - depth - 1);
  uint32_t c = 0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const uint64_t l = lo[int64_t(t) * 3 + a];
    const double mid = m + S * (static_cast<double>(l + half) * kKeyScale);
    if (xt[int64_t(t) * D + a] >= mid) {
      c |= 1u << a;
      lo[int64_t(t) * 3 + a] = l + half;
    }
  }
  keep[i] = 1;
  nkey[i] = (static_cast<uint32_t>(g) << D) | c;
}

// Leaf regions: (depth, packed lo) per tree vertex.
template <int D>
__global__ void k_leaf_regions(int64_t n, const int32_t* __restrict__ leaf_depth,
                               const uint64_t* __restrict__ lo, int B, uint32_t* __restrict__ rd,
                               uint64_t* __restrict__ rk) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (t >= n) return;
  const int s = kKeyBits - B;
  uint64_t k = 0;
#pragma unroll
  for (int a = 0; a < D; ++a) k |= (lo[t * 3 + a] >> s) << (a * B);
  rd[t] = static_cast<uint32_t>(leaf_depth[t]);
  rk[t] = k;
}

__global__ void k_region_heads(int64_t n, const uint32_t* rd, const uint64_t* rk, uint8_t* head) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (i < n) head[i] = (i == 0 || rd[i] != rd[i - 1] || rk[i] != rk[i - 1]) ? 1 : 0;
}

// ---- prolongation triplets (2^d slots per row; weight 0 = no entry)
// Fine level -> level 1: multilinear interpolation in the vertex's leaf.
template <int D>
__global__ void k_fine_triplets(int64_t nf, const int32_t* __restrict__ ftp,
                                const int32_t* __restrict__ leaf_depth, const uint64_t* __restrict__ lo,
                                const double* __restrict__ xt, double m, double S, int B,
                                uint64_t* __restrict__ tk, double* __restrict__ tw) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (i >= nf) return;
  const int32_t t = ftp[i];
  const int dep = leaf_depth[t];
  const uint64_t s = uint64_t(1) << (kKeyBits - dep);
  const int sh = kKeyBits - B;
  double tup[D], tdn[D];
  uint64_t l[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    l[a] = lo[int64_t(t) * 3 + a];
    const double lc = m + S * (static_cast<double>(l[a]) * kKeyScale);
    const double hc = m + S * (static_cast<double>(l[a] + s) * kKeyScale);
    const double x = xt[int64_t(t) * D + a];
    tup[a] = (x - lc) / (hc - lc);
    tdn[a] = (hc - x) / (hc - lc);
  }
  for (int b = 0; b < (1 << D); ++b) {
    double w = 1.0;
    uint64_t k = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const bool up = (b >> a) & 1;
      w = w * (up ? tup[a] : tdn[a]);
      k |= ((l[a] + (up ? s : 0)) >> sh) << (a * B);
    }
    tk[(i << D) + b] = k;
    tw[(i << D) + b] = w;
  }
}

// Regions at the deepest depth Dstar (positions >= first of the sorted list)
// become their parents; the others stay.
template <int D>
__global__ void k_merge_parents(int64_t nR, int64_t first, const uint32_t* __restrict__ rd,
                                const uint64_t* __restrict__ rk, uint32_t Dstar, uint64_t ps, int B,
                                uint32_t* __restrict__ rd2, uint64_t* __restrict__ rk2) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (i >= nR) return;
  if (i < first) {
    rd2[i] = rd[i];
    rk2[i] = rk[i];
  } else {
    rd2[i] = Dstar - 1;
    rk2[i] = round_down<D>(rk[i], ps, B);
  }
}

// (corner, parent lo) of every merged region's 2^d corners
template <int D>
__global__ void k_corner_parent(int64_t nm, const uint64_t* __restrict__ rk, uint64_t s, uint64_t ps, int B,
                                uint64_t* __restrict__ cpk, uint64_t* __restrict__ cpp) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (q >= (nm << D)) return;
  const int64_t j = q >> D;
  const int b = static_cast<int>(q & ((1 << D) - 1));
  uint64_t k = rk[j];
#pragma unroll
  for (int a = 0; a < D; ++a)
    if ((b >> a) & 1) k += s << (a * B);
  cpk[q] = k;
  cpp[q] = round_down<D>(rk[j], ps, B);
}

// every corner of every region
template <int D>
__global__ void k_region_corners(int64_t n, const uint32_t* __restrict__ rd, const uint64_t* __restrict__ rk,
                                 int B, uint64_t* __restrict__ out) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (q >= (n << D)) return;
  const int64_t j = q >> D;
  const int b = static_cast<int>(q & ((1 << D) - 1));
  const uint64_t s = uint64_t(1) << (B - static_cast<int>(rd[j]));
  uint64_t k = rk[j];
#pragma unroll
  for (int a = 0; a < D; ++a)
    if ((b >> a) & 1) k += s << (a * B);
  out[q] = k;
}

// Level l -> l + 1 after a merge: a vertex that is a corner of a next-level
// region is injected (weight 1), any other is interpolated in the merged parent
// it is a corner of (the first such parent in key order), per axis weight 1 or
// 0 at the parent's faces and 1/2 at its midplane.
template <int D>
__global__ void k_coarse_triplets(int64_t ncur, const uint64_t* __restrict__ ck, const uint64_t* __restrict__ na,
                                  int64_t nna, const uint64_t* __restrict__ cpk,
                                  const uint64_t* __restrict__ cpp, int64_t ncp, uint64_t ps, int B,
                                  uint64_t* __restrict__ tk, double* __restrict__ tw, int* __restrict__ err) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (i >= ncur) return;
  const uint64_t kv = ck[i];
  const int64_t p = lower_bound(na, nna, kv);
  if (p < nna && na[p] == kv) {
    tk[i << D] = kv;
    tw[i << D] = 1.0;
    for (int b = 1; b < (1 << D); ++b) {
      tk[(i << D) + b] = 0;
      tw[(i << D) + b] = 0.0;
    }
    return;
  }
  const int64_t c = lower_bound(cpk, ncp, kv);
  if (c >= ncp || cpk[c] != kv) {
    *err = 1;
    for (int b = 0; b < (1 << D); ++b) {
      tk[(i << D) + b] = 0;
      tw[(i << D) + b] = 0.0;
    }
    return;
  }
  const uint64_t plo = cpp[c];
  double up[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const uint64_t rel = axis_of(kv, a, B) - axis_of(plo, a, B);
    up[a] = rel == ps ? 1.0 : (rel == 0 ? 0.0 : 0.5);
  }
  for (int b = 0; b < (1 << D); ++b) {
    double w = 1.0;
    uint64_t k = plo;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const bool hi = (b >> a) & 1;
      w = w * (hi ? up[a] : 1.0 - up[a]);
      if (hi) k += ps << (a * B);
    }
    tk[(i << D) + b] = k;
    tw[(i << D) + b] = w;
  }
}

// ---- triplets -> CSR
__global__ void k_nonzero(int64_t n, const double* __restrict__ w, uint8_t* __restrict__ f) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (i < n) f[i] = w[i] != 0.0 ? 1 : 0;
}

template <int D>
__global__ void k_row_count(int64_t nrows, const double* __restrict__ tw, int64_t* __restrict__ cnt) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (i >= nrows) return;
  int64_t c = 0;
  for (int b = 0; b < (1 << D); ++b) c += tw[(i << D) + b] != 0.0 ? 1 : 0;
  cnt[i] = c;
}

// row i's entries: columns = ranks of the slot keys among the distinct keys,
// ascending (distinct within a row)
template <int D>
__global__ void k_row_fill(int64_t nrows, const uint64_t* __restrict__ tk, const double* __restrict__ tw,
                           const uint64_t* __restrict__ keys, int64_t nkeys, const int64_t* __restrict__ ptr,
                           int32_t* __restrict__ col, double* __restrict__ val) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (i >= nrows) return;
  int32_t c[1 << D];
  double v[1 << D];
  int k = 0;
  for (int b = 0; b < (1 << D); ++b) {
    const double w = tw[(i << D) + b];
    if (w == 0.0) continue;
    const int32_t j = static_cast<int32_t>(lower_bound(keys, nkeys, tk[(i << D) + b]));
    int q = k++;
    while (q > 0 && c[q - 1] > j) {
      c[q] = c[q - 1];
      v[q] = v[q - 1];
      --q;
    }
    c[q] = j;
    v[q] = w;
  }
  const int64_t p = ptr[i];
  for (int q = 0; q < k; ++q) {
    col[p + q] = c[q];
    val[p + q] = v[q];
  }
}

// Device prolongation (rows = this level's vertices, columns = the next level's)
struct DevP {
  int64_t nrows = 0, ncols = 0, nnz = 0;
  int64_t* ptr = nullptr;
  int32_t* col = nullptr;
  double* val = nullptr;
};

// Assembles P from nrows * 2^d triplet slots; keys_out = the next level's
// packed keys (sorted, distinct), their count in nkeys_out.
template <int D>
DevP triplets_to_csr(Arena& A, int64_t nrows, const uint64_t* tk, const double* tw, int B,
                     uint64_t*& keys_out, int64_t& nkeys_out, int64_t* d_count) {
  const int64_t ns = nrows << D;
  uint8_t* f = A.get<uint8_t>(ns);
  k_nonzero<<<grid_for(ns), kThreads, 0, A.stream()>>>(ns, tw, f);
  uint64_t* kk = A.get<uint64_t>(ns);
  const int64_t nk = select_flagged(A, tk, f, kk, ns, d_count);
  uint64_t* ks = A.get<uint64_t>(nk);
  sort_keys(A, kk, ks, nk, D * B);
  uint64_t* uk = A.get<uint64_t>(nk);
  const int64_t nu = unique_sorted(A, ks, uk, nk, d_count);
  DevP P;
  P.nrows = nrows;
  P.ncols = nu;
  P.ptr = A.get<int64_t>(nrows + 1);
  int64_t* cnt = A.get<int64_t>(nrows);
  k_row_count<D><<<grid_for(nrows), kThreads, 0, A.stream()>>>(nrows, tw, cnt);
  check(hipMemsetAsync(P.ptr, 0, sizeof(int64_t), A.stream()), "clear");
  inclusive_sum(A, cnt, P.ptr + 1, nrows);
  P.nnz = nrows > 0 ? A.fetch(P.ptr + nrows) : 0;
  if (P.nnz != nk) throw Error{VASMG_EINVAL, "internal error: prolongation entry count"};
  P.col = A.get<int32_t>(P.nnz);
  P.val = A.get<double>(P.nnz);
  k_row_fill<D><<<grid_for(nrows), kThreads, 0, A.stream()>>>(nrows, tk, tw, uk, nu, P.ptr, P.col, P.val);
  check(hipGetLastError(), "launch");
  keys_out = uk;
  nkeys_out = nu;
  return P;
}

// Sorts regions by (depth, key) and drops repeats.
template <int D>
int64_t sort_unique_regions(Arena& A, const uint32_t* rd, const uint64_t* rk, int64_t n, int B,
                            uint32_t*& rd_out, uint64_t*& rk_out, int64_t* d_count) {
  uint64_t* k1 = A.get<uint64_t>(n);
  uint32_t* d1 = A.get<uint32_t>(n);
  sort_pairs(A, rk, k1, rd, d1, n, D * B);          // by key, then stably by depth
  uint32_t* d2 = A.get<uint32_t>(n);
  uint64_t* k2 = A.get<uint64_t>(n);
  sort_pairs(A, d1, d2, k1, k2, n, 6);              // depths <= 32
  uint8_t* h = A.get<uint8_t>(n);
  k_region_heads<<<grid_for(n), kThreads, 0, A.stream()>>>(n, d2, k2, h);
  rd_out = A.get<uint32_t>(n);
  rk_out = A.get<uint64_t>(n);
  select_flagged(A, d2, h, rd_out, n, d_count);
  return select_flagged(A, k2, h, rk_out, n, d_count);
}

__global__ void k_tail_info(int64_t nR, const uint32_t* rd, int64_t* out) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const uint32_t Dstar = rd[nR - 1];
  out[0] = Dstar;
  out[1] = lower_bound(rd, nR, Dstar);   // first region at depth Dstar (sorted by depth)
}

struct LevelOut {
  uint64_t* keys = nullptr;   // packed, canonical order
  int64_t n = 0;
  int max_region_depth = 0;
  DevP P;                     // to the next level (none on the last)
};

template <typename T>
void download(std::vector<T>& h, const T* d, int64_t n, hipStream_t st) {
  h.resize(static_cast<size_t>(n));
  if (n > 0) check(hipMemcpyAsync(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost, st), "download");
}

template <int D>
bool build(GalerkinDevice* g, hipStream_t st, const MeshView& mesh, const std::vector<int32_t>& tree_vtx,
           const std::vector<int32_t>& free_vertices, const std::vector<int32_t>& pos_in_tree,
           int cap, Transfers& out) {
  const int64_t N = static_cast<int64_t>(tree_vtx.size());
  const int64_t nf = static_cast<int64_t>(free_vertices.size());
  // 32-bit group keys (group << d | child) and int32 positions
  if (N == 0 || N >= (int64_t(1) << 28)) return false;
  const int max_pack = D == 3 ? 21 : 32;
  // root box: one min and one max over every coordinate of the tree vertices
  double m = mesh.coords[int64_t(tree_vtx[0]) * D], M = m;
  std::vector<double> xt(static_cast<size_t>(N) * D);
  for (int64_t i = 0; i < N; ++i)
    for (int a = 0; a < D; ++a) {
      const double x = mesh.coords[int64_t(tree_vtx[i]) * D + a];
      xt[i * D + a] = x;
      m = std::min(m, x);
      M = std::max(M, x);
    }
  const double S = M - m;
  std::vector<int32_t> ftp(static_cast<size_t>(nf));
  for (int64_t i = 0; i < nf; ++i) ftp[i] = pos_in_tree[free_vertices[i]];

  Arena A(st);
  int64_t* d_count = A.get<int64_t>(2);
  int* d_flag = A.get<int>(1);
  check(hipMemsetAsync(d_flag, 0, sizeof(int), st), "clear");
  double* d_x = A.get<double>(N * D);
  check(hipMemcpyAsync(d_x, xt.data(), xt.size() * sizeof(double), hipMemcpyHostToDevice, st), "upload");
  int32_t* d_ftp = A.get<int32_t>(nf);
  check(hipMemcpyAsync(d_ftp, ftp.data(), ftp.size() * sizeof(int32_t), hipMemcpyHostToDevice, st), "upload");

  // ---- tree: rounds until every vertex sits in a leaf
  uint64_t* lo = A.get<uint64_t>(N * 3);
  check(hipMemsetAsync(lo, 0, N * 3 * sizeof(uint64_t), st), "clear");
  int32_t* leaf_depth = A.get<int32_t>(N);
  int32_t* act = A.get<int32_t>(N);
  int32_t* act2 = A.get<int32_t>(N);
  uint32_t* key = A.get<uint32_t>(N);
  uint32_t* key2 = A.get<uint32_t>(N);
  uint32_t* nkey = A.get<uint32_t>(N);
  int32_t* head = A.get<int32_t>(N);
  int32_t* gid = A.get<int32_t>(N);
  int32_t* start = A.get<int32_t>(N + 1);
  uint8_t* keep = A.get<uint8_t>(N);
  k_iota<<<grid_for(N), kThreads, 0, st>>>(N, act);
  check(hipMemsetAsync(key, 0, N * sizeof(uint32_t), st), "clear");   // all in the root
  int64_t n = N;
  int depth = 1;
  for (;; ++depth) {
    k_heads<<<grid_for(n), kThreads, 0, st>>>(n, key, head);
    inclusive_sum(A, head, gid, n);
    k_group_starts<<<grid_for(n), kThreads, 0, st>>>(n, head, gid, start);
    k_split<D><<<grid_for(n), kThreads, 0, st>>>(n, depth, cap, max_pack, m, S, d_x, act, gid, start, lo,
                                                  leaf_depth, keep, nkey, d_flag);
    check(hipGetLastError(), "launch");
    const int64_t n2 = select_flagged(A, act, keep, act2, n, d_count);
    if (n2 == 0) break;
    select_flagged(A, nkey, keep, key2, n, d_count);
    sort_pairs(A, key2, key, act2, act, n2, 32);
    n = n2;
  }
  if (A.fetch(d_flag)) return false;   // too deep for packed keys
  const int max_depth = depth;
  const int B = max_depth;

  // ---- level-1 regions: the distinct leaves, sorted by (depth, key)
  uint32_t* rd0 = A.get<uint32_t>(N);
  uint64_t* rk0 = A.get<uint64_t>(N);
  k_leaf_regions<D><<<grid_for(N), kThreads, 0, st>>>(N, leaf_depth, lo, B, rd0, rk0);
  uint32_t* rd = nullptr;
  uint64_t* rk = nullptr;
  int64_t nR = sort_unique_regions<D>(A, rd0, rk0, N, B, rd, rk, d_count);

  // ---- fine level -> level 1
  std::vector<LevelOut> levels(1);
  {
    uint64_t* tk = A.get<uint64_t>(nf << D);
    double* tw = A.get<double>(nf << D);
    k_fine_triplets<D><<<grid_for(nf), kThreads, 0, st>>>(nf, d_ftp, leaf_depth, lo, d_x, m, S, B, tk, tw);
    check(hipGetLastError(), "launch");
    LevelOut next;
    levels[0].P = triplets_to_csr<D>(A, nf, tk, tw, B, next.keys, next.n, d_count);
    levels.push_back(next);
  }

  // ---- Section 3.1.2: merge the deepest regions until only the root is left
  for (;;) {
    if (static_cast<int>(levels.size()) > kKeyBits + 1)
      throw Error{VASMG_EINVAL, "internal error: too many levels"};
    LevelOut& cur = levels.back();
    k_tail_info<<<1, 1, 0, st>>>(nR, rd, d_count);
    int64_t info[2];
    check(hipMemcpyAsync(info, d_count, sizeof(info), hipMemcpyDeviceToHost, st), "copy");
    check(hipStreamSynchronize(st), "synchronise");
    const uint32_t Dstar = static_cast<uint32_t>(info[0]);
    const int64_t first = info[1];
    cur.max_region_depth = static_cast<int>(Dstar);
    if (nR == 1 && Dstar == 1) break;
    const uint64_t ps = uint64_t(1) << (B - static_cast<int>(Dstar) + 1);   // parent side
    const uint64_t s = uint64_t(1) << (B - static_cast<int>(Dstar));        // merged region side
    const int64_t nm = nR - first;
    // next regions
    uint32_t* rdm = A.get<uint32_t>(nR);
    uint64_t* rkm = A.get<uint64_t>(nR);
    k_merge_parents<D><<<grid_for(nR), kThreads, 0, st>>>(nR, first, rd, rk, Dstar, ps, B, rdm, rkm);
    // (corner, parent) of the merged regions, sorted by corner then parent
    const int64_t ncp = nm << D;
    uint64_t* cpk0 = A.get<uint64_t>(ncp);
    uint64_t* cpp0 = A.get<uint64_t>(ncp);
    k_corner_parent<D><<<grid_for(ncp), kThreads, 0, st>>>(nm, rk + first, s, ps, B, cpk0, cpp0);
    uint64_t* cpp1 = A.get<uint64_t>(ncp);
    uint64_t* cpk1 = A.get<uint64_t>(ncp);
    sort_pairs(A, cpp0, cpp1, cpk0, cpk1, ncp, D * B);
    uint64_t* cpk = A.get<uint64_t>(ncp);
    uint64_t* cpp = A.get<uint64_t>(ncp);
    sort_pairs(A, cpk1, cpk, cpp1, cpp, ncp, D * B);
    uint32_t* rdn = nullptr;
    uint64_t* rkn = nullptr;
    const int64_t nRn = sort_unique_regions<D>(A, rdm, rkm, nR, B, rdn, rkn, d_count);
    // every corner of the next regions
    const int64_t nc = nRn << D;
    uint64_t* c0 = A.get<uint64_t>(nc);
    k_region_corners<D><<<grid_for(nc), kThreads, 0, st>>>(nRn, rdn, rkn, B, c0);
    uint64_t* c1 = A.get<uint64_t>(nc);
    sort_keys(A, c0, c1, nc, D * B);
    uint64_t* na = A.get<uint64_t>(nc);
    const int64_t nna = unique_sorted(A, c1, na, nc, d_count);
    // this level -> the next
    uint64_t* tk = A.get<uint64_t>(cur.n << D);
    double* tw = A.get<double>(cur.n << D);
    k_coarse_triplets<D><<<grid_for(cur.n), kThreads, 0, st>>>(cur.n, cur.keys, na, nna, cpk, cpp, ncp, ps,
                                                                 B, tk, tw, d_flag);
    check(hipGetLastError(), "launch");
    if (A.fetch(d_flag))
      throw Error{VASMG_EINVAL, "internal error: interpolated vertex is not a corner of a merged region"};
    LevelOut next;
    cur.P = triplets_to_csr<D>(A, cur.n, tk, tw, B, next.keys, next.n, d_count);
    levels.push_back(next);   // cur is not used after this
    rd = rdn;
    rk = rkn;
    nR = nRn;
  }

  // ---- to the host: keys unpacked to key units, P as host CSR
  const int L = static_cast<int>(levels.size());
  std::vector<std::vector<uint64_t>> packed(L);
  out = Transfers();
  out.m = m;
  out.M = M;
  out.max_depth = max_depth;
  out.keys.resize(L);
  out.max_region_depth.assign(L, 0);
  out.P.resize(L - 1);
  for (int l = 0; l < L; ++l) {
    if (l >= 1) download(packed[l], levels[l].keys, levels[l].n, st);
    out.max_region_depth[l] = levels[l].max_region_depth;
    if (l + 1 < L) {
      const DevP& P = levels[l].P;
      ScalarCSR& H = out.P[l];
      H.nrows = P.nrows;
      H.ncols = P.ncols;
      download(H.rowptr, P.ptr, P.nrows + 1, st);
      download(H.col, P.col, P.nnz, st);
      download(H.val, P.val, P.nnz, st);
    }
  }
  // device copies of the prolongations for the Galerkin products (owned by the
  // context from here on)
  for (int l = 0; l + 1 < L; ++l) {
    const DevP& P = levels[l].P;
    int64_t* ptr = nullptr;
    int32_t* col = nullptr;
    double* val = nullptr;
    check(hipMallocAsync(reinterpret_cast<void**>(&ptr), (P.nrows + 1) * sizeof(int64_t), st), "allocation");
    check(hipMallocAsync(reinterpret_cast<void**>(&col), std::max<int64_t>(P.nnz, 1) * sizeof(int32_t), st),
          "allocation");
    check(hipMallocAsync(reinterpret_cast<void**>(&val), std::max<int64_t>(P.nnz, 1) * sizeof(double), st),
          "allocation");
    check(hipMemcpyAsync(ptr, P.ptr, (P.nrows + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice, st), "copy");
    if (P.nnz > 0) {
      check(hipMemcpyAsync(col, P.col, P.nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, st), "copy");
      check(hipMemcpyAsync(val, P.val, P.nnz * sizeof(double), hipMemcpyDeviceToDevice, st), "copy");
    }
    galerkin_device_adopt_prolongation(g, l, P.nrows, P.ncols, P.nnz, ptr, col, val);
  }
  check(hipStreamSynchronize(st), "download");
  const int sh = kKeyBits - B;
  for (int l = 1; l < L; ++l) {
    std::vector<Key>& K = out.keys[l];
    K.resize(packed[l].size());
    for (size_t i = 0; i < K.size(); ++i) {
      Key k{0, 0, 0};
      for (int a = 0; a < D; ++a) k[a] = axis_of(packed[l][i], a, B) << sh;
      K[i] = k;
    }
  }
  return true;
}

// ---- vertex -> element lists (the host's vertex_elements, elements ascending)
__global__ void k_ve_count(int64_t nslots, const int32_t* __restrict__ elems,
                           unsigned long long* __restrict__ cnt) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (q < nslots) atomicAdd(&cnt[elems[q]], 1ull);
}

__global__ void k_ve_fill(int64_t nslots, int nvpe, const int32_t* __restrict__ elems,
                          const int64_t* __restrict__ vptr, int* __restrict__ fill,
                          int32_t* __restrict__ velem) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (q >= nslots) return;
  const int32_t v = elems[q];
  velem[vptr[v] + atomicAdd(&fill[v], 1)] = static_cast<int32_t>(q / nvpe);
}

// each vertex's list in ascending element order (the slots were claimed in any order)
__global__ void k_ve_sort(int64_t nv, const int64_t* __restrict__ vptr, int32_t* __restrict__ velem) {
  const int64_t v = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (v >= nv) return;
  const int64_t b = vptr[v], e = vptr[v + 1];
  for (int64_t i = b + 1; i < e; ++i) {
    const int32_t t = velem[i];
    int64_t j = i;
    while (j > b && velem[j - 1] > t) {
      velem[j] = velem[j - 1];
      --j;
    }
    velem[j] = t;
  }
}

// ---- transpose of a scalar CSR matrix
__global__ void k_row_of(int64_t nrows, const int64_t* __restrict__ ptr, int32_t* __restrict__ row) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (r >= nrows) return;
  for (int64_t p = ptr[r]; p < ptr[r + 1]; ++p) row[p] = static_cast<int32_t>(r);
}

__global__ void k_count_cols(int64_t nnz, const int32_t* __restrict__ col, unsigned long long* __restrict__ cnt) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (p < nnz) atomicAdd(&cnt[col[p]], 1ull);
}

__global__ void k_gather_transposed(int64_t nnz, const int32_t* __restrict__ order,
                                    const int32_t* __restrict__ row, const double* __restrict__ val,
                                    int32_t* __restrict__ tcol, double* __restrict__ tval) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (q >= nnz) return;
  const int32_t p = order[q];
  tcol[q] = row[p];
  tval[q] = val[p];
}

}  // namespace tree

void transpose_device(void* stream, int64_t nrows, int64_t ncols, int64_t nnz, const int64_t* ptr,
                      const int32_t* col, const double* val, int64_t* tptr, int32_t* tcol, double* tval) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  tree::Arena A(st);
  tree::check(hipMemsetAsync(tptr, 0, sizeof(int64_t), st), "clear");
  if (nnz > 0) {
    int32_t* row = A.get<int32_t>(nnz);
    tree::k_row_of<<<tree::grid_for(nrows), tree::kThreads, 0, st>>>(nrows, ptr, row);
    int32_t* idx = A.get<int32_t>(nnz);
    tree::k_iota<<<tree::grid_for(nnz), tree::kThreads, 0, st>>>(nnz, idx);
    // entries by column, stably (row order kept inside a column); columns >= 0
    uint32_t* ks = A.get<uint32_t>(nnz);
    int32_t* order = A.get<int32_t>(nnz);
    int bits = 1;
    while ((int64_t(1) << bits) < ncols) ++bits;
    tree::sort_pairs(A, reinterpret_cast<const uint32_t*>(col), ks, idx, order, nnz, bits);
    tree::k_gather_transposed<<<tree::grid_for(nnz), tree::kThreads, 0, st>>>(nnz, order, row, val, tcol, tval);
  }
  if (ncols > 0) {
    auto* cnt = A.get<unsigned long long>(ncols);
    tree::check(hipMemsetAsync(cnt, 0, ncols * sizeof(unsigned long long), st), "clear");
    if (nnz > 0) tree::k_count_cols<<<tree::grid_for(nnz), tree::kThreads, 0, st>>>(nnz, col, cnt);
    tree::inclusive_sum(A, reinterpret_cast<const int64_t*>(cnt), tptr + 1, ncols);
  }
  tree::check(hipGetLastError(), "launch");
}

namespace tree {

// Row lengths of P in device order: row i is canonical row perm[i].
__global__ void k_perm_rowlen(int64_t n, const int64_t* __restrict__ ptr, const int32_t* __restrict__ perm,
                              int64_t* __restrict__ len) {
  const int64_t i = blockIdx.x * int64_t(kThreads) + threadIdx.x;
  if (i < n) len[i] = ptr[perm[i] + 1] - ptr[perm[i]];
}

// Row i's entries: canonical row perm[i] in its order, columns renumbered.
__global__ void k_perm_fill(int64_t n, const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
                            const double* __restrict__ val, const int32_t* __restrict__ perm,
                            const int32_t* __restrict__ inv_next, const int64_t* __restrict__ pptr,
                            int32_t* __restrict__ pidx, double* __restrict__ pw) {
  const int64_t i = blockIdx.x * int64_t(kThreads) + threadIdx.x;
  if (i >= n) return;
  const int64_t b = ptr[perm[i]], e = ptr[perm[i] + 1];
  int64_t q = pptr[i];
  for (int64_t p = b; p < e; ++p, ++q) {
    pidx[q] = inv_next[col[p]];
    pw[q] = val[p];
  }
}

__global__ void k_narrow_ptr(int64_t n, const int64_t* __restrict__ p64, int32_t* __restrict__ p32) {
  const int64_t i = blockIdx.x * int64_t(kThreads) + threadIdx.x;
  if (i < n) p32[i] = static_cast<int32_t>(p64[i]);
}

__global__ void k_round_f32(int64_t n, const double* __restrict__ v, float* __restrict__ w) {
  const int64_t i = blockIdx.x * int64_t(kThreads) + threadIdx.x;
  if (i < n) w[i] = static_cast<float>(v[i]);
}

}  // namespace tree

void transfers_layout_device(void* stream, int64_t n, int64_t nn, int64_t nnz, const int64_t* ptr,
                             const int32_t* col, const double* val, const int32_t* perm,
                             const int32_t* inv_next, int32_t* pptr, int32_t* pidx, double* pw64,
                             float* pw32, int32_t* tptr, int32_t* tidx, double* tw64, float* tw32) {
  if (nnz > INT32_MAX) throw Error{VASMG_EINVAL, "prolongation too large for 32-bit row pointers"};
  hipStream_t st = static_cast<hipStream_t>(stream);
  tree::Arena A(st);
  int64_t* pptr64 = A.get<int64_t>(n + 1);
  int64_t* tptr64 = A.get<int64_t>(nn + 1);
  double* pw = pw64 ? pw64 : A.get<double>(nnz);
  double* tw = tw64 ? tw64 : A.get<double>(nnz);
  tree::check(hipMemsetAsync(pptr64, 0, sizeof(int64_t), st), "clear");
  if (n > 0) {
    int64_t* len = A.get<int64_t>(n);
    tree::k_perm_rowlen<<<tree::grid_for(n), tree::kThreads, 0, st>>>(n, ptr, perm, len);
    tree::inclusive_sum(A, len, pptr64 + 1, n);
    tree::k_perm_fill<<<tree::grid_for(n), tree::kThreads, 0, st>>>(n, ptr, col, val, perm, inv_next, pptr64,
                                                                  pidx, pw);
  }
  transpose_device(st, n, nn, nnz, pptr64, pidx, pw, tptr64, tidx, tw);
  tree::k_narrow_ptr<<<tree::grid_for(n + 1), tree::kThreads, 0, st>>>(n + 1, pptr64, pptr);
  tree::k_narrow_ptr<<<tree::grid_for(nn + 1), tree::kThreads, 0, st>>>(nn + 1, tptr64, tptr);
  if (pw32 && nnz > 0) tree::k_round_f32<<<tree::grid_for(nnz), tree::kThreads, 0, st>>>(nnz, pw, pw32);
  if (tw32 && nnz > 0) tree::k_round_f32<<<tree::grid_for(nnz), tree::kThreads, 0, st>>>(nnz, tw, tw32);
  tree::check(hipGetLastError(), "launch");
  // the arena's temporaries are released in stream order; the caller synchronises
  // before it uses the results off this stream
}

void vertex_elements_device(void* stream, const int32_t* elems, int64_t ne, int nvpe, int64_t nv,
                            int64_t* vptr, int32_t* velem) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  tree::Arena A(st);
  const int64_t ns = ne * nvpe;
  auto* cnt = A.get<unsigned long long>(nv);
  int* fill = A.get<int>(nv);
  tree::check(hipMemsetAsync(cnt, 0, nv * sizeof(unsigned long long), st), "clear");
  tree::check(hipMemsetAsync(fill, 0, nv * sizeof(int), st), "clear");
  tree::check(hipMemsetAsync(vptr, 0, sizeof(int64_t), st), "clear");
  tree::k_ve_count<<<tree::grid_for(ns), tree::kThreads, 0, st>>>(ns, elems, cnt);
  tree::inclusive_sum(A, reinterpret_cast<const int64_t*>(cnt), vptr + 1, nv);
  tree::k_ve_fill<<<tree::grid_for(ns), tree::kThreads, 0, st>>>(ns, nvpe, elems, vptr, fill, velem);
  tree::k_ve_sort<<<tree::grid_for(nv), tree::kThreads, 0, st>>>(nv, vptr, velem);
  tree::check(hipGetLastError(), "launch");
}

bool transfers_device(void* ctx, const MeshView& m, const std::vector<int32_t>& tree_vtx,
                      const std::vector<int32_t>& free_vertices, const std::vector<int32_t>& pos_in_tree,
                      int capacity, Transfers& out) {
  auto* g = static_cast<GalerkinDevice*>(ctx);
  hipStream_t st = static_cast<hipStream_t>(galerkin_device_stream(g));
  if (m.d == 3) return tree::build<3>(g, st, m, tree_vtx, free_vertices, pos_in_tree, capacity, out);
  return tree::build<2>(g, st, m, tree_vtx, free_vertices, pos_in_tree, capacity, out);
}

}  // namespace vasmg
