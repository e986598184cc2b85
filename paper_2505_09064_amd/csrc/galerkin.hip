// Galerkin coarse operators on the device: A_{l+1} = P_l^T A_l P_l (Section 3,
// equation (Ac); P = P_s (x) I_d, so every scalar weight scales a whole d x d
// block).
//
// The product is formed as two row-wise sparse products, AP = A P and then
// A_c = P^T (AP), each in three launches:
//   1. symbolic count: the distinct columns of every output row, found with a
//      bitmap in LDS over a window of columns (rows whose column range exceeds
//      the window take several passes);
//   2. symbolic fill: the same bitmap walk writes the columns, ascending, at
//      offsets from the host's prefix sum of the counts;
//   3. numeric: one thread per output block; it walks the row's contributions in
//      a fixed order (X entries ascending, then Y entries ascending) and adds the
//      ones that land on its column. No atomics: the result is the same bit for
//      bit on every run and for every launch shape.
// Values are FP64 throughout. The order of the sums differs from the host's
// single-pass triple product, so the two agree to rounding, not bit for bit; the
// column structure is identical.
//
// Every level's canonical operator stays resident until the device layout of the
// level (colour-ordered rows, off-cell L / U parts, cell matrices or diagonals,
// in the solve precisions) has been built from it by the layout kernels below;
// the host receives each product's structure at once (cells and colours are
// built from it) and its values from a background download. The layout kernels
// also serve uploads of host-built hierarchies (the operator copied in first).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "hierarchy.hpp"
#include "vasmg.h"

namespace vasmg {
namespace gal {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kMaxWindowCols = 65536;   // LDS bitmap: 8 KiB per workgroup

void check(hipError_t e, const char* what) {
  if (e != hipSuccess)
    throw Error{VASMG_EDEVICE, std::string("device Galerkin product: ") + what + ": " +
                                   hipGetErrorString(e)};
}

// CSR operand on the device: scalar values ([nnz]) or d x d blocks ([nnz][d*d]).
struct Csr {
  const int64_t* __restrict__ ptr;
  const int32_t* __restrict__ col;
  const double* __restrict__ val;
};

__device__ __forceinline__ int wave_min(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// Exclusive prefix sum of v over the workgroup; *total gets the sum.
__device__ __forceinline__ int block_exclusive_scan(int v, int* sh, int* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int inc = v;
  for (int o = 1; o < 64; o <<= 1) {
    const int u = __shfl_up(inc, o, 64);
    if (lane >= o) inc += u;
  }
  if (lane == 63) sh[wave] = inc;
  __syncthreads();
  int base = 0, all = 0;
  for (int w = 0; w < kWaves; ++w) {
    const int s = sh[w];
    if (w < wave) base += s;
    all += s;
  }
  __syncthreads();
  *total = all;
  return base + inc - v;
}

// Row i of X * Y: its distinct columns, counted (FILL = false: cnt[i]) or written
// ascending to ccol[cptr[i] ...] (FILL = true). One workgroup per row; thread t
// takes the X entries t, t + 256, ... and their whole Y rows.
template <bool FILL>
__global__ __launch_bounds__(kThreads) void k_symbolic(int32_t nrows, Csr X, Csr Y, int window,
                                                       int64_t* __restrict__ cnt,
                                                       const int64_t* __restrict__ cptr,
                                                       int32_t* __restrict__ ccol) {
  __shared__ uint32_t bits[kMaxWindowCols / 32];
  __shared__ int sh[2 * kWaves];
  const int32_t i = blockIdx.x;
  if (i >= nrows) return;
  const int t = threadIdx.x;
  const int64_t xb = X.ptr[i], xe = X.ptr[i + 1];

  int lo = INT_MAX, hi = -1;
  for (int64_t p = xb + t; p < xe; p += kThreads) {
    const int k = X.col[p];
    for (int64_t q = Y.ptr[k], qe = Y.ptr[k + 1]; q < qe; ++q) {
      const int j = Y.col[q];
      lo = min(lo, j);
      hi = max(hi, j);
    }
  }
  lo = wave_min(lo);
  hi = wave_max(hi);
  if ((t & 63) == 0) {
    sh[t >> 6] = lo;
    sh[kWaves + (t >> 6)] = hi;
  }
  __syncthreads();
  lo = INT_MAX;
  hi = -1;
  for (int w = 0; w < kWaves; ++w) {
    lo = min(lo, sh[w]);
    hi = max(hi, sh[kWaves + w]);
  }
  __syncthreads();

  int64_t done = 0;   // columns of this row found in earlier windows
  for (int64_t w0 = lo; w0 <= hi; w0 += window) {
    const int ncols = static_cast<int>(min<int64_t>(window, hi - w0 + 1));
    const int nwords = (ncols + 31) >> 5;
    for (int w = t; w < nwords; w += kThreads) bits[w] = 0u;
    __syncthreads();
    for (int64_t p = xb + t; p < xe; p += kThreads) {
      const int k = X.col[p];
      for (int64_t q = Y.ptr[k], qe = Y.ptr[k + 1]; q < qe; ++q) {
        const int64_t r = static_cast<int64_t>(Y.col[q]) - w0;
        if (r >= 0 && r < ncols) atomicOr(&bits[r >> 5], 1u << (r & 31));
      }
    }
    __syncthreads();
    const int per = (nwords + kThreads - 1) / kThreads;
    const int wb = min(t * per, nwords), we = min(wb + per, nwords);
    int c = 0;
    for (int w = wb; w < we; ++w) c += __popc(bits[w]);
    int total = 0;
    const int off = block_exclusive_scan(c, sh, &total);
    if (FILL) {
      int64_t pos = cptr[i] + done + off;
      for (int w = wb; w < we; ++w) {
        uint32_t b = bits[w];
        while (b) {
          const int bit = __ffs(b) - 1;
          b &= b - 1;
          ccol[pos++] = static_cast<int32_t>(w0 + (static_cast<int64_t>(w) << 5) + bit);
        }
      }
    }
    done += total;
    __syncthreads();   // the bitmap is cleared for the next window
  }
  if (!FILL && t == 0) cnt[i] = done;
}

// Values of row i of X * Y at the columns the symbolic pass wrote. XB: X holds
// d x d blocks and Y scalars (A P); else X scalars and Y blocks (P^T (AP)).
template <int D, bool XB>
__global__ __launch_bounds__(kThreads) void k_numeric(int32_t nrows, Csr X, Csr Y,
                                                      const int64_t* __restrict__ cptr,
                                                      const int32_t* __restrict__ ccol,
                                                      double* __restrict__ cval) {
  constexpr int DD = D * D;
  constexpr int U = 8;
  const int32_t i = blockIdx.x;
  if (i >= nrows) return;
  const int64_t cb = cptr[i], ce = cptr[i + 1];
  const int64_t xb = X.ptr[i], xe = X.ptr[i + 1];
  for (int64_t s0 = cb; s0 < ce; s0 += kThreads) {
    if (s0 + (threadIdx.x & ~63) >= ce) break;   // this wave owns no block of the row
    const int64_t s = s0 + threadIdx.x;
    const int my = s < ce ? ccol[s] : -1;
    double acc[DD];
#pragma unroll
    for (int e = 0; e < DD; ++e) acc[e] = 0.0;
    for (int64_t p = xb; p < xe; ++p) {
      const int k = X.col[p];
      const int64_t qb = Y.ptr[k], qe = Y.ptr[k + 1];
      auto add = [&](int64_t q) {
        if constexpr (XB) {
          const double w = Y.val[q];
#pragma unroll
          for (int e = 0; e < DD; ++e) acc[e] += X.val[p * DD + e] * w;
        } else {
          const double w = X.val[p];
#pragma unroll
          for (int e = 0; e < DD; ++e) acc[e] += w * Y.val[q * DD + e];
        }
      };
      int64_t q = qb;
      for (; q + U <= qe; q += U) {
        int j[U];
#pragma unroll
        for (int u = 0; u < U; ++u) j[u] = Y.col[q + u];
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (j[u] == my) add(q + u);
      }
      for (; q < qe; ++q)
        if (Y.col[q] == my) add(q);
    }
    if (s < ce) {
#pragma unroll
      for (int e = 0; e < DD; ++e) cval[s * DD + e] = acc[e];
    }
  }
}

// Allocations and frees are ordered on the product stream: no device-wide
// synchronisation, so a setup can run beside other threads' solves and graph
// captures (a server's setup workers).
template <typename T>
T* dmalloc(size_t n, hipStream_t st, const char* what) {
  void* p = nullptr;
  check(hipMallocAsync(&p, std::max<size_t>(n, 1) * sizeof(T), st), what);
  return static_cast<T*>(p);
}

// Device CSR owned by the product driver.
struct DevCsr {
  int64_t nrows = 0, nnz = 0;
  int64_t* ptr = nullptr;
  int32_t* col = nullptr;
  double* val = nullptr;
  void release(hipStream_t st) {
    if (ptr) (void)hipFreeAsync(ptr, st);
    if (col) (void)hipFreeAsync(col, st);
    if (val) (void)hipFreeAsync(val, st);
    ptr = nullptr;
    col = nullptr;
    val = nullptr;
    nrows = nnz = 0;
  }
  Csr view() const { return Csr{ptr, col, val}; }
};

}  // namespace gal

struct GalerkinDevice {
  int device = 0;
  hipStream_t st = nullptr;   // products and layouts
  hipStream_t dl = nullptr;   // background value downloads
  int window = gal::kMaxWindowCols;
  const BlockCSR* cached = nullptr;   // host operator of the last resident level
  std::vector<gal::DevCsr> lev;       // resident canonical operators, by level
  struct Pending {
    int level;
    BlockCSR* host;
  };
  std::vector<Pending> pending;       // value downloads not started yet
  std::vector<std::thread> downloads;
  std::mutex mu;
  std::string dl_error;
  void join() {
    for (auto& t : downloads)
      if (t.joinable()) t.join();
    downloads.clear();
  }
  ~GalerkinDevice() {
    join();   // downloads not started by now are not needed
    for (auto& L : lev) L.release(st);
    if (st) (void)hipStreamSynchronize(st);
    if (st) (void)hipStreamDestroy(st);
    if (dl) (void)hipStreamDestroy(dl);
  }
};

namespace gal {

void upload(DevCsr& D, int64_t nrows, const std::vector<int64_t>& ptr,
            const std::vector<int32_t>& col, const std::vector<double>& val, hipStream_t st) {
  D.nrows = nrows;
  D.nnz = static_cast<int64_t>(col.size());
  D.ptr = dmalloc<int64_t>(ptr.size(), st, "rowptr");
  D.col = dmalloc<int32_t>(col.size(), st, "columns");
  D.val = dmalloc<double>(val.size(), st, "values");
  check(hipMemcpyAsync(D.ptr, ptr.data(), ptr.size() * sizeof(int64_t), hipMemcpyHostToDevice, st), "copy");
  check(hipMemcpyAsync(D.col, col.data(), col.size() * sizeof(int32_t), hipMemcpyHostToDevice, st), "copy");
  check(hipMemcpyAsync(D.val, val.data(), val.size() * sizeof(double), hipMemcpyHostToDevice, st), "copy");
}

// C = X * Y with one block operand (XB: X), columns ascending per row.
template <int D, bool XB>
void product(GalerkinDevice& G, const DevCsr& X, const DevCsr& Y, int64_t ncols, DevCsr& C) {
  constexpr int DD = D * D;
  hipStream_t st = G.st;
  const int64_t n = X.nrows;
  if (n > INT32_MAX || ncols > INT32_MAX) throw Error{VASMG_EINVAL, "level too large for int32 indices"};
  const int32_t n32 = static_cast<int32_t>(n);
  C.nrows = n;
  C.ptr = dmalloc<int64_t>(n + 1, st, "rowptr");
  int64_t* cnt = dmalloc<int64_t>(n, st, "row counts");
  if (n > 0)
    hipLaunchKernelGGL(k_symbolic<false>, dim3(n32), dim3(kThreads), 0, st, n32, X.view(), Y.view(),
                       G.window, cnt, nullptr, nullptr);
  check(hipGetLastError(), "symbolic count launch");
  std::vector<int64_t> h(n + 1, 0);
  check(hipMemcpyAsync(h.data() + 1, cnt, n * sizeof(int64_t), hipMemcpyDeviceToHost, st), "copy");
  check(hipStreamSynchronize(st), "symbolic count");
  for (int64_t r = 0; r < n; ++r) h[r + 1] += h[r];
  C.nnz = h[n];
  check(hipMemcpyAsync(C.ptr, h.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st), "copy");
  C.col = dmalloc<int32_t>(C.nnz, st, "columns");
  C.val = dmalloc<double>(C.nnz * DD, st, "values");
  if (n > 0) {
    hipLaunchKernelGGL(k_symbolic<true>, dim3(n32), dim3(kThreads), 0, st, n32, X.view(), Y.view(),
                       G.window, nullptr, C.ptr, C.col);
    check(hipGetLastError(), "symbolic fill launch");
    hipLaunchKernelGGL((k_numeric<D, XB>), dim3(n32), dim3(kThreads), 0, st, n32, X.view(),
                       Y.view(), C.ptr, C.col, C.val);
    check(hipGetLastError(), "numeric launch");
  }
  check(hipStreamSynchronize(st), "product");
  (void)hipFreeAsync(cnt, st);
}

// Copies the values of resident level l into host->val (allocated here, so the
// pages are touched by this thread); with free_after, then releases the level's
// device copy (ordered on the download stream). Runs on its own thread.
void download_values(GalerkinDevice* G, int l, BlockCSR* host, bool free_after) {
  DevCsr L;
  {
    std::lock_guard<std::mutex> g(G->mu);
    L = G->lev[l];
  }
  const size_t count = static_cast<size_t>(L.nnz) * host->d * host->d;
  hipError_t e = hipSetDevice(G->device);
  if (e == hipSuccess) {
    try {
      host->val.resize(count);
    } catch (const std::bad_alloc&) {
      std::lock_guard<std::mutex> g(G->mu);
      G->dl_error = "device Galerkin product: host allocation of the level values failed";
      return;
    }
    e = hipMemcpyAsync(host->val.data(), L.val, count * sizeof(double), hipMemcpyDeviceToHost, G->dl);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(G->dl);
  if (e == hipSuccess && free_after) {
    std::lock_guard<std::mutex> g(G->mu);
    G->lev[l].release(G->dl);
  }
  if (e != hipSuccess) {
    std::lock_guard<std::mutex> g(G->mu);
    G->dl_error = std::string("device Galerkin product: value download: ") + hipGetErrorString(e);
  }
}

template <int D>
void galerkin_d(GalerkinDevice& G, const BlockCSR& A, const ScalarCSR& P, BlockCSR& Ac,
                bool coarsest) {
  constexpr int DD = D * D;
  hipStream_t st = G.st;
  if (G.lev.empty()) {
    G.lev.emplace_back();
    upload(G.lev.back(), A.n, A.rowptr, A.col, A.val, st);
  } else if (G.cached != &A) {
    throw Error{VASMG_EINVAL, "internal: device Galerkin products out of level order"};
  }
  const DevCsr& dA = G.lev.back();
  // P and its transpose (rows = coarse vertices), built on the host: <= 2^d
  // entries per P row
  ScalarCSR PT;
  PT.nrows = P.ncols;
  PT.ncols = P.nrows;
  PT.rowptr.assign(P.ncols + 1, 0);
  for (int32_t c : P.col) PT.rowptr[c + 1]++;
  for (int64_t r = 0; r < P.ncols; ++r) PT.rowptr[r + 1] += PT.rowptr[r];
  PT.col.resize(P.col.size());
  PT.val.resize(P.col.size());
  {
    std::vector<int64_t> fill(PT.rowptr.begin(), PT.rowptr.end() - 1);
    for (int64_t r = 0; r < P.nrows; ++r)
      for (int64_t p = P.rowptr[r]; p < P.rowptr[r + 1]; ++p) {
        const int64_t q = fill[P.col[p]]++;
        PT.col[q] = static_cast<int32_t>(r);
        PT.val[q] = P.val[p];
      }
  }
  DevCsr dP, dPT, AP, C;
  try {
    upload(dP, P.nrows, P.rowptr, P.col, P.val, st);
    upload(dPT, PT.nrows, PT.rowptr, PT.col, PT.val, st);
    product<D, true>(G, dA, dP, P.ncols, AP);
    product<D, false>(G, dPT, AP, P.ncols, C);
    Ac.n = P.ncols;
    Ac.d = D;
    Ac.rowptr.resize(C.nrows + 1);
    Ac.col.resize(C.nnz);
    check(hipMemcpyAsync(Ac.rowptr.data(), C.ptr, (C.nrows + 1) * sizeof(int64_t),
                         hipMemcpyDeviceToHost, st), "copy");
    check(hipMemcpyAsync(Ac.col.data(), C.col, C.nnz * sizeof(int32_t), hipMemcpyDeviceToHost, st), "copy");
    if (coarsest) {
      Ac.val.resize(C.nnz * DD);
      check(hipMemcpyAsync(Ac.val.data(), C.val, C.nnz * DD * sizeof(double), hipMemcpyDeviceToHost, st),
            "copy");
    }
    check(hipStreamSynchronize(st), "download");
  } catch (...) {
    dP.release(st);
    dPT.release(st);
    AP.release(st);
    C.release(st);
    throw;
  }
  dP.release(st);
  dPT.release(st);
  AP.release(st);
  G.lev.push_back(C);
  G.cached = &Ac;
  if (!coarsest) G.pending.push_back({static_cast<int>(G.lev.size()) - 1, &Ac});
}

// ---------------------------------------------------------------------------
// device layout of a level from its resident canonical operator
// ---------------------------------------------------------------------------
constexpr int kLayoutStage = 1024;   // device columns of one row staged in LDS

// Off-cell blocks below / above the row's cell. One wavefront per device row.
__global__ __launch_bounds__(kThreads) void k_layout_count(int n, Csr A, const int* __restrict__ perm,
                                                           const int* __restrict__ inv,
                                                           const int* __restrict__ lo_,
                                                           const int* __restrict__ hi_,
                                                           int* __restrict__ cntL,
                                                           int* __restrict__ cntU) {
  const int i = blockIdx.x * kWaves + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  const int c = perm[i];
  const int lo = lo_[i], hi = hi_[i];
  int cl = 0, cu = 0;
  for (int64_t p = A.ptr[c] + lane; p < A.ptr[c + 1]; p += 64) {
    const int j = inv[A.col[p]];
    cl += j < lo;
    cu += j >= hi;
  }
  for (int o = 32; o > 0; o >>= 1) {
    cl += __shfl_xor(cl, o, 64);
    cu += __shfl_xor(cu, o, 64);
  }
  if (lane == 0) {
    cntL[i] = cl;
    cntU[i] = cu;
  }
}

// One wavefront per device row: the row's device columns are staged in LDS
// (rows longer than the stage read them from memory), each off-cell block goes
// to position (number of same-part blocks with a smaller column) of its part.
template <int D>
__global__ __launch_bounds__(kThreads) void k_layout_fill(Csr A, LayoutArgs a) {
  constexpr int DD = D * D, NU = (1 << D) * D;
  __shared__ int sj[kWaves][kLayoutStage];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * kWaves + w;
  const bool valid = i < a.n;
  const int c = valid ? a.perm[i] : 0;
  const int64_t rb = valid ? A.ptr[c] : 0, re = valid ? A.ptr[c + 1] : 0;
  const int len = static_cast<int>(re - rb);
  const bool staged = len <= kLayoutStage;
  if (staged)
    for (int e = lane; e < len; e += 64) sj[w][e] = a.inv[A.col[rb + e]];
  __syncthreads();
  if (!valid) return;
  const int lo = a.lo[i], hi = a.hi[i];
  auto col_of = [&](int e) { return staged ? sj[w][e] : a.inv[A.col[rb + e]]; };
  for (int e = lane; e < len; e += 64) {
    const int j = col_of(e);
    const double* blk = A.val + (rb + e) * DD;
    if (j < lo || j >= hi) {
      const bool low = j < lo;
      int rank = 0;
      for (int f = 0; f < len; ++f) {
        const int jf = col_of(f);
        rank += jf < j && (low || jf >= hi);
      }
      const int64_t q = (low ? a.Lptr[i] : a.Uptr[i]) + rank;
      const int64_t stride = low ? a.nL : a.nU;
      (low ? a.Lcol : a.Ucol)[q] = j;
      float* v32 = low ? a.L32 : a.U32;
      double* v64 = low ? a.L64 : a.U64;
#pragma unroll
      for (int t = 0; t < DD; ++t) {
        if (v64) v64[t * stride + q] = blk[t];
        if (v32) v32[t * stride + q] = static_cast<float>(blk[t]);
      }
    } else if (a.cell_of_row) {
      const int64_t base = static_cast<int64_t>(a.cell_of_row[i]) * NU * NU;
      const int ki = i - lo, kj = j - lo;
#pragma unroll
      for (int r = 0; r < D; ++r)
#pragma unroll
        for (int s = 0; s < D; ++s) {
          const int64_t m = base + (kj * D + s) * NU + (ki * D + r);
          if (a.M64) a.M64[m] = blk[r * D + s];
          if (a.M32) a.M32[m] = static_cast<float>(blk[r * D + s]);
        }
    } else {
#pragma unroll
      for (int t = 0; t < DD; ++t) {
        if (a.M64) a.M64[static_cast<int64_t>(i) * DD + t] = blk[t];
        if (a.M32) a.M32[static_cast<int64_t>(i) * DD + t] = static_cast<float>(blk[t]);
      }
    }
  }
  // padding of the rows' parts: column i, zero blocks
  for (int part = 0; part < 2; ++part) {
    const int64_t b = (part ? a.Uptr[i] : a.Lptr[i]) + (part ? a.cntU[i] : a.cntL[i]);
    const int64_t e = part ? a.Uptr[i + 1] : a.Lptr[i + 1];
    const int64_t stride = part ? a.nU : a.nL;
    for (int64_t q = b + lane; q < e; q += 64) {
      (part ? a.Ucol : a.Lcol)[q] = i;
      float* v32 = part ? a.U32 : a.L32;
      double* v64 = part ? a.U64 : a.L64;
      for (int t = 0; t < DD; ++t) {
        if (v64) v64[t * stride + q] = 0.0;
        if (v32) v32[t * stride + q] = 0.0f;
      }
    }
  }
}

}  // namespace gal

GalerkinDevice* galerkin_device_create(int window_cols) {
  auto* G = new GalerkinDevice();
  if (window_cols > 0) G->window = std::min(window_cols, gal::kMaxWindowCols);
  hipError_t e = hipGetDevice(&G->device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&G->st, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&G->dl, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete G;
    gal::check(e, "stream");
  }
  return G;
}

void galerkin_device_destroy(GalerkinDevice* G) { delete G; }

void galerkin_device(void* ctx, const BlockCSR& A, const ScalarCSR& P, BlockCSR& Ac, bool coarsest) {
  auto& G = *static_cast<GalerkinDevice*>(ctx);
  if (A.d == 2)
    gal::galerkin_d<2>(G, A, P, Ac, coarsest);
  else
    gal::galerkin_d<3>(G, A, P, Ac, coarsest);
}

void galerkin_device_start_downloads(GalerkinDevice* G, bool free_after) {
  for (const auto& p : G->pending)
    G->downloads.emplace_back(gal::download_values, G, p.level, p.host, free_after);
  G->pending.clear();
}

void galerkin_device_join(GalerkinDevice* G) {
  galerkin_device_start_downloads(G, false);
  G->join();
  std::lock_guard<std::mutex> g(G->mu);
  if (!G->dl_error.empty()) throw Error{VASMG_EDEVICE, G->dl_error};
}

bool galerkin_device_operator(const GalerkinDevice* G, int l, DevOperator* out) {
  if (!G || l < 0 || l >= static_cast<int>(G->lev.size())) return false;
  const gal::DevCsr& L = G->lev[l];
  *out = DevOperator{L.nrows, L.ptr, L.col, L.val};
  return true;
}

void* galerkin_device_stream(const GalerkinDevice* G) { return G ? static_cast<void*>(G->st) : nullptr; }

void layout_count(const DevOperator& A, const LayoutArgs& a, int* cntL, int* cntU, void* stream) {
  if (A.n != a.n) throw Error{VASMG_EINVAL, "internal: layout operator size"};
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int grid = (a.n + gal::kWaves - 1) / gal::kWaves;
  if (a.n > 0)
    hipLaunchKernelGGL(gal::k_layout_count, dim3(grid), dim3(gal::kThreads), 0, st, a.n,
                       gal::Csr{A.ptr, A.col, A.val}, a.perm, a.inv, a.lo, a.hi, cntL, cntU);
  gal::check(hipGetLastError(), "layout count launch");
  gal::check(hipStreamSynchronize(st), "layout count");
}

void layout_fill(const DevOperator& A, const LayoutArgs& a, void* stream) {
  if (A.n != a.n) throw Error{VASMG_EINVAL, "internal: layout operator size"};
  if (a.d != 2 && a.d != 3) throw Error{VASMG_EINVAL, "internal: layout dimension"};
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (a.M32) gal::check(hipMemsetAsync(a.M32, 0, a.m_len * sizeof(float), st), "clear");
  if (a.M64) gal::check(hipMemsetAsync(a.M64, 0, a.m_len * sizeof(double), st), "clear");
  const int grid = (a.n + gal::kWaves - 1) / gal::kWaves;
  const gal::Csr op{A.ptr, A.col, A.val};
  if (a.n > 0) {
    if (a.d == 2)
      hipLaunchKernelGGL(gal::k_layout_fill<2>, dim3(grid), dim3(gal::kThreads), 0, st, op, a);
    else
      hipLaunchKernelGGL(gal::k_layout_fill<3>, dim3(grid), dim3(gal::kThreads), 0, st, op, a);
  }
  gal::check(hipGetLastError(), "layout fill launch");
  gal::check(hipStreamSynchronize(st), "layout fill");
}

}  // namespace vasmg
