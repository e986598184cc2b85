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
#include <future>
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
// NT threads per row: 64 for A P, whose rows hold a few dozen blocks (a larger
// workgroup would leave most of its wavefronts idle and fewer rows resident).
template <int D, bool XB, int NT>
__global__ __launch_bounds__(NT) void k_numeric(int32_t nrows, Csr X, Csr Y,
                                                      const int64_t* __restrict__ cptr,
                                                      const int32_t* __restrict__ ccol,
                                                      double* __restrict__ cval) {
  constexpr int DD = D * D;
  const int32_t i = blockIdx.x;
  if (i >= nrows) return;
  const int64_t cb = cptr[i], ce = cptr[i + 1];
  const int64_t xb = X.ptr[i], xe = X.ptr[i + 1];
  for (int64_t s0 = cb; s0 < ce; s0 += NT) {
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
      // Y's rows hold distinct columns in ascending order: at most one entry
      // matches, found by bisection
      int64_t lo = qb, hi = qe;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (Y.col[mid] < my)
          lo = mid + 1;
        else
          hi = mid;
      }
      if (lo < qe && Y.col[lo] == my) add(lo);
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
  hipStream_t sd = nullptr;   // structure downloads (beside the next product)
  int window = gal::kMaxWindowCols;
  const BlockCSR* cached = nullptr;   // host operator of the last resident level
  std::vector<gal::DevCsr> lev;       // resident canonical operators, by level
  std::vector<gal::DevCsr> adopted;   // prolongations built on the device, by level
  std::vector<int64_t> adopted_cols;
  std::vector<gal::DevCsr> kept;      // each level's prolongation after its product,
  std::vector<int64_t> kept_cols;     // for the device-numbered transfers of the upload
  struct Pending {
    int level;
    BlockCSR* host;
  };
  std::vector<Pending> pending;       // value downloads not started yet
  // each product's structure (and the coarsest's values) on its way to the host,
  // by level; the next product runs meanwhile
  std::vector<std::shared_future<void>> structure;   // guarded by smu
  std::mutex smu;
  // level < 0: all; rethrows a download's error. Any thread: it waits on copies
  // of the futures taken under the lock (the products append to the list).
  void wait_structure(int level) {
    std::vector<std::shared_future<void>> w;
    {
      std::lock_guard<std::mutex> g(smu);
      for (size_t k = 0; k < structure.size(); ++k)
        if ((level < 0 || static_cast<int>(k) == level) && structure[k].valid()) w.push_back(structure[k]);
    }
    for (auto& f : w) f.get();
  }
  std::vector<std::thread> downloads;
  std::mutex mu;
  std::string dl_error;
  void join() {
    for (auto& t : downloads)
      if (t.joinable()) t.join();
    downloads.clear();
  }
  ~GalerkinDevice() {
    for (auto& f : structure)   // the device copies they read stay until they end
      if (f.valid()) f.wait();
    join();   // downloads not started by now are not needed
    for (auto& L : lev) L.release(st);
    for (auto& P : adopted) P.release(st);
    for (auto& P : kept) P.release(st);
    if (st) (void)hipStreamSynchronize(st);
    if (st) (void)hipStreamDestroy(st);
    if (dl) (void)hipStreamDestroy(dl);
    if (sd) (void)hipStreamDestroy(sd);
  }
};

namespace gal {

// Maps the pages of a freshly sized host array from several threads (one write
// per page), so that the kernel's page faults and page clearing are spread
// over cores instead of falling on the single thread that copies into it.
void first_touch(void* p, size_t bytes) {
  constexpr size_t kPage = 4096;
  constexpr int kThreads = 8;
  if (bytes < (size_t(16) << 20)) return;
  char* b = static_cast<char*>(p);
  std::vector<std::thread> th;
  th.reserve(kThreads);
  for (int t = 0; t < kThreads; ++t) {
    const size_t lo = bytes * t / kThreads, hi = bytes * (t + 1) / kThreads;
    th.emplace_back([b, lo, hi] {
      for (size_t o = lo; o < hi; o += kPage) reinterpret_cast<volatile char*>(b)[o] = 0;
    });
  }
  for (auto& x : th) x.join();
}

template <class ColV>   // std::vector<int32_t> or ColVec
void upload(DevCsr& D, int64_t nrows, const std::vector<int64_t>& ptr, const ColV& col,
            const std::vector<double>& val, hipStream_t st) {
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
  struct FreeCounts {   // released on every path; C itself is the caller's
    int64_t* p;
    hipStream_t st;
    ~FreeCounts() { (void)hipFreeAsync(p, st); }
  } free_counts{cnt, st};
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
    constexpr int NT = XB ? 64 : kThreads;
    hipLaunchKernelGGL((k_numeric<D, XB, NT>), dim3(n32), dim3(NT), 0, st, n32, X.view(),
                       Y.view(), C.ptr, C.col, C.val);
    check(hipGetLastError(), "numeric launch");
  }
  check(hipStreamSynchronize(st), "product");
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
  const size_t l = G.lev.size() - 1;
  DevCsr dP, dPT, AP, C;
  if (l < G.adopted.size() && G.adopted[l].ptr && G.adopted[l].nrows == P.nrows &&
      G.adopted[l].nnz == static_cast<int64_t>(P.col.size()) && G.adopted_cols[l] == P.ncols) {
    // P already on the device (device tree build): its transpose built there too
    dP = G.adopted[l];
    G.adopted[l] = DevCsr();
    dPT.nrows = P.ncols;
    dPT.nnz = dP.nnz;
    try {
      dPT.ptr = dmalloc<int64_t>(P.ncols + 1, st, "rowptr");
      dPT.col = dmalloc<int32_t>(dP.nnz, st, "columns");
      dPT.val = dmalloc<double>(dP.nnz, st, "values");
      transpose_device(st, dP.nrows, P.ncols, dP.nnz, dP.ptr, dP.col, dP.val, dPT.ptr, dPT.col, dPT.val);
    } catch (...) {
      dP.release(st);
      dPT.release(st);
      throw;
    }
  }
  // else P and its transpose (rows = coarse vertices), built on the host: <= 2^d
  // entries per P row
  ScalarCSR PT;
  if (!dP.ptr) {
    PT.nrows = P.ncols;
    PT.ncols = P.nrows;
    PT.rowptr.assign(P.ncols + 1, 0);
    for (int32_t c : P.col) PT.rowptr[c + 1]++;
    for (int64_t r = 0; r < P.ncols; ++r) PT.rowptr[r + 1] += PT.rowptr[r];
    PT.col.resize(P.col.size());
    PT.val.resize(P.col.size());
    std::vector<int64_t> fill(PT.rowptr.begin(), PT.rowptr.end() - 1);
    for (int64_t r = 0; r < P.nrows; ++r)
      for (int64_t p = P.rowptr[r]; p < P.rowptr[r + 1]; ++p) {
        const int64_t q = fill[P.col[p]]++;
        PT.col[q] = static_cast<int32_t>(r);
        PT.val[q] = P.val[p];
      }
  }
  try {
    if (!dP.ptr) {
      upload(dP, P.nrows, P.rowptr, P.col, P.val, st);
      upload(dPT, PT.nrows, PT.rowptr, PT.col, PT.val, st);
    }
    product<D, true>(G, dA, dP, P.ncols, AP);
    product<D, false>(G, dPT, AP, P.ncols, C);
    Ac.n = P.ncols;
    Ac.d = D;
    // the structure (and the coarsest's values) goes to the host on a thread of
    // its own while the next product runs; whoever reads it first waits for it
    // (galerkin_device_wait_structure). C stays resident until the download ends.
    GalerkinDevice* Gp = &G;
    const DevCsr Cs = C;
    BlockCSR* host = &Ac;
    std::lock_guard<std::mutex> guard(G.smu);
    if (G.structure.size() <= l + 1) G.structure.resize(l + 2);
    G.structure[l + 1] = std::async(std::launch::async, [Gp, Cs, host, coarsest] {
                           check(hipSetDevice(Gp->device), "device");
                           host->rowptr.resize(Cs.nrows + 1);
                           host->col.resize(Cs.nnz);   // not cleared: the copy fills it
                           first_touch(host->col.data(), Cs.nnz * sizeof(int32_t));
                           check(hipMemcpyAsync(host->rowptr.data(), Cs.ptr, (Cs.nrows + 1) * sizeof(int64_t),
                                                hipMemcpyDeviceToHost, Gp->sd), "copy");
                           check(hipMemcpyAsync(host->col.data(), Cs.col, Cs.nnz * sizeof(int32_t),
                                                hipMemcpyDeviceToHost, Gp->sd), "copy");
                           if (coarsest) {
                             host->val.resize(Cs.nnz * DD);
                             check(hipMemcpyAsync(host->val.data(), Cs.val, Cs.nnz * DD * sizeof(double),
                                                  hipMemcpyDeviceToHost, Gp->sd), "copy");
                           }
                           check(hipStreamSynchronize(Gp->sd), "structure download");
                         }).share();
  } catch (...) {
    dP.release(st);
    dPT.release(st);
    AP.release(st);
    C.release(st);
    throw;
  }
  // P stays for the upload's device-numbered transfers (canonical rows and columns)
  if (G.kept.size() <= l) {
    G.kept.resize(l + 1);
    G.kept_cols.resize(l + 1, 0);
  }
  G.kept[l].release(st);
  G.kept[l] = dP;
  G.kept_cols[l] = P.ncols;
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

// Part of an off-cell block in device column j of a row with cell [lo, hi)
// and colour block [blo, bhi); -1 inside the cell.
__device__ __forceinline__ int layout_part(int j, int lo, int hi, int blo, int bhi) {
  if (j >= lo && j < hi) return -1;
  if (j < blo) return kPartL;
  if (j < lo) return kPartE;
  if (j < bhi) return kPartF;
  return kPartU;
}

// Off-cell blocks of each part. One wavefront per device row.
__global__ __launch_bounds__(kThreads) void k_layout_count(int n, Csr A, LayoutArgs a) {
  const int i = blockIdx.x * kWaves + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  const int c = a.perm[i];
  const int lo = a.lo[i], hi = a.hi[i];
  const int blo = a.blo ? a.blo[i] : lo, bhi = a.bhi ? a.bhi[i] : hi;
  int cnt[kParts] = {0, 0, 0, 0};
  for (int64_t p = A.ptr[c] + lane; p < A.ptr[c + 1]; p += 64) {
    const int q = layout_part(a.inv[A.col[p]], lo, hi, blo, bhi);
#pragma unroll
    for (int k = 0; k < kParts; ++k) cnt[k] += q == k;
  }
#pragma unroll
  for (int k = 0; k < kParts; ++k)
    for (int o = 32; o > 0; o >>= 1) cnt[k] += __shfl_xor(cnt[k], o, 64);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < kParts; ++k)
      if (a.part[k].cnt) a.part[k].cnt[i] = cnt[k];
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
  const int blo = a.blo ? a.blo[i] : lo, bhi = a.bhi ? a.bhi[i] : hi;
  auto col_of = [&](int e) { return staged ? sj[w][e] : a.inv[A.col[rb + e]]; };
  for (int e = lane; e < len; e += 64) {
    const int j = col_of(e);
    const double* blk = A.val + (rb + e) * DD;
    const int pq = layout_part(j, lo, hi, blo, bhi);
    if (pq >= 0) {
      int rank = 0;
      for (int f = 0; f < len; ++f) {
        const int jf = col_of(f);
        rank += jf < j && layout_part(jf, lo, hi, blo, bhi) == pq;
      }
      const LayoutPart& P = a.part[pq];
      const int64_t q = P.ptr[i] + rank;
      P.col[q] = j;
#pragma unroll
      for (int t = 0; t < DD; ++t) {
        if (P.v64) P.v64[t * P.n + q] = blk[t];
        if (P.v32) P.v32[t * P.n + q] = static_cast<float>(blk[t]);
      }
    } else if (a.cell_of_row) {
      const int64_t base = static_cast<int64_t>(a.cell_of_row[i]) * NU * NU;
      const int ki = i - lo, kj = j - lo;
      const int fx = (j == i && a.fixed) ? a.fixed[i] : 0;
#pragma unroll
      for (int r = 0; r < D; ++r)
#pragma unroll
        for (int s = 0; s < D; ++s) {
          const int64_t m = base + (kj * D + s) * NU + (ki * D + r);
          const double v = (r == s && ((fx >> r) & 1)) ? 1.0 : blk[r * D + s];
          if (a.M64) a.M64[m] = v;
          if (a.M32) a.M32[m] = static_cast<float>(v);
        }
    } else {
      const int fx = (j == i && a.fixed) ? a.fixed[i] : 0;
#pragma unroll
      for (int t = 0; t < DD; ++t) {
        const double v = (t / D == t % D && ((fx >> (t / D)) & 1)) ? 1.0 : blk[t];
        if (a.M64) a.M64[static_cast<int64_t>(i) * DD + t] = v;
        if (a.M32) a.M32[static_cast<int64_t>(i) * DD + t] = static_cast<float>(v);
      }
    }
  }
  // padding of the rows' parts: column i, zero blocks
  for (int pq = 0; pq < kParts; ++pq) {
    const LayoutPart& P = a.part[pq];
    if (!P.cnt) continue;
    const int64_t b = P.ptr[i] + P.cnt[i];
    const int64_t e = P.ptr[i + 1];
    for (int64_t q = b + lane; q < e; q += 64) {
      P.col[q] = i;
      for (int t = 0; t < DD; ++t) {
        if (P.v64) P.v64[t * P.n + q] = 0.0;
        if (P.v32) P.v32[t * P.n + q] = 0.0f;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// fine-level assembly (Section 2: the P1 element stiffness of linear
// elasticity, summed element by element). This file is built without
// floating-point contraction, and the arithmetic below follows the host
// assembly operation by operation, so the values agree bit for bit.
// ---------------------------------------------------------------------------
struct MeshDev {
  int d = 0, nvpe = 0;
  const double* coords = nullptr;    // [nv][d]
  const int32_t* elems = nullptr;    // [ne][d+1]
  const double* E = nullptr;         // [ne]
  const double* nu = nullptr;        // [ne]
  const int32_t* vfree = nullptr;    // mesh vertex -> free index or -1
  const int32_t* fine2mesh = nullptr;
  const int64_t* vptr = nullptr;     // vertex -> elements (ascending)
  const int32_t* velem = nullptr;
};

constexpr int kAsmStage = 512;   // element corners of one row staged in LDS

// Zeroes the rows and columns of constrained components (fixed[row] bit a =
// component a of that vertex). One thread per stored block.
template <int D>
__global__ __launch_bounds__(kThreads) void k_zero_constrained(int64_t n, const int64_t* __restrict__ ptr,
                                                              const int32_t* __restrict__ col,
                                                              double* __restrict__ val,
                                                              const uint8_t* __restrict__ fixed) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(kWaves) + (threadIdx.x >> 6);
  if (i >= n) return;
  const uint8_t fr = fixed[i];
  for (int64_t p = ptr[i] + (threadIdx.x & 63); p < ptr[i + 1]; p += 64) {
    const uint8_t fc = fixed[col[p]];
    if (!fr && !fc) continue;
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = 0; b < D; ++b)
        if (((fr >> a) & 1) || ((fc >> b) & 1)) val[p * D * D + a * D + b] = 0.0;
  }
}

// Free index of corner c of row i's element list (c = element slot * (d+1) + corner).
__device__ __forceinline__ int asm_corner(const MeshDev& M, int64_t kb, int c) {
  const int e = M.velem[kb + c / M.nvpe];
  return M.vfree[M.elems[static_cast<int64_t>(e) * M.nvpe + c % M.nvpe]];
}

// Distinct free vertices sharing an element with row i's vertex (itself
// included): counted (FILL = false) or written ascending (FILL = true). One
// wavefront per row; a corner counts if no earlier corner names the same vertex.
template <bool FILL>
__global__ __launch_bounds__(kThreads) void k_asm_pattern(int n, MeshDev M, int64_t* __restrict__ cnt,
                                                          const int64_t* __restrict__ rowptr,
                                                          int32_t* __restrict__ col) {
  __shared__ int sc[kWaves][kAsmStage];   // corners
  __shared__ int sf[kWaves][kAsmStage];   // the vertex at its first occurrence, else -1
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * kWaves + w;
  const bool valid = i < n;
  const int v = valid ? M.fine2mesh[i] : 0;
  const int64_t kb = valid ? M.vptr[v] : 0, ke = valid ? M.vptr[v + 1] : 0;
  const int T = static_cast<int>(ke - kb) * M.nvpe;
  const bool staged = T <= kAsmStage;
  auto corner = [&](int c) { return staged ? sc[w][c] : asm_corner(M, kb, c); };
  auto first = [&](int c) {   // vertex of corner c if it is its first occurrence, else -1
    const int f = corner(c);
    if (f < 0) return -1;
    for (int c2 = 0; c2 < c; ++c2)
      if (corner(c2) == f) return -1;
    return f;
  };
  if (staged)
    for (int c = lane; c < T; c += 64) sc[w][c] = asm_corner(M, kb, c);
  __syncthreads();
  if (staged)
    for (int c = lane; c < T; c += 64) sf[w][c] = first(c);
  __syncthreads();
  if (!valid) return;
  auto first_of = [&](int c) { return staged ? sf[w][c] : first(c); };
  int count = 0;
  for (int c = lane; c < T; c += 64) {
    const int f = first_of(c);
    if (f < 0) continue;
    ++count;
    if (FILL) {
      int rank = 0;
      for (int c2 = 0; c2 < T; ++c2) {
        const int g = first_of(c2);
        rank += g >= 0 && g < f;
      }
      col[rowptr[i] + rank] = f;
    }
  }
  if (!FILL) {
    for (int o = 32; o > 0; o >>= 1) count += __shfl_xor(count, o, 64);
    if (lane == 0) cnt[i] = count;
  }
}

// Gradients of the barycentric functions of one element and the signed
// determinant of its edge matrix X (rows x_a - x_0): grad lambda_a = row a of
// X^{-T}, grad lambda_0 = -(sum of the others); inverse by cofactors.
template <int D>
__device__ __forceinline__ double asm_grads(const double* const* xs, double G[4][3]) {
  double X[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int a = 0; a < D; ++a)
    for (int k = 0; k < D; ++k) X[a][k] = xs[a + 1][k] - xs[0][k];
  double det, inv[3][3];
  if (D == 2) {
    det = X[0][0] * X[1][1] - X[0][1] * X[1][0];
    inv[0][0] = X[1][1] / det;
    inv[0][1] = -X[0][1] / det;
    inv[1][0] = -X[1][0] / det;
    inv[1][1] = X[0][0] / det;
  } else {
    const double c00 = X[1][1] * X[2][2] - X[1][2] * X[2][1];
    const double c01 = X[1][2] * X[2][0] - X[1][0] * X[2][2];
    const double c02 = X[1][0] * X[2][1] - X[1][1] * X[2][0];
    det = X[0][0] * c00 + X[0][1] * c01 + X[0][2] * c02;
    inv[0][0] = c00 / det;
    inv[1][0] = c01 / det;
    inv[2][0] = c02 / det;
    inv[0][1] = (X[0][2] * X[2][1] - X[0][1] * X[2][2]) / det;
    inv[1][1] = (X[0][0] * X[2][2] - X[0][2] * X[2][0]) / det;
    inv[2][1] = (X[0][1] * X[2][0] - X[0][0] * X[2][1]) / det;
    inv[0][2] = (X[0][1] * X[1][2] - X[0][2] * X[1][1]) / det;
    inv[1][2] = (X[0][2] * X[1][0] - X[0][0] * X[1][2]) / det;
    inv[2][2] = (X[0][0] * X[1][1] - X[0][1] * X[1][0]) / det;
  }
  for (int a = 0; a < D; ++a)
    for (int k = 0; k < D; ++k) G[a + 1][k] = inv[k][a];
  for (int k = 0; k < D; ++k) {
    double s = 0.0;
    for (int a = 1; a <= D; ++a) s += G[a][k];
    G[0][k] = -s;
  }
  return det;
}

// Values of row i: lane q owns block (i, col q) and adds, element by element in
// ascending order, vol (mu (grad_a . grad_b) delta_ij + mu d_j phi_a d_i phi_b +
// lambda d_i phi_a d_j phi_b) for the element's corner b at that column.
template <int D>
__global__ __launch_bounds__(kThreads) void k_asm_values(int n, MeshDev M,
                                                         const int64_t* __restrict__ rowptr,
                                                         const int32_t* __restrict__ col,
                                                         double* __restrict__ val) {
  constexpr int DD = D * D, NV = D + 1;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * kWaves + w;
  if (i >= n) return;
  const int v = M.fine2mesh[i];
  const int64_t kb = M.vptr[v], ke = M.vptr[v + 1];
  const int64_t rb = rowptr[i], re = rowptr[i + 1];
  for (int64_t q = rb + lane; q < re; q += 64) {
    const int j = col[q];
    double acc[DD];
    for (int t = 0; t < DD; ++t) acc[t] = 0.0;
    for (int64_t k = kb; k < ke; ++k) {
      const int e = M.velem[k];
      const int32_t* ev = M.elems + static_cast<int64_t>(e) * NV;
      int hit = -1, la = 0;
      for (int a = 0; a < NV; ++a) {
        if (ev[a] == v) la = a;
        if (M.vfree[ev[a]] == j) hit = a;
      }
      if (hit < 0) continue;
      const double* xs[4];
      for (int a = 0; a < NV; ++a) xs[a] = M.coords + static_cast<int64_t>(ev[a]) * D;
      double G[4][3];
      const double det = asm_grads<D>(xs, G);
      const double vol = fabs(det) / (D == 2 ? 2.0 : 6.0);
      const double E = M.E[e], nu = M.nu[e];
      const double mu = E / (2.0 * (1.0 + nu));
      const double lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
      const int b = hit;
      double gab = 0.0;
      for (int k2 = 0; k2 < D; ++k2) gab += G[la][k2] * G[b][k2];
      for (int ci = 0; ci < D; ++ci)
        for (int cj = 0; cj < D; ++cj) {
          double t = mu * G[la][cj] * G[b][ci] + lam * G[la][ci] * G[b][cj];
          if (ci == cj) t += mu * gab;
          acc[ci * D + cj] += vol * t;
        }
    }
    for (int t = 0; t < DD; ++t) val[q * DD + t] = acc[t];
  }
}

template <typename T>
const T* upload_temp(const std::vector<T>& v, hipStream_t st, std::vector<void*>& owned) {
  T* p = dmalloc<T>(v.size(), st, "mesh");
  owned.push_back(p);
  if (!v.empty())
    check(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st), "copy");
  return p;
}

template <typename T>
const T* upload_temp(const T* v, size_t count, hipStream_t st, std::vector<void*>& owned) {
  T* p = dmalloc<T>(count, st, "mesh");
  owned.push_back(p);
  if (count) check(hipMemcpyAsync(p, v, count * sizeof(T), hipMemcpyHostToDevice, st), "copy");
  return p;
}

}  // namespace gal

GalerkinDevice* galerkin_device_create(int window_cols) {
  auto* G = new GalerkinDevice();
  if (window_cols > 0) G->window = std::min(window_cols, gal::kMaxWindowCols);
  hipError_t e = hipGetDevice(&G->device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&G->st, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&G->dl, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&G->sd, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete G;
    gal::check(e, "stream");
  }
  return G;
}

void galerkin_device_destroy(GalerkinDevice* G) { delete G; }

void galerkin_device_adopt_prolongation(GalerkinDevice* G, int level, int64_t nrows, int64_t ncols,
                                        int64_t nnz, int64_t* ptr, int32_t* col, double* val) {
  if (level < 0) return;
  if (static_cast<size_t>(level) >= G->adopted.size()) {
    G->adopted.resize(level + 1);
    G->adopted_cols.resize(level + 1, 0);
  }
  G->adopted[level].release(G->st);
  gal::DevCsr& D = G->adopted[level];
  D.nrows = nrows;
  D.nnz = nnz;
  D.ptr = ptr;
  D.col = col;
  D.val = val;
  G->adopted_cols[level] = ncols;
}

void galerkin_device(void* ctx, const BlockCSR& A, const ScalarCSR& P, BlockCSR& Ac, bool coarsest) {
  auto& G = *static_cast<GalerkinDevice*>(ctx);
  if (A.d == 2)
    gal::galerkin_d<2>(G, A, P, Ac, coarsest);
  else
    gal::galerkin_d<3>(G, A, P, Ac, coarsest);
}

void assemble_device(void* ctx, const MeshView& m, const std::vector<int32_t>& vfree,
                     int64_t nfree, BlockCSR& A) {
  auto& G = *static_cast<GalerkinDevice*>(ctx);
  if (!G.lev.empty()) throw Error{VASMG_EINVAL, "internal: device assembly after other levels"};
  if (nfree > INT32_MAX || m.ne > INT32_MAX)
    throw Error{VASMG_EINVAL, "mesh too large for int32 indexing"};
  hipStream_t st = G.st;
  const int d = m.d, nvpe = d + 1, dd = d * d;
  const int n = static_cast<int>(nfree);
  std::vector<int32_t> f2m(nfree);
  for (int64_t v = 0; v < m.nv; ++v)
    if (vfree[v] >= 0) f2m[vfree[v]] = static_cast<int32_t>(v);
  std::vector<void*> owned;
  std::vector<uint8_t> fx;   // constrained components per fine row (stays until the copies end)
  gal::DevCsr A0;
  auto release_temps = [&] {
    for (void* p : owned) (void)hipFreeAsync(p, st);
    owned.clear();
  };
  try {
    gal::MeshDev M;
    M.d = d;
    M.nvpe = nvpe;
    M.coords = gal::upload_temp(m.coords, static_cast<size_t>(m.nv) * d, st, owned);
    M.elems = gal::upload_temp(m.elems, static_cast<size_t>(m.ne) * nvpe, st, owned);
    M.E = gal::upload_temp(m.E, static_cast<size_t>(m.ne), st, owned);
    M.nu = gal::upload_temp(m.nu, static_cast<size_t>(m.ne), st, owned);
    M.vfree = gal::upload_temp(vfree, st, owned);
    M.fine2mesh = gal::upload_temp(f2m, st, owned);
    {   // vertex -> element lists, built on the device
      int64_t* vp = gal::dmalloc<int64_t>(m.nv + 1, st, "vertex elements");
      owned.push_back(vp);
      int32_t* ve = gal::dmalloc<int32_t>(m.ne * nvpe, st, "vertex elements");
      owned.push_back(ve);
      vertex_elements_device(st, M.elems, m.ne, nvpe, m.nv, vp, ve);
      M.vptr = vp;
      M.velem = ve;
    }
    const int grid = (n + gal::kWaves - 1) / gal::kWaves;
    int64_t* cnt = gal::dmalloc<int64_t>(n, st, "row counts");
    owned.push_back(cnt);
    if (n > 0)
      hipLaunchKernelGGL(gal::k_asm_pattern<false>, dim3(grid), dim3(gal::kThreads), 0, st, n, M,
                         cnt, nullptr, nullptr);
    gal::check(hipGetLastError(), "assembly pattern launch");
    A.n = nfree;
    A.d = d;
    A.rowptr.assign(nfree + 1, 0);
    gal::check(hipMemcpyAsync(A.rowptr.data() + 1, cnt, n * sizeof(int64_t), hipMemcpyDeviceToHost, st),
               "copy");
    gal::check(hipStreamSynchronize(st), "assembly pattern");
    for (int64_t r = 0; r < nfree; ++r) A.rowptr[r + 1] += A.rowptr[r];
    const int64_t nnz = A.rowptr[nfree];
    A0.nrows = nfree;
    A0.nnz = nnz;
    A0.ptr = gal::dmalloc<int64_t>(nfree + 1, st, "rowptr");
    A0.col = gal::dmalloc<int32_t>(nnz, st, "columns");
    A0.val = gal::dmalloc<double>(nnz * dd, st, "values");
    gal::check(hipMemcpyAsync(A0.ptr, A.rowptr.data(), (nfree + 1) * sizeof(int64_t),
                              hipMemcpyHostToDevice, st), "copy");
    if (n > 0) {
      hipLaunchKernelGGL(gal::k_asm_pattern<true>, dim3(grid), dim3(gal::kThreads), 0, st, n, M,
                         nullptr, A0.ptr, A0.col);
      gal::check(hipGetLastError(), "assembly columns launch");
      if (d == 2)
        hipLaunchKernelGGL(gal::k_asm_values<2>, dim3(grid), dim3(gal::kThreads), 0, st, n, M, A0.ptr,
                           A0.col, A0.val);
      else
        hipLaunchKernelGGL(gal::k_asm_values<3>, dim3(grid), dim3(gal::kThreads), 0, st, n, M, A0.ptr,
                           A0.col, A0.val);
      gal::check(hipGetLastError(), "assembly values launch");
      // vertices with some components fixed: zero rows and columns there
      fx.assign(nfree, 0);
      bool any = false;
      for (int64_t r = 0; r < nfree; ++r) {
        for (int a = 0; a < d; ++a)
          if (m.fixed[static_cast<int64_t>(f2m[r]) * d + a]) fx[r] |= static_cast<uint8_t>(1u << a);
        any = any || fx[r] != 0;
      }
      if (any) {
        const uint8_t* dfx = gal::upload_temp(fx, st, owned);
        if (d == 2)
          hipLaunchKernelGGL(gal::k_zero_constrained<2>, dim3(grid), dim3(gal::kThreads), 0, st,
                             static_cast<int64_t>(n), A0.ptr, A0.col, A0.val, dfx);
        else
          hipLaunchKernelGGL(gal::k_zero_constrained<3>, dim3(grid), dim3(gal::kThreads), 0, st,
                             static_cast<int64_t>(n), A0.ptr, A0.col, A0.val, dfx);
        gal::check(hipGetLastError(), "constrained rows launch");
      }
    }
    A.col.resize(nnz);
    gal::check(hipMemcpyAsync(A.col.data(), A0.col, nnz * sizeof(int32_t), hipMemcpyDeviceToHost, st),
               "copy");
    gal::check(hipStreamSynchronize(st), "assembly");
  } catch (...) {
    release_temps();
    A0.release(st);
    throw;
  }
  release_temps();
  G.lev.push_back(A0);
  G.cached = &A;
  G.pending.push_back({0, &A});
}

void galerkin_device_settle(void* ctx) { galerkin_device_join(static_cast<GalerkinDevice*>(ctx)); }

void galerkin_device_wait_structure(void* ctx, int level) {
  static_cast<GalerkinDevice*>(ctx)->wait_structure(level);
}

void galerkin_device_start_downloads(GalerkinDevice* G, bool free_after) {
  G->wait_structure(-1);   // value downloads may free the levels these read
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

bool galerkin_device_prolongation(GalerkinDevice* G, int level, int64_t* nrows, int64_t* ncols,
                                  int64_t* nnz, const int64_t** ptr, const int32_t** col,
                                  const double** val) {
  if (!G || level < 0 || static_cast<size_t>(level) >= G->kept.size() || !G->kept[level].ptr)
    return false;
  const gal::DevCsr& P = G->kept[level];
  *nrows = P.nrows;
  *ncols = G->kept_cols[level];
  *nnz = P.nnz;
  *ptr = P.ptr;
  *col = P.col;
  *val = P.val;
  return true;
}

void galerkin_device_release_prolongation(GalerkinDevice* G, int level) {
  if (G && level >= 0 && static_cast<size_t>(level) < G->kept.size()) G->kept[level].release(G->st);
}

void layout_count(const DevOperator& A, const LayoutArgs& a, void* stream) {
  if (A.n != a.n) throw Error{VASMG_EINVAL, "internal: layout operator size"};
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int grid = (a.n + gal::kWaves - 1) / gal::kWaves;
  if (a.n > 0)
    hipLaunchKernelGGL(gal::k_layout_count, dim3(grid), dim3(gal::kThreads), 0, st, a.n,
                       gal::Csr{A.ptr, A.col, A.val}, a);
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
