// Device hierarchy, V-cycle schedule, PCG driver and the C ABI of libvasmg.
//
// Solve phase of arXiv 2505.09064: PCG (Section 2.2, Algorithm 2) with one
// V-cycle (Section 3, Algorithm 3 applied recursively) as the preconditioner.
// All steps run in the kernels of kernels.hpp. One PCG iteration is split in
// two captured hipGraphs:
//   graph A: q = A p with p.q partials, alpha, x += alpha p, r -= alpha q with
//            ||r||^2 partials (and the FP32 copy of r), convergence flag;
//   graph B: z = B r (the V-cycle), r.z partials, beta, p = z + beta p.
// The host reads the device flag after graph A (the only per-iteration sync).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <chrono>
#include <mutex>
#include <numeric>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/vasmg.h"
#include "hierarchy.hpp"
#include "kernels.hpp"
#include "block.hpp"
#include "packed.hpp"

using namespace vasmg;
using dev::Scalars;

namespace {

thread_local std::string g_last_error;
std::atomic<int> g_galerkin_window{0};   // test hook: device Galerkin window (0 = max)

#define HIP_CHECK(expr)                                                                    \
  do {                                                                                     \
    hipError_t _e = (expr);                                                                \
    if (_e != hipSuccess)                                                                  \
      throw vasmg::Error{VASMG_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)}; \
  } while (0)

inline int pow2_ceil(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

inline int grid_for(int64_t items, int per_block) {
  return static_cast<int>(std::max<int64_t>(1, (items + per_block - 1) / per_block));
}

constexpr int kFlatGrid = 1024;   // fixed grid of the flat reduction kernels

// -------------------------------------------------------------------------
struct DevLevel {
  int n = 0;
  int d = 0;
  int ncolors = 0;
  int64_t nnz = 0;                 // off-diagonal (point) or off-cell (cell) blocks
  int64_t nnz_lo = 0, nnz_up = 0;  // blocks coupling to earlier / later colours
  int64_t Lstride = 0, Ustride = 0; // stored L / U entries (plane stride; rows padded on cell levels)
  int64_t p_nnz = 0;               // entries of P_l
  int G = 8;                       // lanes per block row (Gauss-Seidel, residual)
  int Gspmv = 8;                   // lanes per block row of the fine FP64 SpMV
  int mcGL = 0;                    // block right-hand sides: lanes per block row
  std::vector<int> color_ptr;      // host: device rows (point levels) or cells (cell
                                   // levels) of colour c = [ptr[c], ptr[c+1])
  bool cells = false;              // coarse lattice level: Gauss-Seidel over cells
  int ncells = 0;
  int* cell_ptr = nullptr;         // cell levels: first device row of each cell
  // colour-block levels (cells grouped into blocks of several cells, a colour
  // per block): color_ptr then counts blocks, block_ptr gives each block's
  // first cell, and the off-cell blocks inside a row's colour block form the
  // parts E (earlier cells) and F (later cells)
  bool blocks = false;
  int nblocks = 0;
  int* block_ptr = nullptr;
  int *Eptr = nullptr, *Ecol = nullptr, *Fptr = nullptr, *Fcol = nullptr;
  float *Eval32 = nullptr, *Fval32 = nullptr;
  double *Eval64 = nullptr, *Fval64 = nullptr;
  int64_t nnz_e = 0, nnz_f = 0, Estride = 0, Fstride = 0;
  int* color_ptr_dev = nullptr;    // device copy of color_ptr (fused bottom levels only)
  float* cellM32 = nullptr;        // cell levels: dense in-cell blocks (column-major)
  double* cellM64 = nullptr;
  int* perm = nullptr;             // device row -> canonical index
  uint8_t* fixed = nullptr;        // constrained components per device row (null: none)
  // off-diagonal blocks to earlier colours (L) and to later colours (U)
  int *Lptr = nullptr, *Lcol = nullptr, *Uptr = nullptr, *Ucol = nullptr;
  float *Lval32 = nullptr, *Uval32 = nullptr;
  double *Lval64 = nullptr, *Uval64 = nullptr;
  float* diag32 = nullptr;
  double* diag64 = nullptr;
  // damped vertex-block Jacobi smoother (option smoother = JACOBI)
  float* dinv32 = nullptr;
  double* dinv64 = nullptr;
  double omega = 0.0;
  // prolongation to the next level (device numbering on both sides)
  int nnext = 0;
  int* p_ptr = nullptr;
  int* p_idx = nullptr;
  float* p_w32 = nullptr;
  double* p_w64 = nullptr;
  int* pt_ptr = nullptr;
  int* pt_idx = nullptr;
  float* pt_w32 = nullptr;
  double* pt_w64 = nullptr;
  // V-cycle work vectors (padded, V-cycle precision)
  void* b = nullptr;
  void* x = nullptr;
  void* s = nullptr;
  void* r = nullptr;
  bool has32 = false, has64 = false;
};

}  // namespace

// Pinned host blocks for the per-iteration scalar read-back. Freeing pinned
// memory synchronises the whole device (it would stall every other solve in
// flight), so blocks are recycled through this pool and never freed.
class PinnedPool {
 public:
  static constexpr size_t kBytes = 4096;
  static constexpr int kBatch = 64;
  void* get() {
    std::lock_guard<std::mutex> g(mu_);
    if (!free_.empty()) {
      void* p = free_.back();
      free_.pop_back();
      return p;
    }
    // one allocation per 64 blocks: pinned allocations are rare and early
    char* p = nullptr;
    if (hipHostMalloc(reinterpret_cast<void**>(&p), kBytes * kBatch) != hipSuccess)
      throw vasmg::Error{VASMG_ENOMEM, "pinned host allocation failed"};
    for (int i = kBatch - 1; i > 0; --i) free_.push_back(p + static_cast<size_t>(i) * kBytes);
    return p;
  }
  void put(void* p) {
    if (!p) return;
    std::lock_guard<std::mutex> g(mu_);
    free_.push_back(p);
  }

 private:
  std::mutex mu_;
  std::vector<void*> free_;
};

PinnedPool& pinned_pool() {
  static PinnedPool* pool = new PinnedPool;   // lives until the process ends
  return *pool;
}

struct vasmg_ctx {
  Hierarchy H;
  vasmg_options opt{};
  int d = 0, DP = 0;
  int L = 0;                        // index of the coarsest level
  bool host_only = true;
  bool vc32 = false;                // V-cycle precision FP32
  int device = 0;
  std::vector<void*> allocs;
  hipStream_t alloc_stream = nullptr;   // set: stream-ordered allocations on it
  int64_t dev_bytes = 0;                // device bytes allocated so far
  void* pinned = nullptr;               // pinned block: h_sc, h_rtol, kh_sc
  std::vector<DevLevel> lev;
  double* chol = nullptr;           // coarsest factor
  double* cinv = nullptr;           // coarsest inverse (small coarsest levels), else null
  // fused bottom (k_bottom): levels bottom_lo..L-1 and the coarsest solve in one
  // workgroup; -1 when the cycle has none
  int bottom_lo = -1;
  int64_t bottom_vec = 0, bottom_int = 0;   // its LDS elements: vectors (T), pointers (int)
  dev::BottomLevel<float>* bottom32 = nullptr;
  dev::BottomLevel<double>* bottom64 = nullptr;
  int64_t n_coarse = 0;
  double upload_ms[3] = {0.0, 0.0, 0.0};   // last upload's layouts, autotune, graph capture
  // PCG state (FP64, padded, fine device numbering)
  int n0 = 0;
  int64_t n0p = 0;                  // n0 * DP
  int* user_map = nullptr;          // fine device row -> mesh vertex
  double *F = nullptr, *X = nullptr, *R = nullptr, *P = nullptr, *Q = nullptr, *Z = nullptr;
  double* partial = nullptr;
  int n_partial = 0;
  Scalars* sc = nullptr;
  Scalars* h_sc = nullptr;          // pinned host copy
  double* h_rtol = nullptr;         // pinned
  int* zero_flag = nullptr;         // device int 0 (debug entry points)
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gA = nullptr, gB = nullptr;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  // block right-hand sides: K columns interleaved per vertex (K = 0: none)
  int K = 0;
  std::vector<void*> kb, kx, ks, kr;   // per level V-cycle vectors [n][K][DP]
  double *kF = nullptr, *kX = nullptr, *kR = nullptr, *kP = nullptr, *kQ = nullptr;
  double* kpartial = nullptr;
  int kn_partial = 0;                  // partial sums per column
  Scalars* ksc = nullptr;              // [K]
  Scalars* kh_sc = nullptr;            // pinned host copy [K]
  hipGraphExec_t kgA = nullptr, kgB = nullptr;
  GalerkinDevice* gdev = nullptr;     // setup_device = 1, during the upload only
  GalerkinDevice* gdev_bg = nullptr;  // owned: value downloads still running after setup
  // packed problems (vasmg_pack): nseg segments of the fine level, each with its
  // own PCG scalars (0: one problem)
  int nseg = 0;
  std::vector<int64_t> seg_vertex_off;   // [nseg + 1] mesh-vertex offsets of the parts
  std::vector<int64_t> seg_free_off;     // [nseg + 1] fine canonical vertex offsets
  int *seg_ptr = nullptr, *seg_rows = nullptr, *seg_of_row = nullptr;
  Scalars* ssc = nullptr;                // [nseg]
  int* seg_running = nullptr;            // segments still iterating
  hipGraphExec_t sgA = nullptr, sgB = nullptr;
  mutable std::vector<std::vector<int>> order_cache;   // device numbering per level (setup)

  template <class T>
  T* dalloc(int64_t count) {
    void* p = nullptr;
    if (count <= 0) count = 1;
    const size_t bytes = sizeof(T) * static_cast<size_t>(count);
    hipError_t e;
    if (alloc_stream) {
      e = hipMallocAsync(&p, bytes, alloc_stream);
      if (e == hipSuccess) e = hipStreamSynchronize(alloc_stream);
    } else {
      e = hipMalloc(&p, bytes);
    }
    if (e != hipSuccess)
      throw vasmg::Error{VASMG_ENOMEM, "device allocation of " + std::to_string(bytes) +
                                           " bytes failed: " + hipGetErrorString(e)};
    allocs.push_back(p);
    dev_bytes += static_cast<int64_t>(bytes);
    return static_cast<T*>(p);
  }
  // Setup-time copies and clears: on the allocation stream when there is one
  // (a server's handle must not touch the legacy null stream while other
  // handles capture graphs), else the synchronous calls.
  void copy(void* dst, const void* src, size_t bytes, hipMemcpyKind kind) {
    if (alloc_stream) {
      HIP_CHECK(hipMemcpyAsync(dst, src, bytes, kind, alloc_stream));
      HIP_CHECK(hipStreamSynchronize(alloc_stream));
    } else {
      HIP_CHECK(hipMemcpy(dst, src, bytes, kind));
    }
  }
  void clear(void* p, size_t bytes) {
    if (alloc_stream) {
      HIP_CHECK(hipMemsetAsync(p, 0, bytes, alloc_stream));
      HIP_CHECK(hipStreamSynchronize(alloc_stream));
    } else {
      HIP_CHECK(hipMemset(p, 0, bytes));
    }
  }
  template <class T>
  T* upload(const std::vector<T>& v) {
    T* p = dalloc<T>(static_cast<int64_t>(v.size()));
    if (!v.empty()) copy(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice);
    return p;
  }
  // Waits for the background downloads of the level values into H, if any.
  void settle_host_values() {
    if (!gdev_bg) return;
    GalerkinDevice* g = gdev_bg;
    gdev_bg = nullptr;
    std::unique_ptr<GalerkinDevice, void (*)(GalerkinDevice*)> own(g, galerkin_device_destroy);
    galerkin_device_join(g);
  }
  ~vasmg_ctx() {
    if (gdev_bg) galerkin_device_destroy(gdev_bg);   // joins the downloads writing into H
    if (gA) (void)hipGraphExecDestroy(gA);
    if (gB) (void)hipGraphExecDestroy(gB);
    if (kgA) (void)hipGraphExecDestroy(kgA);
    if (kgB) (void)hipGraphExecDestroy(kgB);
    if (sgA) (void)hipGraphExecDestroy(sgA);
    if (sgB) (void)hipGraphExecDestroy(sgB);
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (void* p : allocs) {
      if (alloc_stream)
        (void)hipFreeAsync(p, alloc_stream);
      else
        (void)hipFree(p);
    }
    pinned_pool().put(pinned);
  }
};

namespace {

// -------------------------------------------------------------------------
// upload: colour-major renumbering, device-built level layouts, transfers
// -------------------------------------------------------------------------
void upload_transfers(vasmg_ctx& C, int l, bool need32, bool need64, const std::vector<int>& perm,
                      const std::vector<int>& inv_next) {
  const Level& hl = C.H.levels[l];
  DevLevel& dl = C.lev[l];
  const int n = static_cast<int>(hl.n);
  // transfers P_l (rows: this level's device rows; cols: next level's device rows)
  const ScalarCSR& P = hl.P;
  const int nn = static_cast<int>(P.ncols);
  dl.nnext = nn;
  // the canonical P still on the device after its Galerkin product: renumber and
  // transpose it there (the same arrays as below)
  int64_t gn = 0, gnn = 0, gnnz = 0;
  const int64_t* gptr = nullptr;
  const int32_t* gcol = nullptr;
  const double* gval = nullptr;
  if (C.gdev && !C.alloc_stream &&
      galerkin_device_prolongation(C.gdev, l, &gn, &gnn, &gnnz, &gptr, &gcol, &gval) && gn == n &&
      gnn == nn && gnnz == static_cast<int64_t>(P.col.size())) {
    hipStream_t st = static_cast<hipStream_t>(galerkin_device_stream(C.gdev));
    dl.p_nnz = gnnz;
    dl.p_ptr = C.dalloc<int>(n + 1);
    dl.p_idx = C.dalloc<int>(gnnz);
    dl.pt_ptr = C.dalloc<int>(nn + 1);
    dl.pt_idx = C.dalloc<int>(gnnz);
    if (need64) {
      dl.p_w64 = C.dalloc<double>(gnnz);
      dl.pt_w64 = C.dalloc<double>(gnnz);
    }
    if (need32) {
      dl.p_w32 = C.dalloc<float>(gnnz);
      dl.pt_w32 = C.dalloc<float>(gnnz);
    }
    int* d_inv = nullptr;
    HIP_CHECK(hipMallocAsync(reinterpret_cast<void**>(&d_inv), std::max<size_t>(inv_next.size(), 1) * sizeof(int),
                             st));
    HIP_CHECK(hipMemcpyAsync(d_inv, inv_next.data(), inv_next.size() * sizeof(int), hipMemcpyHostToDevice, st));
    transfers_layout_device(st, n, nn, gnnz, gptr, gcol, gval, dl.perm, d_inv, dl.p_ptr, dl.p_idx,
                            dl.p_w64, dl.p_w32, dl.pt_ptr, dl.pt_idx, dl.pt_w64, dl.pt_w32);
    HIP_CHECK(hipFreeAsync(d_inv, st));
    HIP_CHECK(hipStreamSynchronize(st));
    galerkin_device_release_prolongation(C.gdev, l);
    return;
  }
  std::vector<int> pptr(n + 1, 0), pidx(P.col.size());
  std::vector<double> pw(P.col.size());
  for (int i = 0; i < n; ++i) pptr[i + 1] = pptr[i] + static_cast<int>(P.rowptr[perm[i] + 1] - P.rowptr[perm[i]]);
  for (int i = 0; i < n; ++i) {
    int k = pptr[i];
    for (int64_t p = P.rowptr[perm[i]]; p < P.rowptr[perm[i] + 1]; ++p, ++k) {
      pidx[k] = inv_next[P.col[p]];
      pw[k] = P.val[p];
    }
  }
  std::vector<int> tptr(nn + 1, 0), tidx(pidx.size());
  std::vector<double> tw(pidx.size());
  for (int j : pidx) tptr[j + 1]++;
  for (int j = 0; j < nn; ++j) tptr[j + 1] += tptr[j];
  {
    std::vector<int> fill(tptr.begin(), tptr.end() - 1);
    for (int i = 0; i < n; ++i)
      for (int k = pptr[i]; k < pptr[i + 1]; ++k) {
        const int q = fill[pidx[k]]++;
        tidx[q] = i;
        tw[q] = pw[k];
      }
  }
  dl.p_nnz = static_cast<int64_t>(pidx.size());
  dl.p_ptr = C.upload(pptr);
  dl.p_idx = C.upload(pidx);
  dl.pt_ptr = C.upload(tptr);
  dl.pt_idx = C.upload(tidx);
  if (need64) {
    dl.p_w64 = C.upload(pw);
    dl.pt_w64 = C.upload(tw);
  }
  if (need32) {
    dl.p_w32 = C.upload(std::vector<float>(pw.begin(), pw.end()));
    dl.pt_w32 = C.upload(std::vector<float>(tw.begin(), tw.end()));
  }
}

void upload_level_device(vasmg_ctx& C, int l, bool need32, bool need64, const std::vector<int>& inv,
                         const std::vector<int>& cell_lo, const std::vector<int>& cell_hi,
                         const std::vector<int>& cell_ptr, const std::vector<int>& blk_lo,
                         const std::vector<int>& blk_hi);

// Stable counting sort of perm by key[perm[i]] in [0, range).
void counting_sort_by(std::vector<int>& perm, const std::vector<int32_t>& key, int64_t range) {
  std::vector<int64_t> cnt(static_cast<size_t>(range) + 1, 0);
  for (int i : perm) cnt[key[i] + 1]++;
  for (int64_t k = 0; k < range; ++k) cnt[k + 1] += cnt[k];
  std::vector<int> out(perm.size());
  for (int i : perm) out[cnt[key[i]]++] = i;
  perm.swap(out);
}

// Device numbering of level l: canonical rows sorted by colour, colour block,
// cell (ties keep the canonical order); the identity on the coarsest level.
// Three stable counting sorts (cell, then block, then colour), computed once
// per level and kept.
std::vector<int> device_order(const vasmg_ctx& C, int l) {
  if (static_cast<int>(C.order_cache.size()) > l && !C.order_cache[l].empty())
    return C.order_cache[l];
  const Level& hl = C.H.levels[l];
  std::vector<int> perm(static_cast<size_t>(hl.n));
  std::iota(perm.begin(), perm.end(), 0);
  if (l != C.L && hl.n > 0) {
    counting_sort_by(perm, hl.cell, hl.ncells);
    if (hl.block != hl.cell) counting_sort_by(perm, hl.block, hl.nblocks);
    counting_sort_by(perm, hl.color, std::max<int32_t>(hl.ncolors, 1));
  }
  if (static_cast<int>(C.order_cache.size()) <= l) C.order_cache.resize(l + 1);
  C.order_cache[l] = perm;
  return perm;
}

void upload_level(vasmg_ctx& C, int l, bool need32, bool need64, const std::vector<int>& inv_next) {
  const Level& hl = C.H.levels[l];
  DevLevel& dl = C.lev[l];
  const int d = C.d, dd = d * d, n = static_cast<int>(hl.n);
  dl.n = n;
  dl.d = d;
  const bool coarsest = (l == C.L);
  dl.cells = !coarsest && l > 0;
  // device order: colour, colour block, cell, canonical index (identity on the coarsest)
  const std::vector<int> perm = device_order(C, l);
  std::vector<int> inv(n);
  if (coarsest) {
    dl.ncolors = 1;
    dl.color_ptr = {0, n};
  } else {
    dl.ncolors = hl.ncolors;
  }
  for (int i = 0; i < n; ++i) inv[perm[i]] = i;
  dl.perm = C.upload(perm);
  if (!hl.fixed.empty()) {
    std::vector<uint8_t> fx(n);
    for (int i = 0; i < n; ++i) fx[i] = hl.fixed[perm[i]];
    dl.fixed = C.upload(fx);
  }
  if (coarsest && l > 0) return;   // a coarse coarsest level only needs its factor and vectors

  // cell (and colour block) of each device row (single rows on point levels)
  std::vector<int> cell_lo(n), cell_hi(n), cell_ptr, blk_lo, blk_hi, block_ptr;
  if (dl.cells) {
    dl.blocks = hl.block_steps > 2;
    std::vector<int> ccp(dl.ncolors + 1, 0);
    for (int i = 0; i < n; ++i) {
      const bool new_cell = i == 0 || hl.cell[perm[i]] != hl.cell[perm[i - 1]];
      const bool new_block = i == 0 || hl.block[perm[i]] != hl.block[perm[i - 1]];
      if (new_cell) cell_ptr.push_back(i);
      if (new_block) {
        block_ptr.push_back(static_cast<int>(cell_ptr.size()) - 1);
        ccp[hl.color[perm[i]] + 1]++;
      }
    }
    cell_ptr.push_back(n);
    block_ptr.push_back(static_cast<int>(cell_ptr.size()) - 1);
    for (size_t c = 0; c + 1 < cell_ptr.size(); ++c)
      if (cell_ptr[c + 1] - cell_ptr[c] > (1 << d))
        throw vasmg::Error{VASMG_EINVAL, "internal: Gauss-Seidel cell larger than 2^d vertices"};
    for (size_t k = 0; k + 1 < block_ptr.size(); ++k)
      if (block_ptr[k + 1] - block_ptr[k] > (dl.blocks ? (1 << d) : 1))
        throw vasmg::Error{VASMG_EINVAL, "internal: colour block with too many cells"};
    for (int c = 0; c < dl.ncolors; ++c) ccp[c + 1] += ccp[c];
    dl.color_ptr = ccp;   // cells per colour, or colour blocks per colour
    dl.ncells = static_cast<int>(cell_ptr.size()) - 1;
    dl.nblocks = static_cast<int>(block_ptr.size()) - 1;
    for (int c = 0; c < dl.ncells; ++c)
      for (int i = cell_ptr[c]; i < cell_ptr[c + 1]; ++i) {
        cell_lo[i] = cell_ptr[c];
        cell_hi[i] = cell_ptr[c + 1];
      }
    if (dl.blocks) {
      blk_lo.resize(n);
      blk_hi.resize(n);
      for (int k = 0; k < dl.nblocks; ++k)
        for (int i = cell_ptr[block_ptr[k]]; i < cell_ptr[block_ptr[k + 1]]; ++i) {
          blk_lo[i] = cell_ptr[block_ptr[k]];
          blk_hi[i] = cell_ptr[block_ptr[k + 1]];
        }
    }
  } else {
    if (!coarsest) {
      dl.color_ptr.assign(dl.ncolors + 1, 0);
      for (int i = 0; i < n; ++i) dl.color_ptr[hl.color[i] + 1]++;
      for (int c = 0; c < dl.ncolors; ++c) dl.color_ptr[c + 1] += dl.color_ptr[c];
    }
    for (int i = 0; i < n; ++i) {
      cell_lo[i] = i;
      cell_hi[i] = i + 1;
    }
  }
  upload_level_device(C, l, need32, need64, inv, cell_lo, cell_hi, cell_ptr, blk_lo, blk_hi);
  if (dl.blocks) dl.block_ptr = C.upload(block_ptr);
  if (!coarsest) upload_transfers(C, l, need32, need64, perm, inv_next);
  if (!coarsest && C.opt.smoother == VASMG_SMOOTHER_JACOBI) {
    if (C.gdev) galerkin_device_join(C.gdev);   // the host values of the level
    std::vector<double> dinv;
    block_diag_inverse(hl.A, hl.fixed, dinv);
    const double lam = jacobi_lambda_max(hl.A, dinv, 30);
    if (!(lam > 0.0) || !std::isfinite(lam))
      throw vasmg::Error{VASMG_EDEGENERATE, "Jacobi smoother: no positive eigenvalue estimate"};
    dl.omega = (4.0 / 3.0) / lam;
    std::vector<double> dd_dev(dinv.size());
    for (int i = 0; i < n; ++i)
      std::copy(dinv.begin() + static_cast<int64_t>(perm[i]) * dd,
                dinv.begin() + static_cast<int64_t>(perm[i] + 1) * dd,
                dd_dev.begin() + static_cast<int64_t>(i) * dd);
    if (need64) dl.dinv64 = C.upload(dd_dev);
    if (need32) dl.dinv32 = C.upload(std::vector<float>(dd_dev.begin(), dd_dev.end()));
  }
}

// Lanes per block row from the mean off-cell blocks per row: about two blocks per
// lane; 3D cell levels use 16..64; 2D cell levels (short rows) about two quads of
// 4 blocks per lane, 4..64, several cells sharing a wavefront below 16.
void set_lanes(DevLevel& dl) {
  const double avg = dl.n > 0 ? static_cast<double>(dl.nnz) / dl.n : 1.0;
  if (dl.cells && dl.d == 2)
    dl.G = std::min(64, std::max(4, pow2_ceil(static_cast<int>(std::ceil(avg / 8.0)))));
  else
    dl.G = std::min(64, std::max(dl.cells ? 16 : 4, pow2_ceil(static_cast<int>(std::ceil(avg / 2.0)))));
  dl.Gspmv = dl.G;
}

// Row pointers of the L or U part from per-row block counts; rows padded to
// whole quads of 4 blocks on cell levels.
std::vector<int> padded_ptr(const std::vector<int>& cnt, bool cells) {
  const int Q = cells ? dev::kQuad : 1;
  std::vector<int> ptr(cnt.size() + 1, 0);
  for (size_t i = 0; i < cnt.size(); ++i) {
    const int64_t next = static_cast<int64_t>(ptr[i]) + (cnt[i] + Q - 1) / Q * Q;
    if (next > INT32_MAX) throw vasmg::Error{VASMG_EINVAL, "level too large for int32 row pointers"};
    ptr[i + 1] = static_cast<int>(next);
  }
  return ptr;
}

// Device memory that lives for one level's layout: stream-ordered on the upload
// stream when there is one (a server slot's), else plain allocations.
struct TempDev {
  hipStream_t st = nullptr;
  bool ordered = false;
  std::vector<void*> p;
  TempDev(hipStream_t s, bool o) : st(s), ordered(o) {}
  TempDev(const TempDev&) = delete;
  TempDev& operator=(const TempDev&) = delete;
  ~TempDev() {
    for (void* q : p) {
      if (ordered)
        (void)hipFreeAsync(q, st);
      else
        (void)hipFree(q);
    }
  }
  template <class T>
  T* up(const T* src, size_t n) {
    void* q = nullptr;
    const size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
    HIP_CHECK(ordered ? hipMallocAsync(&q, bytes, st) : hipMalloc(&q, bytes));
    p.push_back(q);
    if (n) HIP_CHECK(hipMemcpyAsync(q, src, n * sizeof(T), hipMemcpyHostToDevice, st));
    return static_cast<T*>(q);
  }
  template <class T, class A>
  T* up(const std::vector<T, A>& v) { return up(v.data(), v.size()); }
};

// Device layout of level l: built by the layout kernels from the level's
// canonical FP64 operator, resident from the device Galerkin products
// (setup_device = 1) or copied in from the host hierarchy for the layout only.
// Only the renumbering, the cell ranges and the row pointers travel besides.
void upload_level_device(vasmg_ctx& C, int l, bool need32, bool need64, const std::vector<int>& inv,
                         const std::vector<int>& cell_lo, const std::vector<int>& cell_hi,
                         const std::vector<int>& cell_ptr, const std::vector<int>& blk_lo,
                         const std::vector<int>& blk_hi) {
  const Level& hl = C.H.levels[l];
  DevLevel& dl = C.lev[l];
  const int d = C.d, dd = d * d, n = dl.n, NU = (1 << d) * d;
  hipStream_t st = C.alloc_stream;
  DevOperator A;
  const bool resident = galerkin_device_operator(C.gdev, l, &A);
  if (!st && resident) st = static_cast<hipStream_t>(galerkin_device_stream(C.gdev));
  TempDev tmp(st, C.alloc_stream != nullptr);
  if (!resident) {
    A.n = hl.n;
    A.ptr = tmp.up(hl.A.rowptr);
    A.col = tmp.up(hl.A.col);
    A.val = tmp.up(hl.A.val);
  }
  LayoutArgs a;
  a.d = d;
  a.n = n;
  a.perm = dl.perm;
  a.inv = tmp.up(inv);
  a.lo = tmp.up(cell_lo);
  a.hi = tmp.up(cell_hi);
  if (dl.cells) {
    std::vector<int> cor(n);
    for (int c = 0; c + 1 < static_cast<int>(cell_ptr.size()); ++c)
      for (int i = cell_ptr[c]; i < cell_ptr[c + 1]; ++i) cor[i] = c;
    a.cell_of_row = tmp.up(cor);
  }
  if (dl.blocks) {
    a.blo = tmp.up(blk_lo);
    a.bhi = tmp.up(blk_hi);
  }
  a.fixed = dl.fixed;
  // parts: L (earlier colours), E / F (earlier / later cells of the row's colour
  // block, colour-block levels only), U (later colours)
  const int nparts = dl.blocks ? kParts : 2;
  const int pidx[kParts] = {kPartL, kPartU, kPartE, kPartF};
  std::vector<int> cnt[kParts];
  int* d_cnt[kParts] = {nullptr, nullptr, nullptr, nullptr};
  for (int q = 0; q < nparts; ++q) {
    cnt[pidx[q]].assign(n, 0);
    d_cnt[pidx[q]] = tmp.up(cnt[pidx[q]]);
    a.part[pidx[q]].cnt = d_cnt[pidx[q]];
  }
  layout_count(A, a, st);
  for (int q = 0; q < nparts; ++q)
    HIP_CHECK(hipMemcpyAsync(cnt[pidx[q]].data(), d_cnt[pidx[q]], n * sizeof(int),
                             hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  for (int i = 0; i < n; ++i) {
    dl.nnz_lo += cnt[kPartL][i];
    dl.nnz_up += cnt[kPartU][i];
    if (dl.blocks) {
      dl.nnz_e += cnt[kPartE][i];
      dl.nnz_f += cnt[kPartF][i];
    }
  }
  dl.nnz = dl.nnz_lo + dl.nnz_up + dl.nnz_e + dl.nnz_f;
  set_lanes(dl);
  // every part plane-major over its own blocks; on cell levels every row is
  // padded to whole quads of 4 blocks (zero blocks pointing at the row itself),
  // so a lane reads 4 consecutive blocks with one 16-byte load per plane
  const std::vector<int> Lptr = padded_ptr(cnt[kPartL], dl.cells), Uptr = padded_ptr(cnt[kPartU], dl.cells);
  const int64_t nL = Lptr[n], nU = Uptr[n];
  dl.Lstride = nL;
  dl.Ustride = nU;
  dl.Lptr = C.upload(Lptr);
  dl.Uptr = C.upload(Uptr);
  dl.Lcol = C.dalloc<int>(nL);
  dl.Ucol = C.dalloc<int>(nU);
  int64_t nE = 0, nF = 0;
  if (dl.blocks) {
    const std::vector<int> Eptr = padded_ptr(cnt[kPartE], true), Fptr = padded_ptr(cnt[kPartF], true);
    nE = Eptr[n];
    nF = Fptr[n];
    dl.Estride = nE;
    dl.Fstride = nF;
    dl.Eptr = C.upload(Eptr);
    dl.Fptr = C.upload(Fptr);
    dl.Ecol = C.dalloc<int>(nE);
    dl.Fcol = C.dalloc<int>(nF);
  }
  if (dl.cells) dl.cell_ptr = C.upload(cell_ptr);
  const int64_t m_len = dl.cells ? static_cast<int64_t>(dl.ncells) * NU * NU : static_cast<int64_t>(n) * dd;
  if (need64) {
    dl.Lval64 = C.dalloc<double>(nL * dd);
    dl.Uval64 = C.dalloc<double>(nU * dd);
    if (dl.blocks) {
      dl.Eval64 = C.dalloc<double>(nE * dd);
      dl.Fval64 = C.dalloc<double>(nF * dd);
    }
    (dl.cells ? dl.cellM64 : dl.diag64) = C.dalloc<double>(m_len);
    dl.has64 = true;
  }
  if (need32) {
    dl.Lval32 = C.dalloc<float>(nL * dd);
    dl.Uval32 = C.dalloc<float>(nU * dd);
    if (dl.blocks) {
      dl.Eval32 = C.dalloc<float>(nE * dd);
      dl.Fval32 = C.dalloc<float>(nF * dd);
    }
    (dl.cells ? dl.cellM32 : dl.diag32) = C.dalloc<float>(m_len);
    dl.has32 = true;
  }
  a.part[kPartL] = {dl.Lptr, d_cnt[kPartL], nL, dl.Lcol, dl.Lval32, dl.Lval64};
  a.part[kPartU] = {dl.Uptr, d_cnt[kPartU], nU, dl.Ucol, dl.Uval32, dl.Uval64};
  if (dl.blocks) {
    a.part[kPartE] = {dl.Eptr, d_cnt[kPartE], nE, dl.Ecol, dl.Eval32, dl.Eval64};
    a.part[kPartF] = {dl.Fptr, d_cnt[kPartF], nF, dl.Fcol, dl.Fval32, dl.Fval64};
  }
  a.M32 = dl.cells ? dl.cellM32 : dl.diag32;
  a.M64 = dl.cells ? dl.cellM64 : dl.diag64;
  a.m_len = m_len;
  layout_fill(A, a, st);
}

// inverse permutation of level l's device numbering (canonical -> device)
std::vector<int> device_inverse(const vasmg_ctx& C, int l) {
  const std::vector<int> perm = device_order(C, l);
  std::vector<int> inv(perm.size());
  for (size_t i = 0; i < perm.size(); ++i) inv[perm[i]] = static_cast<int>(i);
  return inv;
}

// A^{-1} = L^{-T} L^{-1} from the lower Cholesky factor L (row-major n x n), in
// FP64; symmetric by construction (each pair of entries computed once).
std::vector<double> coarse_inverse(const std::vector<double>& Lf, int64_t n) {
  std::vector<double> Li(static_cast<size_t>(n * n), 0.0);   // L^{-1}, lower
  for (int64_t j = 0; j < n; ++j) {
    Li[j * n + j] = 1.0 / Lf[j * n + j];
    for (int64_t i = j + 1; i < n; ++i) {
      double s = 0.0;
      for (int64_t k = j; k < i; ++k) s += Lf[i * n + k] * Li[k * n + j];
      Li[i * n + j] = -s / Lf[i * n + i];
    }
  }
  std::vector<double> M(static_cast<size_t>(n * n), 0.0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j <= i; ++j) {
      double s = 0.0;
      for (int64_t k = i; k < n; ++k) s += Li[k * n + i] * Li[k * n + j];
      M[i * n + j] = s;
      M[j * n + i] = s;
    }
  return M;
}

void select_bottom(vasmg_ctx& C);

void upload_all(vasmg_ctx& C) {
  const int nl = static_cast<int>(C.H.levels.size());
  C.L = nl - 1;
  C.lev.assign(nl, DevLevel());
  const bool vasmg = C.opt.preconditioner == VASMG_PRECOND_VASMG;
  const int last = vasmg ? C.L : 0;
  for (int l = 0; l <= last; ++l) {
    const bool fine = (l == 0);
    const bool need64 = fine || !C.vc32;
    const bool need32 = C.vc32 && vasmg;
    std::vector<int> inv_next;
    if (l < C.L) inv_next = device_inverse(C, l + 1);
    upload_level(C, l, need32, need64, inv_next);
  }
  const int T = C.vc32 ? 4 : 8;
  for (int l = 0; l <= last; ++l) {
    DevLevel& dl = C.lev[l];
    const int64_t len = static_cast<int64_t>(C.H.levels[l].n) * C.DP;
    dl.b = C.dalloc<char>(len * T);
    dl.x = C.dalloc<char>(len * T);
    dl.s = C.dalloc<char>(len * T);
    dl.r = C.dalloc<char>(len * T);
    C.clear(dl.b, len * T);
    C.clear(dl.x, len * T);
    C.clear(dl.s, len * T);
    C.clear(dl.r, len * T);
  }
  if (vasmg) {
    C.n_coarse = C.H.n_coarse_dofs;
    if (C.n_coarse > dev::kCoarseMax)
      throw vasmg::Error{VASMG_EINVAL, "coarsest level has more than 4096 DOFs"};
    C.chol = C.upload(C.H.chol);
    if (C.n_coarse <= dev::kCoarseInvMax) C.cinv = C.upload(coarse_inverse(C.H.chol, C.n_coarse));
    if (C.cinv && C.L >= 2 && C.opt.smoother == VASMG_SMOOTHER_GS && C.opt.n_pre >= 1)
      select_bottom(C);
  }
  // PCG vectors
  C.n0 = static_cast<int>(C.H.levels[0].n);
  C.n0p = static_cast<int64_t>(C.n0) * C.DP;
  {
    std::vector<int> um(C.n0);
    std::vector<int> perm0(C.n0);
    C.copy(perm0.data(), C.lev[0].perm, sizeof(int) * C.n0, hipMemcpyDeviceToHost);
    for (int i = 0; i < C.n0; ++i) um[i] = C.H.free_vertices[perm0[i]];
    C.user_map = C.upload(um);
  }
  for (double** v : {&C.F, &C.X, &C.R, &C.P, &C.Q, &C.Z}) {
    *v = C.dalloc<double>(C.n0p);
    C.clear(*v, sizeof(double) * C.n0p);
  }
  // FP64 V-cycle: its fine right-hand side is the PCG residual itself
  if (!C.vc32) C.lev[0].b = C.R;
  // partial sums: the flat reduction grid, or one per workgroup of the fine SpMV
  // (sized for the narrowest workgroup row count any lane width can give)
  C.n_partial = std::max(kFlatGrid, grid_for(C.n0, dev::kBlock / 64));
  C.partial = C.dalloc<double>(C.n_partial);
  C.sc = C.dalloc<Scalars>(1);
  C.clear(C.sc, sizeof(Scalars));
  C.zero_flag = C.dalloc<int>(1);
  C.clear(C.zero_flag, sizeof(int));
  // pinned scalars: Scalars at 0, rtol at 256, block scalars [16] at 512
  static_assert(512 + 16 * sizeof(Scalars) <= PinnedPool::kBytes, "pinned block too small");
  C.pinned = pinned_pool().get();
  C.h_sc = static_cast<Scalars*>(C.pinned);
  C.h_rtol = reinterpret_cast<double*>(static_cast<char*>(C.pinned) + 256);
  for (auto& e : C.ev) HIP_CHECK(hipEventCreate(&e));
  HIP_CHECK(hipStreamCreateWithFlags(&C.cap_stream, hipStreamNonBlocking));
  if (C.nseg > 0) {
    // segment of each fine device row, and each segment's rows (ascending)
    const std::vector<int> perm0 = device_order(C, 0);
    std::vector<int> of(C.n0), cnt(C.nseg + 1, 0);
    for (int i = 0; i < C.n0; ++i) {
      const int64_t v = perm0[i];
      of[i] = static_cast<int>(std::upper_bound(C.seg_free_off.begin(), C.seg_free_off.end(), v) -
                               C.seg_free_off.begin()) - 1;
      cnt[of[i] + 1]++;
    }
    for (int k = 0; k < C.nseg; ++k) cnt[k + 1] += cnt[k];
    std::vector<int> rows(C.n0), fill(cnt.begin(), cnt.end() - 1);
    for (int i = 0; i < C.n0; ++i) rows[fill[of[i]]++] = i;
    C.seg_of_row = C.upload(of);
    C.seg_ptr = C.upload(cnt);
    C.seg_rows = C.upload(rows);
    C.ssc = C.dalloc<Scalars>(C.nseg);
    C.clear(C.ssc, sizeof(Scalars) * C.nseg);
    C.seg_running = C.dalloc<int>(1);
    C.clear(C.seg_running, sizeof(int));
  }
  std::vector<std::vector<int>>().swap(C.order_cache);   // numbering no longer needed
}

// -------------------------------------------------------------------------
// kernel launch helpers
// -------------------------------------------------------------------------
#define DISPATCH_G(Gv, ...)                 \
  switch (Gv) {                             \
    case 4: { constexpr int GG = 4; __VA_ARGS__; } break;   \
    case 8: { constexpr int GG = 8; __VA_ARGS__; } break;   \
    case 16: { constexpr int GG = 16; __VA_ARGS__; } break; \
    case 32: { constexpr int GG = 32; __VA_ARGS__; } break; \
    default: { constexpr int GG = 64; __VA_ARGS__; } break; \
  }

template <typename T>
struct LevelMats;
template <>
struct LevelMats<float> {
  static dev::Part<float> L(const DevLevel& l) { return {l.Lptr, l.Lcol, l.Lval32, l.Lstride}; }
  static dev::Part<float> U(const DevLevel& l) { return {l.Uptr, l.Ucol, l.Uval32, l.Ustride}; }
  static dev::Part<float> E(const DevLevel& l) { return {l.Eptr, l.Ecol, l.Eval32, l.Estride}; }
  static dev::Part<float> F(const DevLevel& l) { return {l.Fptr, l.Fcol, l.Fval32, l.Fstride}; }
  static const float* diag(const DevLevel& l) { return l.diag32; }
  static const float* pw(const DevLevel& l) { return l.p_w32; }
  static const float* ptw(const DevLevel& l) { return l.pt_w32; }
  static const float* cellM(const DevLevel& l) { return l.cellM32; }
  static const float* dinv(const DevLevel& l) { return l.dinv32; }
  static bool ok(const DevLevel& l) { return l.has32; }
};
template <>
struct LevelMats<double> {
  static dev::Part<double> L(const DevLevel& l) { return {l.Lptr, l.Lcol, l.Lval64, l.Lstride}; }
  static dev::Part<double> U(const DevLevel& l) { return {l.Uptr, l.Ucol, l.Uval64, l.Ustride}; }
  static dev::Part<double> E(const DevLevel& l) { return {l.Eptr, l.Ecol, l.Eval64, l.Estride}; }
  static dev::Part<double> F(const DevLevel& l) { return {l.Fptr, l.Fcol, l.Fval64, l.Fstride}; }
  static const double* diag(const DevLevel& l) { return l.diag64; }
  static const double* pw(const DevLevel& l) { return l.p_w64; }
  static const double* ptw(const DevLevel& l) { return l.pt_w64; }
  static const double* cellM(const DevLevel& l) { return l.cellM64; }
  static const double* dinv(const DevLevel& l) { return l.dinv64; }
  static bool ok(const DevLevel& l) { return l.has64; }
};

// cells per colour that the fused bottom takes in at most two rounds of its wavefronts
constexpr int kBottomCellsPerColour = 2 * dev::kBottomThreads / 64;

template <typename T>
dev::BottomLevel<T>* upload_bottom(vasmg_ctx& C) {
  std::vector<dev::BottomLevel<T>> v;
  for (int l = C.bottom_lo; l < C.L; ++l) {
    const DevLevel& lv = C.lev[l];
    if (!LevelMats<T>::ok(lv)) return nullptr;
    dev::BottomLevel<T> b;
    b.n = lv.n;
    b.ncolors = lv.ncolors;
    b.ncells = lv.ncells;
    b.nnext = lv.nnext;
    b.color_ptr = lv.color_ptr_dev;
    b.cell_ptr = lv.cell_ptr;
    b.L = LevelMats<T>::L(lv);
    b.U = LevelMats<T>::U(lv);
    b.cellM = LevelMats<T>::cellM(lv);
    b.p_ptr = lv.p_ptr;
    b.p_idx = lv.p_idx;
    b.p_w = LevelMats<T>::pw(lv);
    b.pt_ptr = lv.pt_ptr;
    b.pt_idx = lv.pt_idx;
    b.pt_w = LevelMats<T>::ptw(lv);
    b.fixed = lv.fixed;
    v.push_back(b);
  }
  return C.upload(v);
}

// Chooses the levels of the fused bottom: from L-1 upwards, cell levels whose
// colours hold few cells (each colour a round or two of the workgroup's
// wavefronts) and whose LDS vectors fit together; one level for the W-cycle,
// which visits the levels above L-1 twice.
void select_bottom(vasmg_ctx& C) {
  // the kernel restricts into (and prolongs from) the coarsest level's DOFs in LDS
  if (static_cast<int64_t>(C.lev[C.L - 1].nnext) * C.d != C.n_coarse || C.n_coarse > dev::kCoarseInvMax)
    return;
  const int tb = C.lev[C.L - 1].has64 ? 8 : 4;
  const int maxlev = C.opt.cycle == VASMG_CYCLE_W ? 1 : dev::kBottomLevels;
  auto fits = [&](const DevLevel& lv) {
    if (!lv.cells || lv.blocks) return false;
    for (int c = 0; c < lv.ncolors; ++c)
      if (lv.color_ptr[c + 1] - lv.color_ptr[c] > kBottomCellsPerColour) return false;
    return true;
  };
  int lo = C.L;
  int64_t nvec = 0, nint = 0;
  while (lo - 1 >= 1 && C.L - (lo - 1) <= maxlev) {
    const DevLevel& lv = C.lev[lo - 1];
    const int64_t e = dev::bottom_vec_elems(lv.n, C.DP);
    const int64_t ie = dev::bottom_int_elems(lv.n, lv.ncolors, lv.ncells);
    if (!fits(lv) || (nvec + e) * tb + (nint + ie) * 4 > dev::kBottomLds) break;
    nvec += e;
    nint += ie;
    --lo;
  }
  if (lo == C.L) return;
  C.bottom_lo = lo;
  C.bottom_vec = nvec;
  C.bottom_int = nint;
  for (int l = lo; l < C.L; ++l) C.lev[l].color_ptr_dev = C.upload(C.lev[l].color_ptr);
  C.bottom32 = upload_bottom<float>(C);
  C.bottom64 = upload_bottom<double>(C);
}

// Returns the number of workgroups (= partial sums written when partial != NULL).
template <typename T, int D>
int launch_spmv(const DevLevel& lv, const T* x, T* y, double* partial, int n_partial,
                const int* done, hipStream_t st) {
  const int G = lv.Gspmv;
  int used = 0;
  DISPATCH_G(G, {
    const int grid = grid_for(lv.n, dev::kBlock / GG);
    if (partial && grid > n_partial)
      throw vasmg::Error{VASMG_EINVAL, "internal: SpMV partial buffer too small"};
    used = grid;
    if (partial)
      hipLaunchKernelGGL((dev::k_spmv<T, D, GG, true>), dim3(grid), dim3(dev::kBlock), 0, st, lv.n,
                         LevelMats<T>::L(lv), LevelMats<T>::U(lv), LevelMats<T>::diag(lv),
                         x, y, partial, done);
    else
      hipLaunchKernelGGL((dev::k_spmv<T, D, GG, false>), dim3(grid), dim3(dev::kBlock), 0, st,
                         lv.n, LevelMats<T>::L(lv), LevelMats<T>::U(lv), LevelMats<T>::diag(lv),
                         x, y, partial, done);
  });
  return used;
}


template <typename T, int D>
void launch_gs_color(const DevLevel& lv, int c, int mode, const T* b, T* x, T* s_save,
                     const int* done, hipStream_t st) {
  const int r0 = lv.color_ptr[c], nr = lv.color_ptr[c + 1] - r0;
  if (nr <= 0) return;
  DISPATCH_G(lv.G, {
    const int grid = grid_for(nr, dev::kBlock / GG);
    if (mode == 0)
      hipLaunchKernelGGL((dev::k_gs_color<T, D, GG, 0>), dim3(grid), dim3(dev::kBlock), 0, st, r0,
                         nr, LevelMats<T>::L(lv), LevelMats<T>::U(lv), LevelMats<T>::diag(lv), b, x,
                         s_save, done);
    else if (mode == 1)
      hipLaunchKernelGGL((dev::k_gs_color<T, D, GG, 1>), dim3(grid), dim3(dev::kBlock), 0, st, r0,
                         nr, LevelMats<T>::L(lv), LevelMats<T>::U(lv), LevelMats<T>::diag(lv), b, x,
                         s_save, done);
    else
      hipLaunchKernelGGL((dev::k_gs_color<T, D, GG, 2>), dim3(grid), dim3(dev::kBlock), 0, st, r0,
                         nr, LevelMats<T>::L(lv), LevelMats<T>::U(lv), LevelMats<T>::diag(lv), b, x,
                         s_save, done);
  });
}

#define DISPATCH_GR(Gv, ...)                                  \
  switch (Gv) {                                               \
    case 4: { constexpr int GR = 4; __VA_ARGS__; } break;     \
    case 8: { constexpr int GR = 8; __VA_ARGS__; } break;     \
    case 16: { constexpr int GR = 16; __VA_ARGS__; } break;   \
    case 32: { constexpr int GR = 32; __VA_ARGS__; } break;   \
    default: { constexpr int GR = 64; __VA_ARGS__; } break;   \
  }

// One colour of a colour-block level: one workgroup per block (k_gs_block).
// The V-cycle kernels do not read the stop flag (see enqueue_iter_B).
template <typename T, int D>
void launch_gs_blocks(const DevLevel& lv, int c, int mode, const T* b, T* x, T* s_save,
                      hipStream_t st) {
  if constexpr (D == 3) {
    const int k0 = lv.color_ptr[c], nk = lv.color_ptr[c + 1] - k0;
    if (nk <= 0) return;
    const T* M = LevelMats<T>::cellM(lv);
    const dev::Part<T> Lp = LevelMats<T>::L(lv), Up = LevelMats<T>::U(lv);
    const dev::Part<T> Ep = LevelMats<T>::E(lv), Fp = LevelMats<T>::F(lv);
    const dim3 grid(nk), blk(dev::BlockShape<D>::threads);
    if (mode == 0)
      hipLaunchKernelGGL((dev::k_gs_block<T, D, 0>), grid, blk, 0, st, k0, lv.block_ptr,
                         lv.cell_ptr, Lp, Up, Ep, Fp, M, b, x, s_save);
    else if (mode == 1)
      hipLaunchKernelGGL((dev::k_gs_block<T, D, 1>), grid, blk, 0, st, k0, lv.block_ptr,
                         lv.cell_ptr, Lp, Up, Ep, Fp, M, b, x, s_save);
    else
      hipLaunchKernelGGL((dev::k_gs_block<T, D, 2>), grid, blk, 0, st, k0, lv.block_ptr,
                         lv.cell_ptr, Lp, Up, Ep, Fp, M, b, x, static_cast<T*>(nullptr));
  } else {
    throw vasmg::Error{VASMG_EINVAL, "internal: colour blocks are built in 3D only"};
  }
}

template <typename T, int D>
void launch_gs_cells(const DevLevel& lv, int c, int mode, const T* b, T* x, T* s_save,
                     const int* done, hipStream_t st) {
  if (lv.blocks) {
    launch_gs_blocks<T, D>(lv, c, mode, b, x, s_save, st);
    return;
  }
  const int c0 = lv.color_ptr[c], nc = lv.color_ptr[c + 1] - c0;
  if (nc <= 0) return;
  const T* M = LevelMats<T>::cellM(lv);
  const dev::Part<T> Lp = LevelMats<T>::L(lv), Up = LevelMats<T>::U(lv);
  DISPATCH_GR(lv.G, {
    using Pack = dev::CellPack<D, GR>;
    const dim3 blk(Pack::threads), grid((nc + Pack::CPW - 1) / Pack::CPW);
    if (mode == 0)
      hipLaunchKernelGGL((dev::k_gs_cell<T, D, GR, 0>), grid, blk, 0, st, c0, nc, lv.cell_ptr,
                         Lp, Up, M, b, x, s_save, done);
    else if (mode == 1)
      hipLaunchKernelGGL((dev::k_gs_cell<T, D, GR, 1>), grid, blk, 0, st, c0, nc, lv.cell_ptr,
                         Lp, Up, M, b, x, s_save, done);
    else
      hipLaunchKernelGGL((dev::k_gs_cell<T, D, GR, 2>), grid, blk, 0, st, c0, nc, lv.cell_ptr,
                         Lp, Up, M, b, x, s_save, done);
  });
}

template <typename T, int D, int KIND>
void launch_cell_apply(const DevLevel& lv, const T* base, const T* x, T* out, const int* done,
                       hipStream_t st) {
  const dev::Part<T> Ep = LevelMats<T>::E(lv), Fp = LevelMats<T>::F(lv);
  DISPATCH_GR(lv.G, {
    using Pack = dev::CellPack<D, GR>;
    const dim3 grid((lv.ncells + Pack::CPW - 1) / Pack::CPW), blk(Pack::threads);
    if (lv.blocks)
      hipLaunchKernelGGL((dev::k_cell_apply<T, D, GR, KIND, true>), grid, blk, 0, st, lv.ncells,
                         lv.cell_ptr, LevelMats<T>::L(lv), LevelMats<T>::U(lv), Ep, Fp,
                         LevelMats<T>::cellM(lv), base, x, out, done);
    else
      hipLaunchKernelGGL((dev::k_cell_apply<T, D, GR, KIND, false>), grid, blk, 0, st, lv.ncells,
                         lv.cell_ptr, LevelMats<T>::L(lv), LevelMats<T>::U(lv), Ep, Fp,
                         LevelMats<T>::cellM(lv), base, x, out, done);
  });
}

template <typename T, int D>
void launch_gs_sweep(const DevLevel& lv, bool backward, bool zero_guess, const T* b, T* x,
                     T* s_save, const int* done, hipStream_t st) {
  if (lv.cells) {
    if (!backward) {
      for (int c = 0; c < lv.ncolors; ++c)
        launch_gs_cells<T, D>(lv, c, zero_guess ? 0 : 1, b, x, s_save, done, st);
    } else {
      for (int c = lv.ncolors - 1; c >= 0; --c) launch_gs_cells<T, D>(lv, c, 2, b, x, nullptr, done, st);
    }
    return;
  }
  if (!backward) {
    for (int c = 0; c < lv.ncolors; ++c)
      launch_gs_color<T, D>(lv, c, zero_guess ? 0 : 1, b, x, s_save, done, st);
  } else {
    for (int c = lv.ncolors - 1; c >= 0; --c) launch_gs_color<T, D>(lv, c, 2, b, x, nullptr, done, st);
  }
}

template <typename T, int D>
void launch_residual_upper(const DevLevel& lv, const T* s, const T* x, T* r, const int* done,
                           hipStream_t st) {
  if (lv.cells) {
    launch_cell_apply<T, D, 0>(lv, s, x, r, done, st);
    return;
  }
  DISPATCH_G(lv.G, {
    hipLaunchKernelGGL((dev::k_residual_upper<T, D, GG>), dim3(grid_for(lv.n, dev::kBlock / GG)),
                       dim3(dev::kBlock), 0, st, lv.n, LevelMats<T>::U(lv), LevelMats<T>::diag(lv),
                       s, x, r, done);
  });
}

template <typename T, int D>
void launch_residual_full(const DevLevel& lv, const T* b, const T* x, T* r, const int* done,
                          hipStream_t st) {
  if (lv.cells) {
    launch_cell_apply<T, D, 1>(lv, b, x, r, done, st);
    return;
  }
  DISPATCH_G(lv.G, {
    hipLaunchKernelGGL((dev::k_residual_full<T, D, GG>), dim3(grid_for(lv.n, dev::kBlock / GG)),
                       dim3(dev::kBlock), 0, st, lv.n, LevelMats<T>::L(lv), LevelMats<T>::U(lv),
                       LevelMats<T>::diag(lv), b, x, r, done);
  });
}

// restriction rows (P^T) hold up to ~27 entries, prolongation rows up to 2^d
constexpr int kRestrictLanes = 8, kProlongLanes = 4;

template <typename T, int D>
void launch_jacobi(const DevLevel& lv, bool first, const T* v, T* x, const int* done,
                   hipStream_t st) {
  const dim3 grid(grid_for(lv.n, dev::kBlock)), blk(dev::kBlock);
  const T om = static_cast<T>(lv.omega);
  if (first)
    hipLaunchKernelGGL((dev::k_jacobi_step<T, D, true>), grid, blk, 0, st, lv.n,
                       LevelMats<T>::dinv(lv), om, v, x, done);
  else
    hipLaunchKernelGGL((dev::k_jacobi_step<T, D, false>), grid, blk, 0, st, lv.n,
                       LevelMats<T>::dinv(lv), om, v, x, done);
}

template <typename T, int D>
void launch_restrict(const DevLevel& lv, const T* r, T* bc, const int* done, hipStream_t st) {
  hipLaunchKernelGGL((dev::k_restrict<T, D, kRestrictLanes>),
                     dim3(grid_for(lv.nnext, dev::kBlock / kRestrictLanes)), dim3(dev::kBlock), 0,
                     st, lv.nnext, lv.pt_ptr, lv.pt_idx, LevelMats<T>::ptw(lv), r, bc, done);
}

template <typename T, int D>
void launch_prolong(const DevLevel& lv, const T* e, T* x, const int* done, hipStream_t st) {
  hipLaunchKernelGGL((dev::k_prolong_add<T, D, kProlongLanes>),
                     dim3(grid_for(lv.n, dev::kBlock / kProlongLanes)), dim3(dev::kBlock), 0, st,
                     lv.n, lv.p_ptr, lv.p_idx, LevelMats<T>::pw(lv), e, x, lv.fixed, done);
}

template <typename T>
void launch_fill(T* a, int64_t n, T v, hipStream_t st) {
  hipLaunchKernelGGL((dev::k_fill<T>), dim3(std::min<int64_t>(kFlatGrid, grid_for(n, dev::kBlock))),
                     dim3(dev::kBlock), 0, st, n, a, v);
}

// -------------------------------------------------------------------------
// Phase profiler: brackets each phase of the schedule with events (outside
// graphs) and accumulates launches, device time and algorithmic HBM bytes.
// -------------------------------------------------------------------------
struct PhaseStat {
  std::string name;
  int level;
  int launches;
  double ms;
  double bytes;
};

struct Profiler {
  hipStream_t st;
  std::vector<PhaseStat> stats;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
  std::vector<size_t> pending_idx;
  template <class F>
  void phase(const std::string& name, int level, int launches, double bytes, F&& fn) {
    hipEvent_t a, b;
    HIP_CHECK(hipEventCreate(&a));
    HIP_CHECK(hipEventCreate(&b));
    HIP_CHECK(hipEventRecord(a, st));
    fn();
    HIP_CHECK(hipEventRecord(b, st));
    size_t idx = stats.size();
    for (size_t i = 0; i < stats.size(); ++i)
      if (stats[i].name == name && stats[i].level == level) idx = i;
    if (idx == stats.size()) stats.push_back({name, level, 0, 0.0, 0.0});
    stats[idx].launches += launches;
    stats[idx].bytes += bytes;
    pending.emplace_back(a, b);
    pending_idx.push_back(idx);
  }
  void finish() {
    HIP_CHECK(hipStreamSynchronize(st));
    for (size_t i = 0; i < pending.size(); ++i) {
      float ms = 0.f;
      HIP_CHECK(hipEventElapsedTime(&ms, pending[i].first, pending[i].second));
      stats[pending_idx[i]].ms += ms;
      (void)hipEventDestroy(pending[i].first);
      (void)hipEventDestroy(pending[i].second);
    }
    pending.clear();
    pending_idx.clear();
  }
};

template <class F>
void run_phase(Profiler* prof, const char* name, int level, int launches, double bytes, F&& fn) {
  if (prof)
    prof->phase(name, level, launches, bytes, fn);
  else
    fn();
}

// Algorithmic HBM bytes of the phases of one level (each array read or written
// once per launch; the gathered neighbour vector counted once per launch).
struct LevelBytes {
  double gs_fwd0, gs_fwd, residual, gs_bwd, restrict_, prolong;
};

LevelBytes level_bytes(const vasmg_ctx& C, int l, int tb) {
  const DevLevel& lv = C.lev[l];
  const int D = C.d, DP = C.DP, dd = D * D;
  const double blk = dd * tb + 4.0;                 // values + column index
  const double n = lv.n, vec = n * DP * tb;
  const int NU = (1 << D) * D;
  const double own = lv.cells ? lv.ncells * (NU * NU * static_cast<double>(tb) + 4.0)
                              : n * dd * static_cast<double>(tb);
  const double rows = n * (lv.blocks ? 20.0 : 12.0);  // row pointers of the parts
  const int launches_per_sweep = lv.ncolors;
  (void)launches_per_sweep;
  LevelBytes b{};
  const double all = static_cast<double>(lv.nnz_lo + lv.nnz_up + lv.nnz_e + lv.nnz_f);
  b.gs_fwd0 = (lv.nnz_lo + lv.nnz_e) * blk + rows + own + 4 * vec;   // b, x(w), s(w), x gathers
  b.gs_fwd = all * blk + rows + own + 5 * vec;
  b.residual = (lv.nnz_up + lv.nnz_f) * blk + rows + own + 4 * vec;  // s, x, gathers, r(w)
  b.gs_bwd = all * blk + rows + own + 4 * vec;
  const double nn = lv.nnext;
  b.restrict_ = lv.p_nnz * (4.0 + tb) + (nn + 1) * 4 + vec + nn * DP * tb;
  b.prolong = lv.p_nnz * (4.0 + tb) + (n + 1) * 4 + nn * DP * tb + 2 * vec;
  return b;
}

template <typename T>
struct BottomOf;
template <>
struct BottomOf<float> {
  static const dev::BottomLevel<float>* get(const vasmg_ctx& C) { return C.bottom32; }
};
template <>
struct BottomOf<double> {
  static const dev::BottomLevel<double>* get(const vasmg_ctx& C) { return C.bottom64; }
};

// One V-cycle: lev[0].b -> lev[0].x (Algorithm 3, recursive, zero initial guess).
// One visit of level l of the multiplicative cycle (Algorithm 3, recursive):
// smoothing from zero (zero_guess) or from the current x, residual, restriction,
// `visits` coarse visits (2 for the W-cycle above the coarsest level),
// prolongation and post-smoothing.
template <typename T, int D>
void enqueue_level(vasmg_ctx& C, int l, bool zero_guess, const int* done, hipStream_t st,
                   Profiler* prof) {
  const int L = C.L;
  const int tb = sizeof(T);
  if (l == L) {
    run_phase(prof, "coarse_solve", L, 1, static_cast<double>(C.n_coarse) * C.n_coarse * 8.0, [&] {
      if (C.cinv)
        hipLaunchKernelGGL((dev::k_coarse_apply<T, D>), dim3(1), dim3(dev::kBlock), 0, st,
                           static_cast<int>(C.n_coarse), C.cinv, static_cast<const T*>(C.lev[L].b),
                           static_cast<T*>(C.lev[L].x), done);
      else
        hipLaunchKernelGGL((dev::k_coarse_solve<T, D>), dim3(1), dim3(dev::kBlock), 0, st,
                           static_cast<int>(C.n_coarse), C.chol, static_cast<const T*>(C.lev[L].b),
                           static_cast<T*>(C.lev[L].x), done);
    });
    return;
  }
  const int npre = C.opt.n_pre, npost = C.opt.n_post;
  DevLevel& lv = C.lev[l];
  T* b = static_cast<T*>(lv.b);
  T* x = static_cast<T*>(lv.x);
  T* s = static_cast<T*>(lv.s);
  T* r = static_cast<T*>(lv.r);
  const LevelBytes by = prof ? level_bytes(C, l, tb) : LevelBytes{};
  const dev::BottomLevel<T>* bottom = BottomOf<T>::get(C);
  if (l == C.bottom_lo && bottom) {
    dev::BottomArgs<T> a;
    a.nlev = L - l;
    a.ncoarse = static_cast<int>(C.n_coarse);
    a.npre = npre;
    a.npost = npost;
    a.zero_guess = zero_guess ? 1 : 0;
    a.lev = bottom;
    a.Minv = C.cinv;
    a.b = b;
    a.x = x;
    double bytes = static_cast<double>(C.n_coarse) * C.n_coarse * 8.0;
    if (prof)
      for (int k = l; k < L; ++k) {
        const LevelBytes bk = level_bytes(C, k, tb);
        bytes += npre * bk.gs_fwd + bk.residual + bk.restrict_ + bk.prolong + npost * bk.gs_bwd;
      }
    const size_t lds = static_cast<size_t>(C.bottom_vec) * sizeof(T) + C.bottom_int * sizeof(int);
    run_phase(prof, "bottom", l, 1, bytes, [&] {
      hipLaunchKernelGGL((dev::k_bottom<T, D>), dim3(1), dim3(dev::kBottomThreads), lds, st, a,
                         done);
    });
    return;
  }
  const bool jac = C.opt.smoother == VASMG_SMOOTHER_JACOBI;
  if (jac) {
    // damped block Jacobi: x = w D^-1 b from zero, then x += w D^-1 (b - A x)
    run_phase(prof, "jacobi_pre", l, 2 * npre, npre * by.gs_fwd, [&] {
      for (int k = 0; k < npre; ++k) {
        if (zero_guess && k == 0) {
          launch_jacobi<T, D>(lv, true, b, x, done, st);
        } else {
          launch_residual_full<T, D>(lv, b, x, r, done, st);
          launch_jacobi<T, D>(lv, false, r, x, done, st);
        }
      }
    });
    run_phase(prof, "residual_full", l, 2, by.gs_fwd, [&] {
      if (npre == 0 && zero_guess) launch_fill<T>(x, static_cast<int64_t>(lv.n) * C.DP, T(0), st);
      launch_residual_full<T, D>(lv, b, x, r, done, st);
    });
  } else if (npre == 0) {
    run_phase(prof, "residual_full", l, 2, by.gs_fwd, [&] {
      if (zero_guess) launch_fill<T>(x, static_cast<int64_t>(lv.n) * C.DP, T(0), st);
      launch_residual_full<T, D>(lv, b, x, r, done, st);
    });
  } else {
    for (int k = 0; k < npre; ++k) {
      const bool z = zero_guess && k == 0;
      run_phase(prof, z ? "gs_fwd_zero" : "gs_fwd", l, lv.ncolors, z ? by.gs_fwd0 : by.gs_fwd,
                [&] { launch_gs_sweep<T, D>(lv, false, z, b, x, s, done, st); });
    }
    run_phase(prof, "residual", l, 1, by.residual,
              [&] { launch_residual_upper<T, D>(lv, s, x, r, done, st); });
  }
  run_phase(prof, "restrict", l, 1, by.restrict_,
            [&] { launch_restrict<T, D>(lv, r, static_cast<T*>(C.lev[l + 1].b), done, st); });
  const int visits = (C.opt.cycle == VASMG_CYCLE_W && l + 1 < L) ? 2 : 1;
  for (int v = 0; v < visits; ++v) enqueue_level<T, D>(C, l + 1, v == 0, done, st, prof);
  run_phase(prof, "prolong", l, 1, by.prolong, [&] {
    launch_prolong<T, D>(lv, static_cast<const T*>(C.lev[l + 1].x), x, done, st);
  });
  for (int k = 0; k < npost; ++k) {
    if (jac)
      run_phase(prof, "jacobi_post", l, 2, by.gs_bwd, [&] {
        launch_residual_full<T, D>(lv, b, x, r, done, st);
        launch_jacobi<T, D>(lv, false, r, x, done, st);
      });
    else
      run_phase(prof, "gs_bwd", l, lv.ncolors, by.gs_bwd,
                [&] { launch_gs_sweep<T, D>(lv, true, false, b, x, nullptr, done, st); });
  }
}

// z = B r with r in lev[0].b, z in lev[0].x (V- or W-cycle, or the additive
// two-level form S r + P_0 B_1 P_0^T r with B_1 the V-cycle of levels 1..L).
template <typename T, int D>
void enqueue_vcycle(vasmg_ctx& C, const int* done, hipStream_t st, Profiler* prof = nullptr) {
  if (C.opt.cycle != VASMG_CYCLE_ADDITIVE || C.L == 0) {
    enqueue_level<T, D>(C, 0, true, done, st, prof);
    return;
  }
  const int tb = sizeof(T);
  DevLevel& l0 = C.lev[0];
  T* b = static_cast<T*>(l0.b);
  T* x = static_cast<T*>(l0.x);
  T* s = static_cast<T*>(l0.s);
  const LevelBytes by = prof ? level_bytes(C, 0, tb) : LevelBytes{};
  run_phase(prof, "restrict", 0, 1, by.restrict_,
            [&] { launch_restrict<T, D>(l0, b, static_cast<T*>(C.lev[1].b), done, st); });
  enqueue_level<T, D>(C, 1, true, done, st, prof);     // V-cycle below (cycle != W)
  if (C.opt.smoother == VASMG_SMOOTHER_JACOBI) {
    T* r = static_cast<T*>(l0.r);
    const int steps = C.opt.n_pre + C.opt.n_post;
    if (steps == 0) launch_fill<T>(x, static_cast<int64_t>(l0.n) * C.DP, T(0), st);
    for (int k = 0; k < steps; ++k)
      run_phase(prof, "jacobi", 0, k == 0 ? 1 : 2, by.gs_fwd, [&] {
        if (k == 0) {
          launch_jacobi<T, D>(l0, true, b, x, done, st);
        } else {
          launch_residual_full<T, D>(l0, b, x, r, done, st);
          launch_jacobi<T, D>(l0, false, r, x, done, st);
        }
      });
  } else {
    for (int k = 0; k < C.opt.n_pre; ++k)
      run_phase(prof, k == 0 ? "gs_fwd_zero" : "gs_fwd", 0, l0.ncolors,
                k == 0 ? by.gs_fwd0 : by.gs_fwd,
                [&] { launch_gs_sweep<T, D>(l0, false, k == 0, b, x, s, done, st); });
    if (C.opt.n_pre == 0)
      launch_fill<T>(x, static_cast<int64_t>(l0.n) * C.DP, T(0), st);
    for (int k = 0; k < C.opt.n_post; ++k)
      run_phase(prof, "gs_bwd", 0, l0.ncolors, by.gs_bwd,
                [&] { launch_gs_sweep<T, D>(l0, true, false, b, x, nullptr, done, st); });
  }
  run_phase(prof, "prolong", 0, 1, by.prolong, [&] {
    launch_prolong<T, D>(l0, static_cast<const T*>(C.lev[1].x), x, done, st);
  });
}

template <int D>
void enqueue_precond(vasmg_ctx& C, const int* done, hipStream_t st) {
  if (C.vc32)
    enqueue_vcycle<float, D>(C, done, st);
  else
    enqueue_vcycle<double, D>(C, done, st);
}

// -------------------------------------------------------------------------
// PCG graphs
// -------------------------------------------------------------------------
template <int D>
void enqueue_iter_A(vasmg_ctx& C, hipStream_t st) {
  const DevLevel& l0 = C.lev[0];
  const int* done = &C.sc->done;
  const int np = launch_spmv<double, D>(l0, C.P, C.Q, C.partial, C.n_partial, done, st);
  hipLaunchKernelGGL((dev::k_finalize<dev::FIN_ALPHA>), dim3(1), dim3(1024), 0, st, C.partial, np,
                     C.sc);
  if (C.vc32)
    hipLaunchKernelGGL((dev::k_update_xr<float>), dim3(kFlatGrid), dim3(dev::kBlock), 0, st, C.n0p,
                       C.sc, C.P, C.Q, C.X, C.R, static_cast<float*>(C.lev[0].b), C.partial);
  else
    hipLaunchKernelGGL((dev::k_update_xr<double>), dim3(kFlatGrid), dim3(dev::kBlock), 0, st,
                       C.n0p, C.sc, C.P, C.Q, C.X, C.R, static_cast<double*>(nullptr), C.partial);
  hipLaunchKernelGGL((dev::k_finalize<dev::FIN_RES>), dim3(1), dim3(1024), 0, st, C.partial,
                     kFlatGrid, C.sc);
}

// z = B r; rho = r.z; beta; p = z + beta p
template <int D>
void enqueue_iter_B(vasmg_ctx& C, hipStream_t st) {
  const int* done = &C.sc->done;
  const int pc = C.opt.preconditioner;
  if (pc == VASMG_PRECOND_VASMG) {
    // the host launches this graph only while the iteration has not stopped, so
    // the V-cycle kernels do not read the flag (it would head their load chains)
    enqueue_precond<D>(C, nullptr, st);
    if (C.vc32) {
      hipLaunchKernelGGL((dev::k_dot<float>), dim3(kFlatGrid), dim3(dev::kBlock), 0, st, C.n0p, C.R,
                         static_cast<const float*>(C.lev[0].x), C.partial, done);
      hipLaunchKernelGGL((dev::k_finalize<dev::FIN_BETA>), dim3(1), dim3(1024), 0, st, C.partial,
                         kFlatGrid, C.sc);
      hipLaunchKernelGGL((dev::k_update_p<float>), dim3(kFlatGrid), dim3(dev::kBlock), 0, st, C.n0p,
                         C.sc, static_cast<const float*>(C.lev[0].x), C.P);
    } else {
      hipLaunchKernelGGL((dev::k_dot<double>), dim3(kFlatGrid), dim3(dev::kBlock), 0, st, C.n0p,
                         C.R, static_cast<const double*>(C.lev[0].x), C.partial, done);
      hipLaunchKernelGGL((dev::k_finalize<dev::FIN_BETA>), dim3(1), dim3(1024), 0, st, C.partial,
                         kFlatGrid, C.sc);
      hipLaunchKernelGGL((dev::k_update_p<double>), dim3(kFlatGrid), dim3(dev::kBlock), 0, st,
                         C.n0p, C.sc, static_cast<const double*>(C.lev[0].x), C.P);
    }
  } else {
    const double* z = C.R;
    if (pc == VASMG_PRECOND_JACOBI) {
      hipLaunchKernelGGL((dev::k_jacobi<D>), dim3(grid_for(C.n0, dev::kBlock)), dim3(dev::kBlock), 0,
                         st, C.n0, C.lev[0].diag64, C.R, C.Z, done);
      z = C.Z;
    }
    hipLaunchKernelGGL((dev::k_dot<double>), dim3(kFlatGrid), dim3(dev::kBlock), 0, st, C.n0p, C.R,
                       z, C.partial, done);
    hipLaunchKernelGGL((dev::k_finalize<dev::FIN_BETA>), dim3(1), dim3(1024), 0, st, C.partial,
                       kFlatGrid, C.sc);
    hipLaunchKernelGGL((dev::k_update_p<double>), dim3(kFlatGrid), dim3(dev::kBlock), 0, st, C.n0p,
                       C.sc, z, C.P);
  }
}

// -------------------------------------------------------------------------
// Autotuner: lanes per block row of each level, by timing the level's own
// kernels (forward zero-guess sweep + residual + backward sweep, and the fine
// FP64 SpMV) with hipEvents; the fastest median of three wins.
// -------------------------------------------------------------------------
template <typename T, int D>
double time_level(vasmg_ctx& C, int l, hipStream_t st) {
  DevLevel& lv = C.lev[l];
  T* b = static_cast<T*>(lv.b);
  T* x = static_cast<T*>(lv.x);
  T* s = static_cast<T*>(lv.s);
  T* r = static_cast<T*>(lv.r);
  hipEvent_t e0, e1;
  HIP_CHECK(hipEventCreate(&e0));
  HIP_CHECK(hipEventCreate(&e1));
  std::vector<float> t;
  for (int rep = 0; rep < 4; ++rep) {
    HIP_CHECK(hipEventRecord(e0, st));
    launch_gs_sweep<T, D>(lv, false, true, b, x, s, nullptr, st);
    launch_residual_upper<T, D>(lv, s, x, r, nullptr, st);
    launch_gs_sweep<T, D>(lv, true, false, b, x, nullptr, nullptr, st);
    HIP_CHECK(hipEventRecord(e1, st));
    HIP_CHECK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
    if (rep > 0) t.push_back(ms);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  std::sort(t.begin(), t.end());
  return t[t.size() / 2];
}

template <int D>
double time_spmv(vasmg_ctx& C, hipStream_t st) {
  hipEvent_t e0, e1;
  HIP_CHECK(hipEventCreate(&e0));
  HIP_CHECK(hipEventCreate(&e1));
  std::vector<float> t;
  for (int rep = 0; rep < 4; ++rep) {
    HIP_CHECK(hipEventRecord(e0, st));
    launch_spmv<double, D>(C.lev[0], C.P, C.Q, C.partial, C.n_partial, nullptr, st);
    HIP_CHECK(hipEventRecord(e1, st));
    HIP_CHECK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
    if (rep > 0) t.push_back(ms);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  std::sort(t.begin(), t.end());
  return t[t.size() / 2];
}

template <int D>
void autotune(vasmg_ctx& C) {
  hipStream_t st = C.cap_stream;
  const int last = C.opt.preconditioner == VASMG_PRECOND_VASMG ? C.L - 1 : -1;
  for (int l = 0; l <= last; ++l) {
    DevLevel& lv = C.lev[l];
    const int64_t len = static_cast<int64_t>(lv.n) * C.DP;
    if (C.vc32) {
      launch_fill<float>(static_cast<float*>(lv.b), len, 1.0f, st);
      launch_fill<float>(static_cast<float*>(lv.x), len, 0.0f, st);
    } else {
      launch_fill<double>(static_cast<double*>(lv.b), len, 1.0, st);
      launch_fill<double>(static_cast<double*>(lv.x), len, 0.0, st);
    }
    std::vector<int> cand = lv.cells ? (D == 3 ? std::vector<int>{8, 16, 32, 64}
                                               : std::vector<int>{4, 8, 16, 32})
                                     : std::vector<int>{4, 8, 16, 32};
    double best = 1e30;
    int bestG = lv.G;
    for (int g : cand) {
      lv.G = g;
      const double ms = C.vc32 ? time_level<float, D>(C, l, st) : time_level<double, D>(C, l, st);
      if (ms < best) {
        best = ms;
        bestG = g;
      }
    }
    lv.G = bestG;
    if (C.opt.verbose)
      std::fprintf(stderr, "[vasmg] autotune level %d: %d lanes per row (%.3f ms per V(1,1) pass)\n",
                   l, bestG, best);
  }
  launch_fill<double>(C.P, C.n0p, 1.0, st);
  double best = 1e30;
  int bestG = C.lev[0].Gspmv;
  for (int g : {4, 8, 16, 32}) {
    C.lev[0].Gspmv = g;
    const double ms = time_spmv<D>(C, st);
    if (ms < best) {
      best = ms;
      bestG = g;
    }
  }
  C.lev[0].Gspmv = bestG;
  if (C.opt.verbose)
    std::fprintf(stderr, "[vasmg] autotune fine SpMV: %d lanes per row (%.3f ms)\n", bestG, best);
  HIP_CHECK(hipStreamSynchronize(st));
}

std::mutex g_capture_mutex;   // one graph capture at a time in the process

hipGraphExec_t capture(vasmg_ctx& C, void (*fn)(vasmg_ctx&, hipStream_t)) {
  std::lock_guard<std::mutex> lock(g_capture_mutex);
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  // relaxed: other threads (a server's slots) may upload, copy or free meanwhile;
  // the captured sequence itself is kernel launches only
  HIP_CHECK(hipStreamBeginCapture(C.cap_stream, hipStreamCaptureModeRelaxed));
  fn(C, C.cap_stream);
  HIP_CHECK(hipGetLastError());
  HIP_CHECK(hipStreamEndCapture(C.cap_stream, &g));
  HIP_CHECK(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
  HIP_CHECK(hipGraphDestroy(g));
  return ge;
}

template <int D>
void ensure_graphs(vasmg_ctx& C) {
  if (!C.gA) C.gA = capture(C, &enqueue_iter_A<D>);
  if (!C.gB) C.gB = capture(C, &enqueue_iter_B<D>);
}

// -------------------------------------------------------------------------
// Packed problems: the shared SpMV and V-cycle, per-segment scalars
// -------------------------------------------------------------------------
// q = A p; alpha_s; x, r updates; ||r||_s and the stopping test; running count
template <int D>
void enqueue_packed_A(vasmg_ctx& C, hipStream_t st) {
  launch_spmv<double, D>(C.lev[0], C.P, C.Q, nullptr, 0, nullptr, st);
  hipLaunchKernelGGL((dev::k_seg_dot<dev::FIN_ALPHA, false, double>), dim3(C.nseg), dim3(dev::kBlock), 0,
                     st, C.seg_ptr, C.seg_rows, C.DP, C.P, C.Q, C.ssc);
  if (C.vc32)
    hipLaunchKernelGGL((dev::k_seg_update_xr<float>), dim3(kFlatGrid), dim3(dev::kBlock), 0, st, C.n0p,
                       C.DP, C.seg_of_row, C.ssc, C.P, C.Q, C.X, C.R, static_cast<float*>(C.lev[0].b));
  else
    hipLaunchKernelGGL((dev::k_seg_update_xr<double>), dim3(kFlatGrid), dim3(dev::kBlock), 0, st, C.n0p,
                       C.DP, C.seg_of_row, C.ssc, C.P, C.Q, C.X, C.R, static_cast<double*>(nullptr));
  hipLaunchKernelGGL((dev::k_seg_dot<dev::FIN_RES, false, double>), dim3(C.nseg), dim3(dev::kBlock), 0,
                     st, C.seg_ptr, C.seg_rows, C.DP, C.R, C.R, C.ssc);
  hipLaunchKernelGGL(dev::k_seg_running, dim3(1), dim3(dev::kBlock), 0, st, C.nseg, C.ssc,
                     C.seg_running);
}

// z = B r (the whole packed V-cycle); rho_s, beta_s; p = z + beta_s p
template <int D>
void enqueue_packed_B(vasmg_ctx& C, hipStream_t st) {
  enqueue_precond<D>(C, nullptr, st);
  if (C.vc32) {
    const float* z = static_cast<const float*>(C.lev[0].x);
    hipLaunchKernelGGL((dev::k_seg_dot<dev::FIN_BETA, false, float>), dim3(C.nseg), dim3(dev::kBlock), 0,
                       st, C.seg_ptr, C.seg_rows, C.DP, C.R, z, C.ssc);
    hipLaunchKernelGGL((dev::k_seg_update_p<float>), dim3(kFlatGrid), dim3(dev::kBlock), 0, st, C.n0p,
                       C.DP, C.seg_of_row, C.ssc, z, C.P);
  } else {
    const double* z = static_cast<const double*>(C.lev[0].x);
    hipLaunchKernelGGL((dev::k_seg_dot<dev::FIN_BETA, false, double>), dim3(C.nseg), dim3(dev::kBlock),
                       0, st, C.seg_ptr, C.seg_rows, C.DP, C.R, z, C.ssc);
    hipLaunchKernelGGL((dev::k_seg_update_p<double>), dim3(kFlatGrid), dim3(dev::kBlock), 0, st, C.n0p,
                       C.DP, C.seg_of_row, C.ssc, z, C.P);
  }
}

template <int D>
void ensure_packed_graphs(vasmg_ctx& C) {
  if (!C.sgA) C.sgA = capture(C, &enqueue_packed_A<D>);
  if (!C.sgB) C.sgB = capture(C, &enqueue_packed_B<D>);
}

// All segments from x0 = 0: d_rhs / d_x the parts' user vectors one after the
// other ([sum n_vertices][D], device); info[nseg].
template <int D>
int solve_packed(vasmg_ctx& C, const double* d_rhs, double* d_x, double rtol, hipStream_t st,
                 vasmg_solve_info* info) {
  ensure_packed_graphs<D>(C);
  const int n0 = C.n0;
  const int64_t n0p = C.n0p;
  const int nseg = C.nseg;
  HIP_CHECK(hipEventRecord(C.ev[0], st));
  hipLaunchKernelGGL((dev::k_gather_user<double, double, D>), dim3(grid_for(n0, dev::kBlock)),
                     dim3(dev::kBlock), 0, st, n0, C.user_map, d_rhs, C.F,
                     static_cast<const uint8_t*>(C.lev[0].fixed));
  hipLaunchKernelGGL((dev::k_seg_dot<dev::FIN_NORMF, false, double>), dim3(nseg), dim3(dev::kBlock), 0, st,
                     C.seg_ptr, C.seg_rows, C.DP, C.F, C.F, C.ssc);
  hipLaunchKernelGGL(dev::k_seg_start, dim3(grid_for(nseg, dev::kBlock)), dim3(dev::kBlock), 0, st, nseg,
                     C.ssc, rtol);
  launch_fill<double>(C.X, n0p, 0.0, st);
  launch_fill<double>(C.P, n0p, 0.0, st);
  hipLaunchKernelGGL((dev::k_convert<double, double>), dim3(kFlatGrid), dim3(dev::kBlock), 0, st, n0p, C.F,
                     C.R);
  if (C.vc32)
    hipLaunchKernelGGL((dev::k_convert<double, float>), dim3(kFlatGrid), dim3(dev::kBlock), 0, st, n0p,
                       C.R, static_cast<float*>(C.lev[0].b));
  hipLaunchKernelGGL(dev::k_seg_running, dim3(1), dim3(dev::kBlock), 0, st, nseg, C.ssc, C.seg_running);
  int running = 0;
  HIP_CHECK(hipMemcpyAsync(&running, C.seg_running, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  if (running > 0) {
    // Algorithm 2 initialisation for every segment: z = B r, p = z, rho = r^T z
    HIP_CHECK(hipGraphLaunch(C.sgB, st));
    for (int k = 0; k < C.opt.max_iters; ++k) {
      HIP_CHECK(hipGraphLaunch(C.sgA, st));
      HIP_CHECK(hipMemcpyAsync(&running, C.seg_running, sizeof(int), hipMemcpyDeviceToHost, st));
      HIP_CHECK(hipStreamSynchronize(st));
      if (running == 0) break;
      HIP_CHECK(hipGraphLaunch(C.sgB, st));
    }
  }
  // true residuals, scatter
  launch_spmv<double, D>(C.lev[0], C.X, C.Q, nullptr, 0, nullptr, st);
  hipLaunchKernelGGL((dev::k_seg_dot<dev::FIN_TRUE, true, double>), dim3(nseg), dim3(dev::kBlock), 0, st,
                     C.seg_ptr, C.seg_rows, C.DP, C.F, C.Q, C.ssc);
  launch_fill<double>(d_x, C.H.n_mesh_vertices * D, 0.0, st);
  hipLaunchKernelGGL((dev::k_scatter_user<double, double, D>), dim3(grid_for(n0, dev::kBlock)),
                     dim3(dev::kBlock), 0, st, n0, C.user_map, C.X, d_x);
  std::vector<Scalars> hs(nseg);
  HIP_CHECK(hipMemcpyAsync(hs.data(), C.ssc, sizeof(Scalars) * nseg, hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipEventRecord(C.ev[1], st));
  HIP_CHECK(hipStreamSynchronize(st));
  HIP_CHECK(hipGetLastError());
  float ms = 0.f;
  HIP_CHECK(hipEventElapsedTime(&ms, C.ev[0], C.ev[1]));
  int worst = VASMG_OK;
  for (int k = 0; k < nseg; ++k) {
    const Scalars& s = hs[k];
    vasmg_solve_info& o = info[k];
    std::memset(&o, 0, sizeof(o));
    const bool conv = s.status != 5 && (s.normF == 0.0 || s.res / s.normF < rtol);
    o.iterations = s.iters;
    o.converged = conv ? 1 : 0;
    o.rel_res = s.normF > 0 ? s.res / s.normF : 0.0;
    o.rel_res_true = s.normF > 0 ? s.res_true / s.normF : 0.0;
    o.t_solve_ms = ms;
    o.status = s.status == 5 ? VASMG_EBREAKDOWN : (conv ? VASMG_OK : VASMG_ENOTCONV);
    if (o.status == VASMG_EBREAKDOWN)
      worst = VASMG_EBREAKDOWN;
    else if (o.status == VASMG_ENOTCONV && worst == VASMG_OK)
      worst = VASMG_ENOTCONV;
  }
  return worst;
}

// -------------------------------------------------------------------------
// one right-hand side: d_rhs/d_x user layout [nv][D] (device), d_x0 may be NULL
// -------------------------------------------------------------------------
template <int D>
int solve_one(vasmg_ctx& C, const double* d_rhs, const double* d_x0, double* d_x, double rtol,
              hipStream_t st, vasmg_solve_info* info) {
  ensure_graphs<D>(C);
  const int n0 = C.n0;
  const int64_t n0p = C.n0p;
  const int gflat = kFlatGrid;
  HIP_CHECK(hipEventRecord(C.ev[0], st));
  hipLaunchKernelGGL((dev::k_gather_user<double, double, D>), dim3(grid_for(n0, dev::kBlock)),
                     dim3(dev::kBlock), 0, st, n0, C.user_map, d_rhs, C.F,
                     static_cast<const uint8_t*>(C.lev[0].fixed));
  // ||F||, then r = F - A x0 (or F), p = 0
  hipLaunchKernelGGL((dev::k_dot<double>), dim3(gflat), dim3(dev::kBlock), 0, st, n0p, C.F, C.F,
                     C.partial, static_cast<const int*>(nullptr));
  hipLaunchKernelGGL((dev::k_finalize<dev::FIN_NORMF>), dim3(1), dim3(1024), 0, st, C.partial, gflat,
                     C.sc);
  *C.h_rtol = rtol;
  HIP_CHECK(hipMemcpyAsync(&C.sc->rtol, C.h_rtol, sizeof(double), hipMemcpyHostToDevice, st));
  if (d_x0) {
    hipLaunchKernelGGL((dev::k_gather_user<double, double, D>), dim3(grid_for(n0, dev::kBlock)),
                       dim3(dev::kBlock), 0, st, n0, C.user_map, d_x0, C.X,
                       static_cast<const uint8_t*>(C.lev[0].fixed));
    launch_spmv<double, D>(C.lev[0], C.X, C.Q, nullptr, 0, nullptr, st);
    hipLaunchKernelGGL(dev::k_sub_norm, dim3(gflat), dim3(dev::kBlock), 0, st, n0p, C.F, C.Q, C.R,
                       C.partial);
    hipLaunchKernelGGL((dev::k_finalize<dev::FIN_TRUE>), dim3(1), dim3(1024), 0, st, C.partial, gflat,
                       C.sc);
  } else {
    launch_fill<double>(C.X, n0p, 0.0, st);
    hipLaunchKernelGGL((dev::k_convert<double, double>), dim3(gflat), dim3(dev::kBlock), 0, st, n0p,
                       C.F, C.R);
  }
  launch_fill<double>(C.P, n0p, 0.0, st);
  if (C.vc32 && C.opt.preconditioner == VASMG_PRECOND_VASMG)
    hipLaunchKernelGGL((dev::k_convert<double, float>), dim3(gflat), dim3(dev::kBlock), 0, st, n0p,
                       C.R, static_cast<float*>(C.lev[0].b));
  HIP_CHECK(hipGetLastError());
  HIP_CHECK(hipMemcpyAsync(C.h_sc, C.sc, sizeof(Scalars), hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  const double normF = C.h_sc->normF;
  int status = VASMG_OK;
  double t_a = 0.0, t_b = 0.0;
  const bool prof = C.opt.profile != 0;
  bool done = false;
  if (!std::isfinite(normF)) {
    status = VASMG_EBREAKDOWN;
    done = true;
  } else if (normF == 0.0) {
    launch_fill<double>(C.X, n0p, 0.0, st);
    done = true;
  } else if (d_x0 && C.h_sc->res_true / normF < rtol) {
    done = true;
  }
  if (!done) {
    // Algorithm 2 initialisation: z = B r, p = z, rho = r^T z
    if (prof) HIP_CHECK(hipEventRecord(C.ev[2], st));
    HIP_CHECK(hipGraphLaunch(C.gB, st));
    if (prof) HIP_CHECK(hipEventRecord(C.ev[3], st));
    int k = 0;
    while (k < C.opt.max_iters) {
      if (prof) {
        HIP_CHECK(hipEventSynchronize(C.ev[3]));
        float ms = 0.f;
        HIP_CHECK(hipEventElapsedTime(&ms, C.ev[2], C.ev[3]));
        t_b += ms;
        HIP_CHECK(hipEventRecord(C.ev[2], st));
      }
      HIP_CHECK(hipGraphLaunch(C.gA, st));
      HIP_CHECK(hipMemcpyAsync(C.h_sc, C.sc, sizeof(Scalars), hipMemcpyDeviceToHost, st));
      if (prof) HIP_CHECK(hipEventRecord(C.ev[3], st));
      HIP_CHECK(hipStreamSynchronize(st));
      if (prof) {
        float ms = 0.f;
        HIP_CHECK(hipEventElapsedTime(&ms, C.ev[2], C.ev[3]));
        t_a += ms;
      }
      ++k;
      if (C.h_sc->done) break;
      if (prof) HIP_CHECK(hipEventRecord(C.ev[2], st));
      HIP_CHECK(hipGraphLaunch(C.gB, st));
      if (prof) HIP_CHECK(hipEventRecord(C.ev[3], st));
    }
  }
  // true residual, scatter
  launch_spmv<double, D>(C.lev[0], C.X, C.Q, nullptr, 0, nullptr, st);
  hipLaunchKernelGGL(dev::k_sub_norm, dim3(gflat), dim3(dev::kBlock), 0, st, n0p, C.F, C.Q,
                     static_cast<double*>(nullptr), C.partial);
  hipLaunchKernelGGL((dev::k_finalize<dev::FIN_TRUE>), dim3(1), dim3(1024), 0, st, C.partial, gflat,
                     C.sc);
  launch_fill<double>(d_x, C.H.n_mesh_vertices * D, 0.0, st);
  hipLaunchKernelGGL((dev::k_scatter_user<double, double, D>), dim3(grid_for(n0, dev::kBlock)),
                     dim3(dev::kBlock), 0, st, n0, C.user_map, C.X, d_x);
  HIP_CHECK(hipMemcpyAsync(C.h_sc, C.sc, sizeof(Scalars), hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipEventRecord(C.ev[1], st));
  HIP_CHECK(hipStreamSynchronize(st));
  HIP_CHECK(hipGetLastError());
  const Scalars& s = *C.h_sc;
  if (status == VASMG_OK) {
    if (s.status == 5)
      status = VASMG_EBREAKDOWN;
    else if (normF != 0.0 && !(s.res / normF < rtol) && !(d_x0 && s.iters == 0))
      status = VASMG_ENOTCONV;
  }
  if (info) {
    float ms = 0.f;
    HIP_CHECK(hipEventElapsedTime(&ms, C.ev[0], C.ev[1]));
    info->iterations = s.iters;
    info->converged = status == VASMG_OK ? 1 : 0;
    info->status = status;
    info->reserved = 0;
    info->rel_res = normF > 0 ? s.res / normF : 0.0;
    info->rel_res_true = normF > 0 ? s.res_true / normF : 0.0;
    info->t_solve_ms = ms;
    info->t_spmv_ms = t_a;
    info->t_precond_ms = t_b;
    info->t_vector_ms = 0.0;
    info->bytes_model = 0.0;
  }
  return status;
}

// -------------------------------------------------------------------------
// Block right-hand sides: K PCG recurrences that share every matrix read
// (vectors [row][K][DP], per-column scalars; kernels in block.hpp).
// -------------------------------------------------------------------------
#define DISPATCH_K(Kv, ...)                                  \
  switch (Kv) {                                              \
    case 4: { constexpr int KK = 4; __VA_ARGS__; } break;    \
    case 8: { constexpr int KK = 8; __VA_ARGS__; } break;    \
    default: { constexpr int KK = 16; __VA_ARGS__; } break;  \
  }

void upload_block(vasmg_ctx& C, int K) {
  if (K != 4 && K != 8 && K != 16)
    throw vasmg::Error{VASMG_EINVAL, "block_rhs must be 0, 4, 8 or 16"};
  if (C.opt.preconditioner != VASMG_PRECOND_VASMG || C.opt.n_pre < 1)
    throw vasmg::Error{VASMG_EINVAL, "block_rhs needs the V-ASMG preconditioner with n_pre >= 1"};
  if (C.n_coarse * K > dev::kCoarseMax)
    throw vasmg::Error{VASMG_EINVAL, "block_rhs: coarsest level too large for K columns"};
  C.K = K;
  const int tb = C.vc32 ? 4 : 8;
  const int nl = C.L + 1;
  C.kb.assign(nl, nullptr);
  C.kx.assign(nl, nullptr);
  C.ks.assign(nl, nullptr);
  C.kr.assign(nl, nullptr);
  for (int l = 0; l < nl; ++l) {
    // the fine level keeps the padded stride; coarse levels store D components
    const int stride = l == 0 ? C.DP : C.d;
    const int64_t bytes = static_cast<int64_t>(C.lev[l].n) * K * stride * tb;
    for (auto* v : {&C.kb, &C.kx, &C.ks, &C.kr}) {
      (*v)[l] = C.dalloc<char>(bytes);
      C.clear((*v)[l], bytes);
    }
  }
  const int64_t n = C.n0p * K;
  for (double** v : {&C.kF, &C.kX, &C.kR, &C.kP, &C.kQ}) {
    *v = C.dalloc<double>(n);
    C.clear(*v, sizeof(double) * n);
  }
  if (!C.vc32) C.kb[0] = C.kR;    // FP64 V-cycle: its fine right-hand side is r
  // one partial per workgroup of the block SpMV: sized for the wide lane groups
  // (fewest rows per workgroup), whichever the heuristic, the tuner or the
  // block_lanes option puts on the fine level
  C.kn_partial = std::max(kFlatGrid, grid_for(C.n0, dev::kBlock / dev::kPointLanesWide));
  // lanes per block row: on the cell levels the narrow groups (their rows go
  // through LDS in chunks, which keeps a long row's loads in flight with few
  // slots, and more cells fit on a compute unit: 65^3, K = 16, 56.8 ms per
  // block solve against 58.3 with the wide groups on the long-row levels); on
  // the point level the wide groups for long rows
  for (int l = 0; l < C.L; ++l) {
    DevLevel& lv = C.lev[l];
    const double avg = lv.n > 0 ? static_cast<double>(lv.nnz) / lv.n : 0.0;
    if (lv.cells)
      lv.mcGL = dev::kCellLanesNarrow;
    else
      lv.mcGL = avg >= 24.0 ? dev::kPointLanesWide : dev::kPointLanesNarrow;
    if (C.opt.block_lanes != 0) {   // forced: narrow (1) or wide (2) groups everywhere
      const bool wide = C.opt.block_lanes == 2;
      lv.mcGL = lv.cells ? (wide ? dev::kCellLanesWide : dev::kCellLanesNarrow)
                         : (wide ? dev::kPointLanesWide : dev::kPointLanesNarrow);
    }
  }
  C.kpartial = C.dalloc<double>(static_cast<int64_t>(C.kn_partial) * K);
  C.ksc = C.dalloc<Scalars>(K);
  C.clear(C.ksc, sizeof(Scalars) * K);
  C.kh_sc = reinterpret_cast<Scalars*>(static_cast<char*>(C.pinned) + 512);
}

#define DISPATCH_POINT_GL(GLv, ...)                                         \
  if ((GLv) == dev::kPointLanesWide) {                                      \
    constexpr int GL = dev::kPointLanesWide; __VA_ARGS__;                   \
  } else {                                                                  \
    constexpr int GL = dev::kPointLanesNarrow; __VA_ARGS__;                 \
  }
#define DISPATCH_CELL_GL(GLv, ...)                                          \
  if ((GLv) == dev::kCellLanesWide) {                                       \
    constexpr int GL = dev::kCellLanesWide; __VA_ARGS__;                    \
  } else {                                                                  \
    constexpr int GL = dev::kCellLanesNarrow; __VA_ARGS__;                  \
  }

template <int D, int K>
int launch_spmv_mc(const vasmg_ctx& C, const double* x, double* y, double* partial,
                   hipStream_t st) {
  const DevLevel& lv = C.lev[0];
  int grid = 0;
  DISPATCH_POINT_GL(lv.mcGL, {
    grid = grid_for(lv.n, dev::kBlock / GL);
    if (partial && grid > C.kn_partial)
      throw vasmg::Error{VASMG_EINVAL, "internal: block SpMV partial buffer too small"};
    if (partial)
      hipLaunchKernelGGL((dev::k_spmv_mc<D, K, GL, true>), dim3(grid), dim3(dev::kBlock), 0, st,
                         lv.n, LevelMats<double>::L(lv), LevelMats<double>::U(lv), lv.diag64, x, y,
                         partial);
    else
      hipLaunchKernelGGL((dev::k_spmv_mc<D, K, GL, false>), dim3(grid), dim3(dev::kBlock), 0, st,
                         lv.n, LevelMats<double>::L(lv), LevelMats<double>::U(lv), lv.diag64, x, y,
                         partial);
  });
  return grid;
}

template <typename T, int D, int K>
void launch_gs_sweep_mc(const DevLevel& lv, bool backward, bool zero_guess, const T* b, T* x,
                        T* s, hipStream_t st) {
  const dev::Part<T> Lp = LevelMats<T>::L(lv), Up = LevelMats<T>::U(lv);
  for (int q = 0; q < lv.ncolors; ++q) {
    const int c = backward ? lv.ncolors - 1 - q : q;
    const int mode = backward ? 2 : (zero_guess ? 0 : 1);
    const int r0 = lv.color_ptr[c], nr = lv.color_ptr[c + 1] - r0;
    if (nr <= 0) continue;
    if (lv.cells) {
      const T* M = LevelMats<T>::cellM(lv);
      DISPATCH_CELL_GL(lv.mcGL, {
        const dim3 grid(nr), blk((1 << D) * GL);
        if (mode == 0)
          hipLaunchKernelGGL((dev::k_gs_cell_mc<T, D, K, GL, 0>), grid, blk, 0, st, r0, lv.cell_ptr,
                             Lp, Up, M, b, x, s);
        else if (mode == 1)
          hipLaunchKernelGGL((dev::k_gs_cell_mc<T, D, K, GL, 1>), grid, blk, 0, st, r0, lv.cell_ptr,
                             Lp, Up, M, b, x, s);
        else
          hipLaunchKernelGGL((dev::k_gs_cell_mc<T, D, K, GL, 2>), grid, blk, 0, st, r0, lv.cell_ptr,
                             Lp, Up, M, b, x, static_cast<T*>(nullptr));
      });
    } else {
      const T* dg = LevelMats<T>::diag(lv);
      DISPATCH_POINT_GL(lv.mcGL, {
        const dim3 grid(grid_for(nr, dev::kBlock / GL)), blk(dev::kBlock);
        if (mode == 0)
          hipLaunchKernelGGL((dev::k_gs_color_mc<T, D, K, GL, 0>), grid, blk, 0, st, r0, nr, Lp,
                             Up, dg, b, x, s);
        else if (mode == 1)
          hipLaunchKernelGGL((dev::k_gs_color_mc<T, D, K, GL, 1>), grid, blk, 0, st, r0, nr, Lp,
                             Up, dg, b, x, s);
        else
          hipLaunchKernelGGL((dev::k_gs_color_mc<T, D, K, GL, 2>), grid, blk, 0, st, r0, nr, Lp,
                             Up, dg, b, x, static_cast<T*>(nullptr));
      });
    }
  }
}

// r = b - A x of a level from the forward sweep's saved lower sums s
template <typename T, int D, int K>
void launch_residual_mc(const DevLevel& lv, const T* s, const T* x, T* r, hipStream_t st) {
  if (lv.cells) {
    DISPATCH_CELL_GL(lv.mcGL, {
      hipLaunchKernelGGL((dev::k_cell_residual_mc<T, D, K, GL>), dim3(lv.ncells), dim3((1 << D) * GL), 0,
                         st, lv.cell_ptr, LevelMats<T>::L(lv), LevelMats<T>::U(lv),
                         LevelMats<T>::cellM(lv), s, x, r);
    });
  } else {
    DISPATCH_POINT_GL(lv.mcGL, {
      hipLaunchKernelGGL((dev::k_residual_upper_mc<T, D, K, GL>), dim3(grid_for(lv.n, dev::kBlock / GL)),
                         dim3(dev::kBlock), 0, st, lv.n, LevelMats<T>::U(lv), LevelMats<T>::diag(lv), s, x,
                         r);
    });
  }
}

template <typename T, int D, int K>
void enqueue_vcycle_mc(vasmg_ctx& C, hipStream_t st) {
  const int L = C.L;
  for (int l = 0; l < L; ++l) {
    const DevLevel& lv = C.lev[l];
    T* b = static_cast<T*>(C.kb[l]);
    T* x = static_cast<T*>(C.kx[l]);
    T* s = static_cast<T*>(C.ks[l]);
    T* r = static_cast<T*>(C.kr[l]);
    for (int k = 0; k < C.opt.n_pre; ++k) launch_gs_sweep_mc<T, D, K>(lv, false, k == 0, b, x, s, st);
    launch_residual_mc<T, D, K>(lv, s, x, r, st);
    const dim3 rgrid(grid_for(lv.nnext, dev::kBlock / K));
    if (l == 0)
      hipLaunchKernelGGL((dev::k_restrict_mc<T, D, K, dev::Pad<D>::value>), rgrid, dim3(dev::kBlock),
                         0, st, lv.nnext, lv.pt_ptr, lv.pt_idx, LevelMats<T>::ptw(lv), r,
                         static_cast<T*>(C.kb[l + 1]));
    else
      hipLaunchKernelGGL((dev::k_restrict_mc<T, D, K, D>), rgrid, dim3(dev::kBlock), 0, st,
                         lv.nnext, lv.pt_ptr, lv.pt_idx, LevelMats<T>::ptw(lv), r,
                         static_cast<T*>(C.kb[l + 1]));
  }
  const int nco = static_cast<int>(C.n_coarse);
  const T* bL = static_cast<const T*>(C.kb[L]);
  T* xL = static_cast<T*>(C.kx[L]);
  if (L == 0 && C.cinv)
    hipLaunchKernelGGL((dev::k_coarse_apply_mc<T, D, K, dev::Pad<D>::value>), dim3(1),
                       dim3(dev::kBlock), 0, st, nco, C.cinv, bL, xL);
  else if (L == 0)
    hipLaunchKernelGGL((dev::k_coarse_solve_mc<T, D, K, dev::Pad<D>::value>), dim3(1),
                       dim3(dev::kBlock), 0, st, nco, C.chol, bL, xL);
  else if (C.cinv)
    hipLaunchKernelGGL((dev::k_coarse_apply_mc<T, D, K, D>), dim3(1), dim3(dev::kBlock), 0, st, nco,
                       C.cinv, bL, xL);
  else
    hipLaunchKernelGGL((dev::k_coarse_solve_mc<T, D, K, D>), dim3(1), dim3(dev::kBlock), 0, st, nco,
                       C.chol, bL, xL);
  for (int l = L - 1; l >= 0; --l) {
    const DevLevel& lv = C.lev[l];
    T* b = static_cast<T*>(C.kb[l]);
    T* x = static_cast<T*>(C.kx[l]);
    const dim3 pgrid(grid_for(lv.n, dev::kBlock / K));
    if (l == 0)
      hipLaunchKernelGGL((dev::k_prolong_mc<T, D, K, dev::Pad<D>::value>), pgrid, dim3(dev::kBlock),
                         0, st, lv.n, lv.p_ptr, lv.p_idx, LevelMats<T>::pw(lv),
                         static_cast<const T*>(C.kx[l + 1]), x, static_cast<const uint8_t*>(lv.fixed));
    else
      hipLaunchKernelGGL((dev::k_prolong_mc<T, D, K, D>), pgrid, dim3(dev::kBlock), 0, st, lv.n,
                         lv.p_ptr, lv.p_idx, LevelMats<T>::pw(lv),
                         static_cast<const T*>(C.kx[l + 1]), x, static_cast<const uint8_t*>(lv.fixed));
    for (int k = 0; k < C.opt.n_post; ++k)
      launch_gs_sweep_mc<T, D, K>(lv, true, false, b, x, nullptr, st);
  }
}

// q = A p, alpha, x += alpha p, r -= alpha q, ||r|| and the stop flags (per column)
template <int D, int K>
void enqueue_iter_A_mc(vasmg_ctx& C, hipStream_t st) {
  constexpr int DP = dev::Pad<D>::value;
  const int64_t n = C.n0p * K;
  const int np = launch_spmv_mc<D, K>(C, C.kP, C.kQ, C.kpartial, st);
  hipLaunchKernelGGL((dev::k_finalize_mc<dev::FIN_ALPHA, K>), dim3(K), dim3(dev::kBlock), 0, st,
                     C.kpartial, np, C.ksc);
  if (C.vc32)
    hipLaunchKernelGGL((dev::k_update_xr_mc<float, K, DP>), dim3(kFlatGrid), dim3(dev::kBlock), 0,
                       st, n, C.ksc, C.kP, C.kQ, C.kX, C.kR, static_cast<float*>(C.kb[0]),
                       C.kpartial);
  else
    hipLaunchKernelGGL((dev::k_update_xr_mc<double, K, DP>), dim3(kFlatGrid), dim3(dev::kBlock), 0,
                       st, n, C.ksc, C.kP, C.kQ, C.kX, C.kR, static_cast<double*>(nullptr),
                       C.kpartial);
  hipLaunchKernelGGL((dev::k_finalize_mc<dev::FIN_RES, K>), dim3(K), dim3(dev::kBlock), 0, st,
                     C.kpartial, kFlatGrid, C.ksc);
}

// z = B r, rho = r.z, beta, p = z + beta p (per column)
template <int D, int K>
void enqueue_iter_B_mc(vasmg_ctx& C, hipStream_t st) {
  constexpr int DP = dev::Pad<D>::value;
  const int64_t n = C.n0p * K;
  if (C.vc32) {
    enqueue_vcycle_mc<float, D, K>(C, st);
    hipLaunchKernelGGL((dev::k_dot_mc<K, DP, float>), dim3(kFlatGrid), dim3(dev::kBlock), 0, st, n,
                       C.kR, static_cast<const float*>(C.kx[0]), C.kpartial);
  } else {
    enqueue_vcycle_mc<double, D, K>(C, st);
    hipLaunchKernelGGL((dev::k_dot_mc<K, DP, double>), dim3(kFlatGrid), dim3(dev::kBlock), 0, st,
                       n, C.kR, static_cast<const double*>(C.kx[0]), C.kpartial);
  }
  hipLaunchKernelGGL((dev::k_finalize_mc<dev::FIN_BETA, K>), dim3(K), dim3(dev::kBlock), 0, st,
                     C.kpartial, kFlatGrid, C.ksc);
  if (C.vc32)
    hipLaunchKernelGGL((dev::k_update_p_mc<float, K, DP>), dim3(kFlatGrid), dim3(dev::kBlock), 0, st,
                       n, C.ksc, static_cast<const float*>(C.kx[0]), C.kP);
  else
    hipLaunchKernelGGL((dev::k_update_p_mc<double, K, DP>), dim3(kFlatGrid), dim3(dev::kBlock), 0,
                       st, n, C.ksc, static_cast<const double*>(C.kx[0]), C.kP);
}

// Columns c0 .. c0+nc-1 (nc <= K) of the user arrays [n_rhs][nv][D]; the
// unused columns of the block are zero and stop at once.
template <int D, int K>
void ensure_block_graphs(vasmg_ctx& C) {
  if (!C.kgA) C.kgA = capture(C, &enqueue_iter_A_mc<D, K>);
  if (!C.kgB) C.kgB = capture(C, &enqueue_iter_B_mc<D, K>);
}

template <int D, int K>
int solve_block(vasmg_ctx& C, const double* d_rhs, const double* d_x0, double* d_x, int c0, int nc,
                double rtol, hipStream_t st, vasmg_solve_info* info) {
  constexpr int DP = dev::Pad<D>::value;
  ensure_block_graphs<D, K>(C);
  const int n0 = C.n0;
  const int64_t n = C.n0p * K;
  const int64_t nv = C.H.n_mesh_vertices;
  const int gflat = kFlatGrid;
  const dim3 gk(grid_for(static_cast<int64_t>(n0) * K, dev::kBlock));
  HIP_CHECK(hipEventRecord(C.ev[0], st));
  hipLaunchKernelGGL((dev::k_gather_user_mc<D, K>), gk, dim3(dev::kBlock), 0, st, n0, C.user_map,
                     d_rhs, nv, c0, nc, C.kF, static_cast<const uint8_t*>(C.lev[0].fixed));
  hipLaunchKernelGGL((dev::k_dot_mc<K, DP, double>), dim3(gflat), dim3(dev::kBlock), 0, st, n, C.kF,
                     C.kF, C.kpartial);
  hipLaunchKernelGGL((dev::k_finalize_mc<dev::FIN_NORMF, K>), dim3(K), dim3(dev::kBlock), 0, st,
                     C.kpartial, gflat, C.ksc);
  if (d_x0) {
    hipLaunchKernelGGL((dev::k_gather_user_mc<D, K>), gk, dim3(dev::kBlock), 0, st, n0, C.user_map,
                       d_x0, nv, c0, nc, C.kX, static_cast<const uint8_t*>(C.lev[0].fixed));
    hipLaunchKernelGGL((dev::k_zero_cols_mc<K, DP>), dim3(gflat), dim3(dev::kBlock), 0, st, n, C.ksc,
                       C.kX);
    launch_spmv_mc<D, K>(C, C.kX, C.kQ, nullptr, st);
    hipLaunchKernelGGL((dev::k_sub_norm_mc<K, DP>), dim3(gflat), dim3(dev::kBlock), 0, st, n, C.kF,
                       C.kQ, C.kR, C.kpartial);
    hipLaunchKernelGGL((dev::k_finalize_mc<dev::FIN_TRUE, K>), dim3(K), dim3(dev::kBlock), 0, st,
                       C.kpartial, gflat, C.ksc);
  } else {
    launch_fill<double>(C.kX, n, 0.0, st);
    hipLaunchKernelGGL((dev::k_convert<double, double>), dim3(gflat), dim3(dev::kBlock), 0, st, n,
                       C.kF, C.kR);
  }
  hipLaunchKernelGGL((dev::k_start_mc<K>), dim3(1), dim3(64), 0, st, C.ksc, rtol, d_x0 ? 1 : 0);
  launch_fill<double>(C.kP, n, 0.0, st);
  if (C.vc32)
    hipLaunchKernelGGL((dev::k_convert<double, float>), dim3(gflat), dim3(dev::kBlock), 0, st, n,
                       C.kR, static_cast<float*>(C.kb[0]));
  HIP_CHECK(hipGetLastError());
  HIP_CHECK(hipMemcpyAsync(C.kh_sc, C.ksc, sizeof(Scalars) * K, hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  std::vector<double> normF(K);
  bool all_done = true;
  for (int k = 0; k < K; ++k) {
    normF[k] = C.kh_sc[k].normF;
    all_done = all_done && C.kh_sc[k].done;
  }
  if (!all_done) {
    HIP_CHECK(hipGraphLaunch(C.kgB, st));
    for (int it = 0; it < C.opt.max_iters; ++it) {
      HIP_CHECK(hipGraphLaunch(C.kgA, st));
      HIP_CHECK(hipMemcpyAsync(C.kh_sc, C.ksc, sizeof(Scalars) * K, hipMemcpyDeviceToHost, st));
      HIP_CHECK(hipStreamSynchronize(st));
      all_done = true;
      for (int k = 0; k < K; ++k) all_done = all_done && C.kh_sc[k].done;
      if (all_done) break;
      HIP_CHECK(hipGraphLaunch(C.kgB, st));
    }
  }
  // true residuals, scatter
  launch_spmv_mc<D, K>(C, C.kX, C.kQ, nullptr, st);
  hipLaunchKernelGGL((dev::k_sub_norm_mc<K, DP>), dim3(gflat), dim3(dev::kBlock), 0, st, n, C.kF,
                     C.kQ, static_cast<double*>(nullptr), C.kpartial);
  hipLaunchKernelGGL((dev::k_finalize_mc<dev::FIN_TRUE, K>), dim3(K), dim3(dev::kBlock), 0, st,
                     C.kpartial, gflat, C.ksc);
  launch_fill<double>(d_x + static_cast<int64_t>(c0) * nv * D, static_cast<int64_t>(nc) * nv * D, 0.0,
                      st);                                       // fixed DOFs
  hipLaunchKernelGGL((dev::k_scatter_user_mc<D, K>), gk, dim3(dev::kBlock), 0, st, n0, C.user_map,
                     C.kX, nv, c0, nc, d_x);
  HIP_CHECK(hipMemcpyAsync(C.kh_sc, C.ksc, sizeof(Scalars) * K, hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipEventRecord(C.ev[1], st));
  HIP_CHECK(hipStreamSynchronize(st));
  HIP_CHECK(hipGetLastError());
  float ms = 0.f;
  HIP_CHECK(hipEventElapsedTime(&ms, C.ev[0], C.ev[1]));
  int worst = VASMG_OK;
  for (int k = 0; k < nc; ++k) {
    const Scalars& sk = C.kh_sc[k];
    int status = VASMG_OK;
    if (!std::isfinite(normF[k]) || sk.status == 5)
      status = VASMG_EBREAKDOWN;
    else if (normF[k] != 0.0 && !(sk.res / normF[k] < rtol) && !(d_x0 && sk.iters == 0))
      status = VASMG_ENOTCONV;
    if (status != VASMG_OK && worst == VASMG_OK) worst = status;
    if (info) {
      vasmg_solve_info& f = info[k];
      f.iterations = sk.iters;
      f.converged = status == VASMG_OK ? 1 : 0;
      f.rel_res = normF[k] > 0 ? sk.res / normF[k] : 0.0;
      f.rel_res_true = normF[k] > 0 ? sk.res_true / normF[k] : 0.0;
      f.t_solve_ms = ms;
      f.t_spmv_ms = f.t_precond_ms = f.t_vector_ms = f.bytes_model = 0.0;
      f.status = status;
      f.reserved = 0;
    }
  }
  return worst;
}

bool device_available();

// Device upload of a host-built hierarchy (+ block vectors, autotuning).
// alloc_stream != NULL: allocations are stream-ordered on it.
// Block right-hand sides: lanes per block row of each level (narrow or wide
// groups) by timing the level's own block kernels (forward zero-guess sweep,
// residual, backward sweep; on the fine level also the block SpMV, which shares
// the setting); the fastest median of three wins.
template <typename T, int D, int K>
double time_level_mc(vasmg_ctx& C, int l, hipStream_t st) {
  DevLevel& lv = C.lev[l];
  T* b = static_cast<T*>(C.kb[l]);
  T* x = static_cast<T*>(C.kx[l]);
  T* s = static_cast<T*>(C.ks[l]);
  T* r = static_cast<T*>(C.kr[l]);
  hipEvent_t e0, e1;
  HIP_CHECK(hipEventCreate(&e0));
  HIP_CHECK(hipEventCreate(&e1));
  std::vector<float> t;
  for (int rep = 0; rep < 4; ++rep) {
    HIP_CHECK(hipEventRecord(e0, st));
    launch_gs_sweep_mc<T, D, K>(lv, false, true, b, x, s, st);
    launch_residual_mc<T, D, K>(lv, s, x, r, st);
    launch_gs_sweep_mc<T, D, K>(lv, true, false, b, x, s, st);
    if (l == 0) launch_spmv_mc<D, K>(C, C.kP, C.kQ, nullptr, st);
    HIP_CHECK(hipEventRecord(e1, st));
    HIP_CHECK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
    if (rep > 0) t.push_back(ms);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  std::sort(t.begin(), t.end());
  return t[t.size() / 2];
}

template <int D, int K>
void autotune_block(vasmg_ctx& C) {
  hipStream_t st = C.cap_stream;
  for (int l = 0; l < C.L; ++l) {
    DevLevel& lv = C.lev[l];
    const bool fine64 = l == 0 && !C.vc32;
    int best_gl = lv.mcGL;
    double best = 1e30;
    const int opts[2] = {lv.cells ? dev::kCellLanesNarrow : dev::kPointLanesNarrow,
                         lv.cells ? dev::kCellLanesWide : dev::kPointLanesWide};
    for (int gl : opts) {
      lv.mcGL = gl;
      const double ms = (C.vc32 && !fine64) ? time_level_mc<float, D, K>(C, l, st)
                                            : time_level_mc<double, D, K>(C, l, st);
      if (ms < best) {
        best = ms;
        best_gl = gl;
      }
    }
    lv.mcGL = best_gl;
    if (C.opt.verbose)
      std::fprintf(stderr, "[vasmg] autotune block level %d: %d lanes per row (%.3f ms)\n", l, best_gl,
                   best);
  }
  HIP_CHECK(hipStreamSynchronize(st));
}

void upload_device(vasmg_ctx& C, hipStream_t alloc_stream) {
  if (!device_available()) throw vasmg::Error{VASMG_EDEVICE, "no HIP device available"};
  HIP_CHECK(hipGetDevice(&C.device));
  C.alloc_stream = alloc_stream;
  using Clock = std::chrono::steady_clock;
  auto ms_since = [](Clock::time_point t) {
    return std::chrono::duration<double, std::milli>(Clock::now() - t).count();
  };
  auto t = Clock::now();
  upload_all(C);
  if (C.opt.block_rhs != 0) upload_block(C, C.opt.block_rhs);
  C.upload_ms[0] = ms_since(t);
  t = Clock::now();
  if (C.opt.autotune) {
    if (C.d == 2)
      autotune<2>(C);
    else
      autotune<3>(C);
    if (C.K > 0 && C.opt.block_lanes == 0) {
      if (C.d == 2) {
        DISPATCH_K(C.K, { autotune_block<2, KK>(C); });
      } else {
        DISPATCH_K(C.K, { autotune_block<3, KK>(C); });
      }
    }
  }
  C.upload_ms[1] = ms_since(t);
  t = Clock::now();
  // The PCG graphs are captured here, after the lanes per row are final, and not
  // at the first solve: a solve then instantiates and allocates nothing.
  auto graphs = [&](auto dtag) {
    constexpr int D = decltype(dtag)::value;
    if (C.nseg > 0) {
      ensure_packed_graphs<D>(C);
      return;
    }
    ensure_graphs<D>(C);
    if (C.K > 0) DISPATCH_K(C.K, { ensure_block_graphs<D, KK>(C); });
  };
  if (C.d == 2)
    graphs(std::integral_constant<int, 2>());
  else
    graphs(std::integral_constant<int, 3>());
  C.upload_ms[2] = ms_since(t);
  C.host_only = false;
}

// Upper bound of the device bytes upload_device will allocate, from the host
// hierarchy (every stored block counted as off-diagonal, the transient copy of
// the largest level's canonical operator included, 5% + 1 MiB margin).
int64_t estimate_device_bytes(const vasmg_ctx& C) {
  const Hierarchy& H = C.H;
  const int d = C.d, dd = d * d, DP = C.DP, NU = (1 << d) * d;
  const bool vasmg = C.opt.preconditioner == VASMG_PRECOND_VASMG;
  const int L = static_cast<int>(H.levels.size()) - 1;
  const int last = vasmg ? L : 0;
  const int64_t tbv = C.vc32 ? 4 : 8;
  const int64_t K = C.opt.block_rhs;
  int64_t b = 0;
  for (int l = 0; l <= last; ++l) {
    const Level& lv = H.levels[l];
    const int64_t n = lv.n, nb = lv.A.nnzb();
    const bool need64 = l == 0 || !C.vc32, need32 = C.vc32 && vasmg;
    const int64_t vb = (need64 ? 8 : 0) + (need32 ? 4 : 0);
    b += n * 4 + 2 * (n + 1) * 4 + nb * (4 + dd * vb);
    if (l > 0 && l < L)
      b += lv.ncells * (NU * NU * vb + 4) + 4 * (lv.ncolors + 2);
    else
      b += n * dd * vb;
    if (l < L) {
      const int64_t pn = static_cast<int64_t>(lv.P.col.size());
      b += (n + 1) * 4 + (H.levels[l + 1].n + 1) * 4 + 2 * pn * (4 + vb);
    }
    b += 4 * n * DP * tbv * (1 + K);
  }
  // the largest level's canonical operator, copied in for its layout only, and the
  // layout's per-row arrays
  int64_t transient = 0;
  for (int l = 0; l <= last; ++l) {
    const Level& lv = H.levels[l];
    transient = std::max(transient, lv.A.nnzb() * (4 + dd * 8) + (lv.n + 1) * 8 + 6 * lv.n * 4);
  }
  b += transient;
  const int64_t n0p = H.levels[0].n * DP;
  b += 6 * n0p * 8 + H.levels[0].n * 4 + H.n_coarse_dofs * H.n_coarse_dofs * 16;   // factor + inverse
  b += (std::max<int64_t>(kFlatGrid, H.levels[0].n / 4 + 1)) * 8 * (1 + K);
  b += 5 * n0p * 8 * K;
  if (C.nseg > 0) b += H.levels[0].n * 12 + static_cast<int64_t>(C.nseg + 1) * (4 + sizeof(Scalars));
  return b + b / 20 + (1 << 20);
}

vasmg_status fail_with(const vasmg::Error& e) {
  g_last_error = e.msg;
  return static_cast<vasmg_status>(e.status);
}

bool device_available() {
  int n = 0;
  return hipGetDeviceCount(&n) == hipSuccess && n > 0;
}

}  // namespace

// ---------------------------------------------------------------------------
// Staging of the no-allocation host-pointer solve (vasmg_solve_noalloc): one
// fixed array of this library per GPU, in place of the device buffers
// vasmg_solve allocates per call. In host code `scratch` names a host-side
// stand-in, not device memory: its device address on each GPU comes from
// hipGetSymbolAddress (with that GPU current) and only that address is used.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = static_cast<size_t>(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;                   // guards g_scratch_ptr
void* g_scratch_ptr[kMaxDevices] = {};        // device address of `scratch` per GPU
std::mutex g_scratch_use[kMaxDevices];        // one no-allocation solve per GPU at a time

// Device address of this GPU's copy of `scratch`; dev must be the current device.
unsigned char* scratch_address(int dev) {
  if (dev < 0 || dev >= kMaxDevices)
    throw vasmg::Error{VASMG_EDEVICE, "device index beyond the no-allocation table"};
  std::lock_guard<std::mutex> g(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw vasmg::Error{VASMG_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                            hipGetErrorString(e)};
    g_scratch_ptr[dev] = p;
  }
  return static_cast<unsigned char*>(g_scratch_ptr[dev]);
}

// masked: the level's constrained components read as 0 (the restriction's
// zero prolongation rows)
template <typename T, int D>
void debug_gather(vasmg_ctx& C, int l, const double* src, T* dst, hipStream_t st,
                  bool masked = false) {
  const int n = static_cast<int>(C.H.levels[l].n);
  hipLaunchKernelGGL((dev::k_gather_user<double, T, D>), dim3(grid_for(n, dev::kBlock)),
                     dim3(dev::kBlock), 0, st, n, C.lev[l].perm, src, dst,
                     masked ? static_cast<const uint8_t*>(C.lev[l].fixed) : nullptr);
}
template <typename T, int D>
void debug_scatter(vasmg_ctx& C, int l, const T* src, double* dst, hipStream_t st) {
  const int n = static_cast<int>(C.H.levels[l].n);
  hipLaunchKernelGGL((dev::k_scatter_user<T, double, D>), dim3(grid_for(n, dev::kBlock)),
                     dim3(dev::kBlock), 0, st, n, C.lev[l].perm, src, dst);
}

void check_handle(vasmg_handle h) {
  if (!h) throw vasmg::Error{VASMG_EINVAL, "null handle"};
  if (h->host_only) throw vasmg::Error{VASMG_EDEVICE, "handle was set up host-only"};
  HIP_CHECK(hipSetDevice(h->device));
}

void check_level(vasmg_handle h, int level, bool need_transfer) {
  if (level < 0 || level > h->L) throw vasmg::Error{VASMG_EINVAL, "level out of range"};
  if (need_transfer && level >= h->L) throw vasmg::Error{VASMG_EINVAL, "no transfer on the coarsest level"};
  if (h->opt.preconditioner != VASMG_PRECOND_VASMG && level > 0)
    throw vasmg::Error{VASMG_EINVAL, "hierarchy not uploaded (non-V-ASMG preconditioner)"};
}

template <typename T>
void check_prec(vasmg_handle h, int level) {
  if (level == h->L && level > 0) throw vasmg::Error{VASMG_EINVAL, "coarsest level has no operator on the device"};
  if (!LevelMats<T>::ok(h->lev[level]))
    throw vasmg::Error{VASMG_EINVAL, "requested precision not resident for this level"};
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* vasmg_last_error(void) { return g_last_error.c_str(); }

vasmg_status vasmg_set_galerkin_window(int32_t cols) {
  if (cols < 0) {
    g_last_error = "vasmg_set_galerkin_window: cols must be >= 0";
    return VASMG_EINVAL;
  }
  g_galerkin_window.store(cols);
  return VASMG_OK;
}

vasmg_status vasmg_default_options(int32_t dim, vasmg_options* out) {
  if (!out || (dim != 2 && dim != 3)) {
    g_last_error = "vasmg_default_options: dim must be 2 or 3 and out non-null";
    return VASMG_EINVAL;
  }
  std::memset(out, 0, sizeof(*out));
  out->leaf_capacity = dim == 2 ? 4 : 8;
  out->n_pre = 1;
  out->n_post = 1;
  out->precision = VASMG_FP64;
  out->tree_vertices = VASMG_TREE_ALL;
  out->coarsest_max_dofs = 0;
  out->max_iters = 10000;
  out->preconditioner = VASMG_PRECOND_VASMG;
  return VASMG_OK;
}

vasmg_status vasmg_setup(const vasmg_mesh* mesh, const vasmg_options* opt, vasmg_handle* out) {
  if (out) *out = nullptr;
  try {
    if (!mesh || !out) throw vasmg::Error{VASMG_EINVAL, "null mesh or output pointer"};
    std::unique_ptr<vasmg_ctx> C(new vasmg_ctx());
    if (opt) {
      C->opt = *opt;
    } else if (vasmg_default_options(mesh->dim, &C->opt) != VASMG_OK) {
      throw vasmg::Error{VASMG_EINVAL, "dim must be 2 or 3"};
    }
    vasmg_options& o = C->opt;
    if (o.leaf_capacity == 0) o.leaf_capacity = mesh->dim == 2 ? 4 : 8;
    if (o.leaf_capacity < 1) throw vasmg::Error{VASMG_EINVAL, "leaf_capacity must be >= 1"};
    if (o.n_pre < 0 || o.n_post < 0 || o.n_pre > 16 || o.n_post > 16)
      throw vasmg::Error{VASMG_EINVAL, "n_pre/n_post must be in [0, 16]"};
    if (o.precision != VASMG_FP64 && o.precision != VASMG_FP32_PRECOND)
      throw vasmg::Error{VASMG_EINVAL, "unknown precision"};
    if (o.tree_vertices != VASMG_TREE_ALL && o.tree_vertices != VASMG_TREE_FREE)
      throw vasmg::Error{VASMG_EINVAL, "unknown tree_vertices"};
    if (o.preconditioner < 0 || o.preconditioner > 2)
      throw vasmg::Error{VASMG_EINVAL, "unknown preconditioner"};
    if (o.max_iters <= 0) o.max_iters = 10000;
    if (o.coarsest_max_dofs < 0) throw vasmg::Error{VASMG_EINVAL, "coarsest_max_dofs < 0"};
    if (o.block_rhs != 0 && o.block_rhs != 4 && o.block_rhs != 8 && o.block_rhs != 16)
      throw vasmg::Error{VASMG_EINVAL, "block_rhs must be 0, 4, 8 or 16"};
    if (o.cycle < VASMG_CYCLE_V || o.cycle > VASMG_CYCLE_ADDITIVE)
      throw vasmg::Error{VASMG_EINVAL, "unknown cycle"};
    if (o.smoother != VASMG_SMOOTHER_GS && o.smoother != VASMG_SMOOTHER_JACOBI)
      throw vasmg::Error{VASMG_EINVAL, "unknown smoother"};
    if (o.block_rhs != 0 && (o.cycle != VASMG_CYCLE_V || o.smoother != VASMG_SMOOTHER_GS))
      throw vasmg::Error{VASMG_EINVAL, "block_rhs supports the Gauss-Seidel V-cycle only"};
    if (o.setup_device != 0 && o.setup_device != 1)
      throw vasmg::Error{VASMG_EINVAL, "setup_device must be 0 or 1"};
    MeshView mv{mesh->dim, mesh->n_vertices, mesh->coords, mesh->n_elements, mesh->elems,
                mesh->E, mesh->nu, mesh->fixed};
    if (o.color_blocks != 0 && o.color_blocks != 1)
      throw vasmg::Error{VASMG_EINVAL, "color_blocks must be 0 (off) or 1 (on)"};
    if (o.block_lanes < 0 || o.block_lanes > 2)
      throw vasmg::Error{VASMG_EINVAL, "block_lanes must be 0, 1 (narrow) or 2 (wide)"};
    SetupParams prm{o.leaf_capacity, o.tree_vertices == VASMG_TREE_FREE, o.coarsest_max_dofs};
    // the block right-hand-side kernels sweep one cell per workgroup: no colour blocks
    prm.color_blocks = o.color_blocks == 1 && o.block_rhs == 0;
    std::unique_ptr<GalerkinDevice, void (*)(GalerkinDevice*)> gdev(nullptr, galerkin_device_destroy);
    if (o.setup_device == 1) {
      if (!device_available()) throw vasmg::Error{VASMG_EDEVICE, "no HIP device for setup_device = 1"};
      gdev.reset(galerkin_device_create(g_galerkin_window.load()));
      prm.galerkin = galerkin_device;
      prm.assemble = assemble_device;
      prm.settle = galerkin_device_settle;
      prm.wait_structure = galerkin_device_wait_structure;
      prm.transfers = transfers_device;
      prm.galerkin_ctx = gdev.get();
    }
    build_hierarchy(mv, prm, C->H);
    if (gdev && o.host_only) {   // every value back on the host, no device memory kept
      galerkin_device_join(gdev.get());
      gdev.reset();
    }
    C->d = mesh->dim;
    C->DP = mesh->dim == 3 ? 4 : 2;
    C->L = static_cast<int>(C->H.levels.size()) - 1;
    C->vc32 = o.precision == VASMG_FP32_PRECOND;
    C->host_only = o.host_only != 0;
    if (o.verbose) {
      for (size_t l = 0; l < C->H.levels.size(); ++l) {
        const Level& lv = C->H.levels[l];
        std::fprintf(stderr, "[vasmg] level %zu: %lld vertices, %lld blocks, %d colours\n", l,
                     static_cast<long long>(lv.n), static_cast<long long>(lv.A.nnzb()), lv.ncolors);
      }
      for (const auto& ph : C->H.phase_ms)
        std::fprintf(stderr, "[vasmg] setup %-18s %9.1f ms\n", ph.first.c_str(), ph.second);
    }
    if (!C->host_only) {
      const auto t0 = std::chrono::steady_clock::now();
      C->gdev = gdev.get();
      upload_device(*C, nullptr);
      C->gdev = nullptr;
      if (gdev && o.smoother == VASMG_SMOOTHER_JACOBI) {
        galerkin_device_join(gdev.get());   // already started by the Jacobi set-up
        gdev.reset();
      } else if (gdev) {
        // the host copies of the level values arrive while the caller goes on;
        // each level's device copy is released once its values are home
        galerkin_device_start_downloads(gdev.get(), true);
        C->gdev_bg = gdev.release();
      }
      const double ms =
          std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      // the upload's parts (host time until each returned; device work may run on)
      const double other = ms - C->upload_ms[0] - C->upload_ms[1] - C->upload_ms[2];
      C->H.phase_ms.emplace_back("upload: layouts", C->upload_ms[0] + std::max(other, 0.0));
      if (o.autotune) C->H.phase_ms.emplace_back("upload: autotune", C->upload_ms[1]);
      C->H.phase_ms.emplace_back("upload: graphs", C->upload_ms[2]);
      if (o.verbose)
        std::fprintf(stderr, "[vasmg] setup %-18s %9.1f ms (layouts %.1f, autotune %.1f, graphs %.1f)\n",
                     "upload", ms, C->upload_ms[0], C->upload_ms[1], C->upload_ms[2]);
    }
    *out = C.release();
    return VASMG_OK;
  } catch (const vasmg::Error& e) {
    return fail_with(e);
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return VASMG_ENOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return VASMG_EINVAL;
  }
}

void vasmg_free(vasmg_handle h) {
  if (!h) return;
  if (!h->host_only) (void)hipSetDevice(h->device);
  delete h;
}

vasmg_status vasmg_solve_device(vasmg_handle h, const double* d_rhs, const double* d_x0,
                                double* d_x, int32_t n_rhs, double rtol, void* stream,
                                vasmg_solve_info* info) {
  try {
    check_handle(h);
    if (!d_rhs || !d_x || n_rhs < 1) throw vasmg::Error{VASMG_EINVAL, "bad rhs/x/n_rhs"};
    if (!(rtol > 0.0)) throw vasmg::Error{VASMG_EINVAL, "rtol must be > 0"};
    if (h->nseg > 0) throw vasmg::Error{VASMG_EINVAL, "packed handle: use vasmg_solve_packed(_device)"};
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t stride = h->H.n_mesh_vertices * h->d;
    int worst = VASMG_OK;
    if (h->K > 0 && n_rhs > 1) {
      // block solve: K columns at a time share every matrix read
      for (int c0 = 0; c0 < n_rhs; c0 += h->K) {
        const int nc = std::min(h->K, n_rhs - c0);
        vasmg_solve_info* fi = info ? info + c0 : nullptr;
        int s = VASMG_OK;
        DISPATCH_K(h->K, {
          s = h->d == 2 ? solve_block<2, KK>(*h, d_rhs, d_x0, d_x, c0, nc, rtol, st, fi)
                        : solve_block<3, KK>(*h, d_rhs, d_x0, d_x, c0, nc, rtol, st, fi);
        });
        if (s != VASMG_OK && worst == VASMG_OK) worst = s;
      }
    } else {
      for (int c = 0; c < n_rhs; ++c) {
        const int s = h->d == 2 ? solve_one<2>(*h, d_rhs + c * stride, d_x0 ? d_x0 + c * stride : nullptr,
                                                d_x + c * stride, rtol, st, info ? info + c : nullptr)
                                : solve_one<3>(*h, d_rhs + c * stride, d_x0 ? d_x0 + c * stride : nullptr,
                                                d_x + c * stride, rtol, st, info ? info + c : nullptr);
        if (s != VASMG_OK && worst == VASMG_OK) worst = s;
      }
    }
    if (worst == VASMG_ENOTCONV) g_last_error = "PCG did not reach rtol within max_iters";
    if (worst == VASMG_EBREAKDOWN) g_last_error = "PCG breakdown (p^T A p <= 0 or not finite)";
    return static_cast<vasmg_status>(worst);
  } catch (const vasmg::Error& e) {
    return fail_with(e);
  }
}

vasmg_status vasmg_solve(vasmg_handle h, const double* rhs, const double* x0, double* x,
                         int32_t n_rhs, double rtol, vasmg_solve_info* info) {
  double *drhs = nullptr, *dx0 = nullptr, *dx = nullptr;
  try {
    check_handle(h);
    if (!rhs || !x || n_rhs < 1) throw vasmg::Error{VASMG_EINVAL, "bad rhs/x/n_rhs"};
    const size_t bytes = sizeof(double) * h->H.n_mesh_vertices * h->d * n_rhs;
    HIP_CHECK(hipMalloc(&drhs, bytes));
    HIP_CHECK(hipMalloc(&dx, bytes));
    HIP_CHECK(hipMemcpy(drhs, rhs, bytes, hipMemcpyHostToDevice));
    if (x0) {
      HIP_CHECK(hipMalloc(&dx0, bytes));
      HIP_CHECK(hipMemcpy(dx0, x0, bytes, hipMemcpyHostToDevice));
    }
    const vasmg_status s = vasmg_solve_device(h, drhs, dx0, dx, n_rhs, rtol, nullptr, info);
    const std::string msg = g_last_error;
    HIP_CHECK(hipMemcpy(x, dx, bytes, hipMemcpyDeviceToHost));
    (void)hipFree(drhs);
    (void)hipFree(dx);
    if (dx0) (void)hipFree(dx0);
    g_last_error = msg;
    return s;
  } catch (const vasmg::Error& e) {
    if (drhs) (void)hipFree(drhs);
    if (dx) (void)hipFree(dx);
    if (dx0) (void)hipFree(dx0);
    return fail_with(e);
  }
}

vasmg_status vasmg_solve_noalloc(vasmg_handle h, const double* rhs, const double* x0, double* x,
                                 int32_t n_rhs, double rtol, vasmg_solve_info* info) {
  try {
    check_handle(h);
    if (!rhs || !x || n_rhs < 1) throw vasmg::Error{VASMG_EINVAL, "bad rhs/x/n_rhs"};
    if (h->nseg > 0) throw vasmg::Error{VASMG_EINVAL, "packed handle: use vasmg_solve_packed(_device)"};
    const size_t vec = sizeof(double) * static_cast<size_t>(h->H.n_mesh_vertices) * h->d *
                       static_cast<size_t>(n_rhs);
    const size_t slot = (vec + 255) / 256 * 256;
    const size_t need = slot * (x0 ? 3 : 2);
    if (need > kScratchBytes)
      throw vasmg::Error{VASMG_EINVAL, "vasmg_solve_noalloc: " + std::to_string(need) +
                                           " bytes of staging needed, more than its fixed " +
                                           std::to_string(kScratchBytes) + "-byte array"};
    unsigned char* base = scratch_address(h->device);
    std::lock_guard<std::mutex> use(g_scratch_use[h->device]);
    double* drhs = reinterpret_cast<double*>(base);
    double* dx = reinterpret_cast<double*>(base + slot);
    double* dx0 = x0 ? reinterpret_cast<double*>(base + 2 * slot) : nullptr;
    HIP_CHECK(hipMemcpy(drhs, rhs, vec, hipMemcpyHostToDevice));
    if (x0) HIP_CHECK(hipMemcpy(dx0, x0, vec, hipMemcpyHostToDevice));
    const vasmg_status s = vasmg_solve_device(h, drhs, dx0, dx, n_rhs, rtol, nullptr, info);
    const std::string msg = g_last_error;
    HIP_CHECK(hipMemcpy(x, dx, vec, hipMemcpyDeviceToHost));
    g_last_error = msg;
    return s;
  } catch (const vasmg::Error& e) {
    return fail_with(e);
  }
}

vasmg_status vasmg_pack(const vasmg_handle* parts, int32_t n_parts, vasmg_handle* out) {
  try {
    if (!out) throw vasmg::Error{VASMG_EINVAL, "null output"};
    *out = nullptr;
    if (!parts || n_parts < 1) throw vasmg::Error{VASMG_EINVAL, "no parts to pack"};
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<const Hierarchy*> hs;
    const vasmg_options& o0 = parts[0] ? parts[0]->opt : vasmg_options{};
    int32_t max_iters = 0;
    for (int i = 0; i < n_parts; ++i) {
      vasmg_handle p = parts[i];
      if (!p) throw vasmg::Error{VASMG_EINVAL, "null part handle"};
      if (p->nseg > 0) throw vasmg::Error{VASMG_EINVAL, "a part is itself packed"};
      const vasmg_options& o = p->opt;
      if (o.preconditioner != VASMG_PRECOND_VASMG || o.cycle != VASMG_CYCLE_V ||
          o.smoother != VASMG_SMOOTHER_GS || o.block_rhs != 0 || o.color_blocks != 0)
        throw vasmg::Error{VASMG_EINVAL,
                           "packing needs the V-ASMG Gauss-Seidel V-cycle without block_rhs or colour blocks"};
      if (o.precision != o0.precision || o.n_pre != o0.n_pre || o.n_post != o0.n_post ||
          p->d != parts[0]->d)
        throw vasmg::Error{VASMG_EINVAL, "packed parts differ in dimension, precision or sweeps"};
      p->settle_host_values();
      hs.push_back(&p->H);
      max_iters = std::max(max_iters, o.max_iters);
    }
    auto C = std::make_unique<vasmg_ctx>();
    pack_hierarchies(hs, C->H);
    C->opt = o0;
    C->opt.host_only = 1;
    C->opt.max_iters = max_iters;
    C->d = parts[0]->d;
    C->DP = C->d == 3 ? 4 : 2;
    C->L = static_cast<int>(C->H.levels.size()) - 1;
    C->vc32 = o0.precision == VASMG_FP32_PRECOND;
    C->host_only = true;
    C->nseg = n_parts;
    C->seg_vertex_off.assign(1, 0);
    C->seg_free_off.assign(1, 0);
    for (int i = 0; i < n_parts; ++i) {
      C->seg_vertex_off.push_back(C->seg_vertex_off.back() + parts[i]->H.n_mesh_vertices);
      C->seg_free_off.push_back(C->seg_free_off.back() + parts[i]->H.levels[0].n);
    }
    C->H.phase_ms.emplace_back(
        "pack", std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
    *out = C.release();
    return VASMG_OK;
  } catch (const vasmg::Error& e) {
    return fail_with(e);
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return VASMG_ENOMEM;
  }
}

vasmg_status vasmg_packed_info(vasmg_handle h, int32_t* n_parts, int64_t* vertex_offsets) {
  if (!h) {
    g_last_error = "null handle";
    return VASMG_EINVAL;
  }
  if (n_parts) *n_parts = h->nseg;
  if (vertex_offsets && h->nseg > 0)
    std::copy(h->seg_vertex_off.begin(), h->seg_vertex_off.end(), vertex_offsets);
  return VASMG_OK;
}

vasmg_status vasmg_solve_packed_device(vasmg_handle h, const double* d_rhs, double* d_x, double rtol,
                                       void* stream, vasmg_solve_info* info) {
  try {
    check_handle(h);
    if (h->nseg == 0) throw vasmg::Error{VASMG_EINVAL, "not a packed handle (vasmg_pack)"};
    if (!d_rhs || !d_x || !info) throw vasmg::Error{VASMG_EINVAL, "bad rhs/x/info"};
    if (!(rtol > 0.0)) throw vasmg::Error{VASMG_EINVAL, "rtol must be > 0"};
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int worst = h->d == 2 ? solve_packed<2>(*h, d_rhs, d_x, rtol, st, info)
                                : solve_packed<3>(*h, d_rhs, d_x, rtol, st, info);
    if (worst == VASMG_ENOTCONV) g_last_error = "PCG did not reach rtol within max_iters (some part)";
    if (worst == VASMG_EBREAKDOWN) g_last_error = "PCG breakdown in some part";
    return static_cast<vasmg_status>(worst);
  } catch (const vasmg::Error& e) {
    return fail_with(e);
  }
}

vasmg_status vasmg_solve_packed(vasmg_handle h, const double* rhs, double* x, double rtol,
                                vasmg_solve_info* info) {
  double *drhs = nullptr, *dx = nullptr;
  try {
    check_handle(h);
    if (h->nseg == 0) throw vasmg::Error{VASMG_EINVAL, "not a packed handle (vasmg_pack)"};
    if (!rhs || !x || !info) throw vasmg::Error{VASMG_EINVAL, "bad rhs/x/info"};
    const size_t bytes = sizeof(double) * h->H.n_mesh_vertices * h->d;
    HIP_CHECK(hipMalloc(&drhs, bytes));
    HIP_CHECK(hipMalloc(&dx, bytes));
    HIP_CHECK(hipMemcpy(drhs, rhs, bytes, hipMemcpyHostToDevice));
    const vasmg_status s = vasmg_solve_packed_device(h, drhs, dx, rtol, nullptr, info);
    const std::string msg = g_last_error;
    HIP_CHECK(hipMemcpy(x, dx, bytes, hipMemcpyDeviceToHost));
    (void)hipFree(drhs);
    (void)hipFree(dx);
    g_last_error = msg;
    return s;
  } catch (const vasmg::Error& e) {
    if (drhs) (void)hipFree(drhs);
    if (dx) (void)hipFree(dx);
    return fail_with(e);
  }
}

vasmg_status vasmg_upload(vasmg_handle h, void* stream) {
  try {
    if (!h) throw vasmg::Error{VASMG_EINVAL, "null handle"};
    if (!h->host_only || !h->allocs.empty())
      throw vasmg::Error{VASMG_EINVAL, "handle is already on the device"};
    upload_device(*h, static_cast<hipStream_t>(stream));
    return VASMG_OK;
  } catch (const vasmg::Error& e) {
    return fail_with(e);
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return VASMG_ENOMEM;
  }
}

vasmg_status vasmg_device_bytes(vasmg_handle h, int64_t* bytes) {
  if (!h || !bytes) {
    g_last_error = "null handle or output";
    return VASMG_EINVAL;
  }
  *bytes = h->host_only ? estimate_device_bytes(*h) : h->dev_bytes;
  return VASMG_OK;
}

vasmg_status vasmg_hierarchy_info(vasmg_handle h, int32_t* n_levels, int64_t* n_dofs, int32_t* dim) {
  if (!h) {
    g_last_error = "null handle";
    return VASMG_EINVAL;
  }
  if (n_levels) *n_levels = static_cast<int32_t>(h->H.levels.size());
  if (n_dofs) *n_dofs = h->H.levels[0].n * h->d;
  if (dim) *dim = h->d;
  return VASMG_OK;
}

vasmg_status vasmg_level_info(vasmg_handle h, int32_t level, int64_t* n_vertices, int64_t* n_blocks,
                              int32_t* n_colors, int64_t* p_nnz) {
  if (!h || level < 0 || level >= static_cast<int32_t>(h->H.levels.size())) {
    g_last_error = "null handle or level out of range";
    return VASMG_EINVAL;
  }
  const Level& lv = h->H.levels[level];
  if (n_vertices) *n_vertices = lv.n;
  if (n_blocks) *n_blocks = lv.A.nnzb();
  if (n_colors) *n_colors = lv.ncolors;
  if (p_nnz) *p_nnz = static_cast<int64_t>(lv.P.col.size());
  return VASMG_OK;
}

vasmg_status vasmg_export_level(vasmg_handle h, int32_t level, int64_t* keys, int32_t* cell,
                                int32_t* color, int64_t* rowptr, int32_t* cols, double* vals,
                                int64_t* p_rowptr, int32_t* p_cols, double* p_vals,
                                int32_t* block, uint8_t* fixed) {
  if (!h || level < 0 || level >= static_cast<int32_t>(h->H.levels.size())) {
    g_last_error = "null handle or level out of range";
    return VASMG_EINVAL;
  }
  try {
    h->settle_host_values();
  } catch (const vasmg::Error& e) {
    return fail_with(e);
  }
  const Level& lv = h->H.levels[level];
  const int d = h->d;
  if (keys) {
    for (int64_t i = 0; i < lv.n; ++i)
      for (int a = 0; a < d; ++a)
        keys[i * d + a] = lv.keys.empty() ? -1 : static_cast<int64_t>(lv.keys[i][a]);
  }
  if (color) {
    for (int64_t i = 0; i < lv.n; ++i) color[i] = lv.color.empty() ? 0 : lv.color[i];
  }
  if (cell) {
    for (int64_t i = 0; i < lv.n; ++i) cell[i] = lv.cell.empty() ? 0 : lv.cell[i];
  }
  if (block) {
    for (int64_t i = 0; i < lv.n; ++i) block[i] = lv.block.empty() ? 0 : lv.block[i];
  }
  if (rowptr) std::copy(lv.A.rowptr.begin(), lv.A.rowptr.end(), rowptr);
  if (cols) std::copy(lv.A.col.begin(), lv.A.col.end(), cols);
  if (vals) {
    std::copy(lv.A.val.begin(), lv.A.val.end(), vals);
    if (!lv.fixed.empty())   // identity rows of the constrained components
      for (int64_t i = 0; i < lv.n; ++i)
        for (int64_t p = lv.A.rowptr[i]; p < lv.A.rowptr[i + 1]; ++p)
          if (lv.A.col[p] == i)
            for (int a = 0; a < d; ++a)
              if ((lv.fixed[i] >> a) & 1) vals[p * d * d + a * d + a] = 1.0;
  }
  if (fixed) {
    for (int64_t i = 0; i < lv.n; ++i) fixed[i] = lv.fixed.empty() ? 0 : lv.fixed[i];
  }
  if (p_rowptr) {
    if (lv.P.rowptr.empty())
      std::fill(p_rowptr, p_rowptr + lv.n + 1, 0);
    else
      std::copy(lv.P.rowptr.begin(), lv.P.rowptr.end(), p_rowptr);
  }
  if (p_cols) std::copy(lv.P.col.begin(), lv.P.col.end(), p_cols);
  if (p_vals) std::copy(lv.P.val.begin(), lv.P.val.end(), p_vals);
  return VASMG_OK;
}

vasmg_status vasmg_tree_info(vasmg_handle h, double* m, double* M, int32_t* max_depth) {
  if (!h) {
    g_last_error = "null handle";
    return VASMG_EINVAL;
  }
  if (m) *m = h->H.box_m;
  if (M) *M = h->H.box_M;
  if (max_depth) *max_depth = h->H.max_depth;
  return VASMG_OK;
}

vasmg_status vasmg_setup_phases(vasmg_handle h, vasmg_setup_phase* out, int32_t max_out,
                                int32_t* n_out) {
  if (!h || max_out < 0 || (max_out > 0 && !out)) {
    g_last_error = "null handle or output";
    return VASMG_EINVAL;
  }
  const auto& ph = h->H.phase_ms;
  for (int32_t i = 0; i < max_out && i < static_cast<int32_t>(ph.size()); ++i) {
    std::memset(out[i].name, 0, sizeof(out[i].name));
    std::strncpy(out[i].name, ph[i].first.c_str(), sizeof(out[i].name) - 1);
    out[i].ms = ph[i].second;
  }
  if (n_out) *n_out = static_cast<int32_t>(ph.size());
  return VASMG_OK;
}

#define DEBUG_PRELUDE(NEED_TRANSFER)          \
  check_handle(h);                            \
  check_level(h, level, NEED_TRANSFER);       \
  hipStream_t st = static_cast<hipStream_t>(stream);

vasmg_status vasmg_spmv_device(vasmg_handle h, int32_t level, int32_t precision, const double* d_x,
                               double* d_y, void* stream) {
  try {
    DEBUG_PRELUDE(false);
    DevLevel& lv = h->lev[level];
    auto run = [&](auto tag, auto dtag) {
      using T = decltype(tag);
      constexpr int D = decltype(dtag)::value;
      check_prec<T>(h, level);
      T* xin = static_cast<T*>(lv.x);
      T* yout = static_cast<T*>(lv.r);
      if (precision == VASMG_FP64 && h->vc32) {  // FP64 copy on the fine level of a mixed handle
        xin = reinterpret_cast<T*>(h->Z);
        yout = reinterpret_cast<T*>(h->Q);
      }
      debug_gather<T, D>(*h, level, d_x, xin, st);
      if (lv.cells)
        launch_cell_apply<T, D, 2>(lv, nullptr, xin, yout, nullptr, st);
      else
        launch_spmv<T, D>(lv, xin, yout, nullptr, 0, nullptr, st);
      debug_scatter<T, D>(*h, level, yout, d_y, st);
    };
    if (precision == VASMG_FP64) {
      if (h->d == 2) run(double(), std::integral_constant<int, 2>());
      else run(double(), std::integral_constant<int, 3>());
    } else {
      if (h->d == 2) run(float(), std::integral_constant<int, 2>());
      else run(float(), std::integral_constant<int, 3>());
    }
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipStreamSynchronize(st));
    return VASMG_OK;
  } catch (const vasmg::Error& e) {
    return fail_with(e);
  }
}

vasmg_status vasmg_gs_sweep_device(vasmg_handle h, int32_t level, int32_t precision, int32_t backward,
                                   const double* d_b, double* d_x, void* stream) {
  try {
    DEBUG_PRELUDE(false);
    if (level == h->L) throw vasmg::Error{VASMG_EINVAL, "no smoother on the coarsest level"};
    DevLevel& lv = h->lev[level];
    if ((precision == VASMG_FP64) == h->vc32)
      throw vasmg::Error{VASMG_EINVAL, "GS precision must match the handle's V-cycle precision"};
    auto run = [&](auto tag, auto dtag) {
      using T = decltype(tag);
      constexpr int D = decltype(dtag)::value;
      check_prec<T>(h, level);
      T* b = static_cast<T*>(lv.b);
      T* x = static_cast<T*>(lv.x);
      debug_gather<T, D>(*h, level, d_b, b, st);
      debug_gather<T, D>(*h, level, d_x, x, st);
      launch_gs_sweep<T, D>(lv, backward != 0, false, b, x, static_cast<T*>(lv.s), nullptr, st);
      debug_scatter<T, D>(*h, level, x, d_x, st);
    };
    if (precision == VASMG_FP64) {
      if (h->d == 2) run(double(), std::integral_constant<int, 2>());
      else run(double(), std::integral_constant<int, 3>());
    } else {
      if (h->d == 2) run(float(), std::integral_constant<int, 2>());
      else run(float(), std::integral_constant<int, 3>());
    }
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipStreamSynchronize(st));
    return VASMG_OK;
  } catch (const vasmg::Error& e) {
    return fail_with(e);
  }
}

vasmg_status vasmg_restrict_device(vasmg_handle h, int32_t level, int32_t precision, const double* d_r,
                                   double* d_bc, void* stream) {
  try {
    DEBUG_PRELUDE(true);
    DevLevel& lv = h->lev[level];
    DevLevel& nx = h->lev[level + 1];
    if ((precision == VASMG_FP64) == h->vc32)
      throw vasmg::Error{VASMG_EINVAL, "transfer precision must match the handle's V-cycle precision"};
    auto run = [&](auto tag, auto dtag) {
      using T = decltype(tag);
      constexpr int D = decltype(dtag)::value;
      T* r = static_cast<T*>(lv.r);
      T* bc = static_cast<T*>(nx.b);
      debug_gather<T, D>(*h, level, d_r, r, st, true);
      launch_restrict<T, D>(lv, r, bc, nullptr, st);
      debug_scatter<T, D>(*h, level + 1, bc, d_bc, st);
    };
    if (precision == VASMG_FP64) {
      if (h->d == 2) run(double(), std::integral_constant<int, 2>());
      else run(double(), std::integral_constant<int, 3>());
    } else {
      if (h->d == 2) run(float(), std::integral_constant<int, 2>());
      else run(float(), std::integral_constant<int, 3>());
    }
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipStreamSynchronize(st));
    return VASMG_OK;
  } catch (const vasmg::Error& e) {
    return fail_with(e);
  }
}

vasmg_status vasmg_prolong_device(vasmg_handle h, int32_t level, int32_t precision, const double* d_e,
                                  double* d_x, void* stream) {
  try {
    DEBUG_PRELUDE(true);
    DevLevel& lv = h->lev[level];
    DevLevel& nx = h->lev[level + 1];
    if ((precision == VASMG_FP64) == h->vc32)
      throw vasmg::Error{VASMG_EINVAL, "transfer precision must match the handle's V-cycle precision"};
    auto run = [&](auto tag, auto dtag) {
      using T = decltype(tag);
      constexpr int D = decltype(dtag)::value;
      T* e = static_cast<T*>(nx.x);
      T* x = static_cast<T*>(lv.x);
      debug_gather<T, D>(*h, level + 1, d_e, e, st);
      debug_gather<T, D>(*h, level, d_x, x, st);
      launch_prolong<T, D>(lv, e, x, nullptr, st);
      debug_scatter<T, D>(*h, level, x, d_x, st);
    };
    if (precision == VASMG_FP64) {
      if (h->d == 2) run(double(), std::integral_constant<int, 2>());
      else run(double(), std::integral_constant<int, 3>());
    } else {
      if (h->d == 2) run(float(), std::integral_constant<int, 2>());
      else run(float(), std::integral_constant<int, 3>());
    }
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipStreamSynchronize(st));
    return VASMG_OK;
  } catch (const vasmg::Error& e) {
    return fail_with(e);
  }
}

vasmg_status vasmg_apply_precond_device(vasmg_handle h, const double* d_r, double* d_z, void* stream) {
  try {
    check_handle(h);
    if (h->opt.preconditioner != VASMG_PRECOND_VASMG)
      throw vasmg::Error{VASMG_EINVAL, "handle was not set up with the V-ASMG preconditioner"};
    hipStream_t st = static_cast<hipStream_t>(stream);
    auto run = [&](auto tag, auto dtag) {
      using T = decltype(tag);
      constexpr int D = decltype(dtag)::value;
      T* b = static_cast<T*>(h->lev[0].b);
      T* x = static_cast<T*>(h->lev[0].x);
      debug_gather<T, D>(*h, 0, d_r, b, st);
      if (h->L == 0 && h->cinv) {
        hipLaunchKernelGGL((dev::k_coarse_apply<T, D>), dim3(1), dim3(dev::kBlock), 0, st,
                           static_cast<int>(h->n_coarse), h->cinv, b, x, h->zero_flag);
      } else if (h->L == 0) {
        hipLaunchKernelGGL((dev::k_coarse_solve<T, D>), dim3(1), dim3(dev::kBlock), 0, st,
                           static_cast<int>(h->n_coarse), h->chol, b, x, h->zero_flag);
      } else {
        enqueue_vcycle<T, D>(*h, h->zero_flag, st);
      }
      debug_scatter<T, D>(*h, 0, x, d_z, st);
    };
    if (h->vc32) {
      if (h->d == 2) run(float(), std::integral_constant<int, 2>());
      else run(float(), std::integral_constant<int, 3>());
    } else {
      if (h->d == 2) run(double(), std::integral_constant<int, 2>());
      else run(double(), std::integral_constant<int, 3>());
    }
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipStreamSynchronize(st));
    return VASMG_OK;
  } catch (const vasmg::Error& e) {
    return fail_with(e);
  }
}

vasmg_status vasmg_profile_iteration(vasmg_handle h, int32_t reps, void* stream,
                                     vasmg_phase_stat* out, int32_t max_out, int32_t* n_out) {
  try {
    check_handle(h);
    if (reps < 1 || !out || max_out < 1) throw vasmg::Error{VASMG_EINVAL, "bad reps/out"};
    if (h->opt.preconditioner != VASMG_PRECOND_VASMG)
      throw vasmg::Error{VASMG_EINVAL, "handle was not set up with the V-ASMG preconditioner"};
    hipStream_t st = static_cast<hipStream_t>(stream);
    vasmg_ctx& C = *h;
    // defined inputs: p = 1, V-cycle right-hand side = 1, flags cleared
    launch_fill<double>(C.P, C.n0p, 1.0, st);
    if (C.vc32)
      launch_fill<float>(static_cast<float*>(C.lev[0].b), C.n0p, 1.0f, st);
    else
      launch_fill<double>(static_cast<double*>(C.lev[0].b), C.n0p, 1.0, st);
    const int zero = 0;
    HIP_CHECK(hipMemcpyAsync(&C.sc->done, &zero, sizeof(int), hipMemcpyHostToDevice, st));
    HIP_CHECK(hipStreamSynchronize(st));
    Profiler prof{st, {}, {}, {}};
    const DevLevel& l0 = C.lev[0];
    const double n0 = l0.n, dd = C.d * C.d;
    const int tb = C.vc32 ? 4 : 8;
    const double spmv_bytes = (l0.nnz_lo + l0.nnz_up) * (dd * 8 + 4.0) + (n0 + 1) * 4 +
                              n0 * dd * 8 + 2 * C.n0p * 8.0 + n0 * 4;
    const double vec_bytes = C.n0p * (6 * 8.0 + tb) + C.n0p * (8.0 + tb) + C.n0p * (16.0 + tb);
    for (int r = 0; r < reps; ++r) {
      auto body = [&](auto dtag) {
        constexpr int D = decltype(dtag)::value;
        run_phase(&prof, "spmv_f64", 0, 1, spmv_bytes, [&] {
          launch_spmv<double, D>(l0, C.P, C.Q, C.partial, C.n_partial, nullptr, st);
        });
        run_phase(&prof, "pcg_vectors", -1, 3, vec_bytes, [&] {
          if (C.vc32) {
            hipLaunchKernelGGL((dev::k_update_xr<float>), dim3(kFlatGrid), dim3(dev::kBlock), 0, st,
                               C.n0p, C.sc, C.P, C.Q, C.X, C.R, static_cast<float*>(C.lev[0].b),
                               C.partial);
            hipLaunchKernelGGL((dev::k_dot<float>), dim3(kFlatGrid), dim3(dev::kBlock), 0, st,
                               C.n0p, C.R, static_cast<const float*>(C.lev[0].x), C.partial,
                               nullptr);
            hipLaunchKernelGGL((dev::k_update_p<float>), dim3(kFlatGrid), dim3(dev::kBlock), 0, st,
                               C.n0p, C.sc, static_cast<const float*>(C.lev[0].x), C.P);
          } else {
            hipLaunchKernelGGL((dev::k_update_xr<double>), dim3(kFlatGrid), dim3(dev::kBlock), 0,
                               st, C.n0p, C.sc, C.P, C.Q, C.X, C.R, static_cast<double*>(nullptr),
                               C.partial);
            hipLaunchKernelGGL((dev::k_dot<double>), dim3(kFlatGrid), dim3(dev::kBlock), 0, st,
                               C.n0p, C.R, static_cast<const double*>(C.lev[0].x), C.partial,
                               nullptr);
            hipLaunchKernelGGL((dev::k_update_p<double>), dim3(kFlatGrid), dim3(dev::kBlock), 0,
                               st, C.n0p, C.sc, static_cast<const double*>(C.lev[0].x), C.P);
          }
        });
        if (C.vc32)
          enqueue_vcycle<float, D>(C, C.zero_flag, st, &prof);
        else
          enqueue_vcycle<double, D>(C, C.zero_flag, st, &prof);
      };
      if (C.d == 2)
        body(std::integral_constant<int, 2>());
      else
        body(std::integral_constant<int, 3>());
      HIP_CHECK(hipGetLastError());
      prof.finish();
    }
    const int n = static_cast<int>(std::min<size_t>(prof.stats.size(), max_out));
    for (int i = 0; i < n; ++i) {
      const PhaseStat& p = prof.stats[i];
      std::memset(&out[i], 0, sizeof(out[i]));
      std::snprintf(out[i].name, sizeof(out[i].name), "%s", p.name.c_str());
      out[i].level = p.level;
      out[i].launches = p.launches;
      out[i].ms = p.ms;
      out[i].bytes = p.bytes;
    }
    if (n_out) *n_out = n;
    return VASMG_OK;
  } catch (const vasmg::Error& e) {
    return fail_with(e);
  }
}

}  // extern "C"
