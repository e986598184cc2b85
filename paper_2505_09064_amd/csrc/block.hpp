// Block right-hand-side kernels: K independent PCG recurrences (one per load
// case) that share every matrix read.
//
// Vectors interleave the columns per vertex, v[(row*K + k)*VS + a] (column k,
// component a, stride VS): the K columns of one neighbour are K*VS consecutive
// values, so the lanes of a row that own the K columns gather them in one
// contiguous load while sharing one read of the matrix block (staged in LDS,
// below). The fine level keeps the padded stride (2 / 4: aligned vector loads,
// the layout of the FP64 PCG vectors); the coarse levels store D components with
// no padding (3D: a quarter fewer gathered bytes).
// A row is handled by GL lanes = K columns x (GL/K) block slots; the slots
// stride the row's blocks and are combined with cross-lane shuffles.
// Per-column scalars (alpha, beta, rho, residual, stop flag) follow Algorithm 2
// for every column separately; a column that has converged stops updating its
// vectors while the others go on.
#pragma once

#include <type_traits>

#include "kernels.hpp"

namespace vasmg {
namespace dev {

// Lanes per block row (GL = K columns x GL/K block slots, inside one wavefront
// so the slots combine with shuffles): point levels (fine) use 16 or 64, cell
// levels 32 or 64, chosen per level from its row lengths.
constexpr int kPointLanesNarrow = 16, kPointLanesWide = 64;
constexpr int kCellLanesNarrow = 32, kCellLanesWide = 64;

// Three consecutive FP32 values at 4-byte alignment: one 12-byte load.
struct alignas(4) Float3 {
  float a, b, c;
};

// D components at stride VS: aligned vector loads at the padded stride, one
// 12-byte load for packed 3D FP32 components, else component loads.
template <typename T, int D, int VS>
struct BlockVecIO {
  static __device__ __forceinline__ void load(const T* p, T* v) {
    if constexpr (VS == Pad<D>::value) {
      VecIO<T, D>::load(p, v);
    } else if constexpr (sizeof(T) == 4 && D == 3) {
      const Float3 f = *reinterpret_cast<const Float3*>(p);
      v[0] = f.a;
      v[1] = f.b;
      v[2] = f.c;
    } else {
#pragma unroll
      for (int a = 0; a < D; ++a) v[a] = p[a];
    }
  }
  static __device__ __forceinline__ void store(T* p, const T* v) {
    if constexpr (VS == Pad<D>::value) {
      VecIO<T, D>::store(p, v);
    } else {
#pragma unroll
      for (int a = 0; a < D; ++a) p[a] = v[a];
    }
  }
};

// Sum over the GL/K block slots of a row group (lanes with equal column).
template <typename T, int K, int GL>
__device__ __forceinline__ T slot_sum(T v) {
  static_assert(GL <= 64 && GL % K == 0, "a row group lies inside one wavefront");
#pragma unroll
  for (int off = K; off < GL; off <<= 1) v += __shfl_xor(v, off, GL);
  return v;
}

// acc += sum over blocks [kb, ke) of A_blk x_col(blk)[column k]; lane (slot, k)
// of the row group takes blocks kb + slot, kb + slot + S, ... in ascending order.
// The blocks go in chunks of CH (kStage on the cell levels, 4 per slot on the
// point levels): the row group's GL lanes copy a chunk's D*D planes and columns
// into LDS with coalesced loads (each value read once), and then every lane
// reads its blocks from there. Read directly, each matrix value would be loaded
// by each of the K column lanes, which multiplies what the load path returns
// per block by K. The next chunk's values are loaded while the current one is
// used.
constexpr int kStage = 16;

template <typename T, int D, int CH>
struct StageShape {
  static constexpr int DD = D * D;
  static constexpr int V = 16 / sizeof(T);               // values per 16-byte LDS read
  static constexpr int BS = (DD + V - 1) / V * V;         // LDS stride of one block
  static constexpr int NE = (DD + 1) * CH;                // planes and columns per chunk
};

template <typename T, int D, int CH = kStage>
struct alignas(16) RowStage {
  T val[CH * StageShape<T, D, CH>::BS];
  int col[CH];
};

template <typename T, int D, int K, int S, int VS, int GL, int CH = kStage, int CPL = 1>
__device__ __forceinline__ void mc_row_product_staged(int kb, int ke, int self, int lane, int slot,
                                                      int k, const int* __restrict__ col,
                                                      const T* __restrict__ val, int64_t nnz,
                                                      const T* __restrict__ x, T* acc,
                                                      RowStage<T, D, CH>& st) {
  using SS = StageShape<T, D, CH>;
  using IT = std::conditional_t<sizeof(T) == 4, int32_t, int64_t>;   // a column in a value's bits
  constexpr int NR = (SS::NE + GL - 1) / GL;   // staged values per lane and chunk
  constexpr int PB = CH / S;                   // blocks per lane and chunk
  static_assert(CH % S == 0, "slots divide a chunk");
  T pv[NR];
  auto fetch = [&](int p0) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int e = lane + r * GL;
      const int q = e / CH, b = e % CH;
      T v = T(0);
      if (e < SS::NE && p0 + b < ke) {
        if (q < SS::DD) v = val[q * nnz + p0 + b];
        else v = __builtin_bit_cast(T, static_cast<IT>(col[p0 + b]));
      }
      pv[r] = v;
    }
  };
  auto sync = [] {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  };
  if (kb < ke) fetch(kb);
  for (int p0 = kb; p0 < ke; p0 += CH) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int e = lane + r * GL;
      const int q = e / CH, b = e % CH;
      if (e < SS::NE) {
        if (q < SS::DD) st.val[b * SS::BS + q] = pv[r];
        else st.col[b] = p0 + b < ke ? static_cast<int>(__builtin_bit_cast(IT, pv[r])) : self;
      }
    }
    sync();
    if (p0 + CH < ke) fetch(p0 + CH);
    int j[PB];
#pragma unroll
    for (int i = 0; i < PB; ++i) j[i] = st.col[slot + i * S];
    // CPL columns per lane: k, k + K / CPL, ...; acc[h * D + a] is column h's
    T xv[PB][CPL][D];
#pragma unroll
    for (int i = 0; i < PB; ++i) {
      if (p0 + slot + i * S < ke) {
#pragma unroll
        for (int h = 0; h < CPL; ++h)
          BlockVecIO<T, D, VS>::load(x + (static_cast<int64_t>(j[i]) * K + k + h * (K / CPL)) * VS,
                                     xv[i][h]);
      }
    }
#pragma unroll
    for (int i = 0; i < PB; ++i) {
      const int b = slot + i * S;
      if (p0 + b < ke) {
        const T* m = st.val + b * SS::BS;
#pragma unroll
        for (int a = 0; a < D; ++a) {
#pragma unroll
          for (int c = 0; c < D; ++c) {
            const T mv = m[a * D + c];
#pragma unroll
            for (int h = 0; h < CPL; ++h) acc[h * D + a] += mv * xv[i][h][c];
          }
        }
      }
    }
    sync();   // the buffer is refilled with the next chunk
  }
}

// Point-level rows: staged in chunks of 4 blocks per slot (4 blocks in flight
// per lane), one buffer per row group.
template <typename T, int D, int K, int GL>
using PointStage = RowStage<T, D, 4 * (GL / K)>;

template <typename T, int D, int K, int GL>
__device__ __forceinline__ void mc_part_staged(const Part<T>& p, int i, int lane, int slot, int k,
                                               const T* __restrict__ x, T* acc,
                                               PointStage<T, D, K, GL>& st) {
  constexpr int S = GL / K;
  mc_row_product_staged<T, D, K, S, Pad<D>::value, GL, 4 * S>(p.ptr[i], p.ptr[i + 1], i, lane, slot,
                                                              k, p.col, p.val, p.nnz, x, acc, st);
}

// Per-column block sums: thread t contributes v to column col_of(t); on return
// thread t < K holds column t's sum (fixed order: ascending thread index).
template <int K, class ColOf>
__device__ __forceinline__ double block_sum_cols(double v, double* sh, ColOf col_of) {
  sh[threadIdx.x] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x < K)
    for (int j = 0; j < static_cast<int>(blockDim.x); ++j)
      if (col_of(j) == static_cast<int>(threadIdx.x)) s += sh[j];
  __syncthreads();
  return s;
}

// ---------------------------------------------------------------------------
// Fine-level FP64 SpMV y = A x per column, optional per-column partial x.y.
// ---------------------------------------------------------------------------
template <int D, int K, int GL, bool DOT>
__global__ __launch_bounds__(kBlock) void k_spmv_mc(int n, Part<double> L, Part<double> U,
                                                    const double* __restrict__ diag,
                                                    const double* __restrict__ x,
                                                    double* __restrict__ y,
                                                    double* __restrict__ partial) {
  constexpr int DP = Pad<D>::value;
  const int lane = threadIdx.x % GL, slot = lane / K, k = lane % K;
  const int i = xcd_block() * (kBlock / GL) + threadIdx.x / GL;
  __shared__ PointStage<double, D, K, GL> stg[kBlock / GL];
  double dot = 0.0;
  if (i < n) {
    double acc[D];
#pragma unroll
    for (int a = 0; a < D; ++a) acc[a] = 0.0;
    mc_part_staged<double, D, K, GL>(L, i, lane, slot, k, x, acc, stg[threadIdx.x / GL]);
    mc_part_staged<double, D, K, GL>(U, i, lane, slot, k, x, acc, stg[threadIdx.x / GL]);
#pragma unroll
    for (int a = 0; a < D; ++a) acc[a] = slot_sum<double, K, GL>(acc[a]);
    if (slot == 0) {
      double xi[D], yi[D];
      const int64_t o = (static_cast<int64_t>(i) * K + k) * DP;
      VecIO<double, D>::load(x + o, xi);
      const double* dg = diag + static_cast<int64_t>(i) * D * D;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        double s = acc[a];
#pragma unroll
        for (int b = 0; b < D; ++b) s += dg[a * D + b] * xi[b];
        yi[a] = s;
        if (DOT) dot += xi[a] * s;
      }
      VecIO<double, D>::store(y + o, yi);
    }
  }
  if (DOT) {
    __shared__ double sh[kBlock];
    const double s = block_sum_cols<K>(dot, sh, [](int t) { return t % K; });
    if (threadIdx.x < K) partial[static_cast<int64_t>(blockIdx.x) * K + threadIdx.x] = s;
  }
}

// ---------------------------------------------------------------------------
// Fine-level point Gauss-Seidel colour (MODE as in k_gs_color) and residual.
// ---------------------------------------------------------------------------
template <typename T, int D, int K, int GL, int MODE>
__global__ __launch_bounds__(kBlock) void k_gs_color_mc(
    int row0, int nrows, Part<T> L, Part<T> U, const T* __restrict__ diag,
    const T* __restrict__ b, T* x, T* __restrict__ s_save) {
  constexpr int DP = Pad<D>::value;
  const int lane = threadIdx.x % GL, slot = lane / K, k = lane % K;
  const int g = xcd_block() * (kBlock / GL) + threadIdx.x / GL;
  if (g >= nrows) return;
  const int i = row0 + g;
  T lo[D], up[D];
#pragma unroll
  for (int a = 0; a < D; ++a) { lo[a] = T(0); up[a] = T(0); }
  __shared__ PointStage<T, D, K, GL> stg[kBlock / GL];
  mc_part_staged<T, D, K, GL>(L, i, lane, slot, k, x, lo, stg[threadIdx.x / GL]);
  if (MODE != 0) mc_part_staged<T, D, K, GL>(U, i, lane, slot, k, x, up, stg[threadIdx.x / GL]);
#pragma unroll
  for (int a = 0; a < D; ++a) {
    lo[a] = slot_sum<T, K, GL>(lo[a]);
    if (MODE != 0) up[a] = slot_sum<T, K, GL>(up[a]);
  }
  if (slot != 0) return;
  const int64_t o = (static_cast<int64_t>(i) * K + k) * DP;
  T dg[D * D], xi[D], bi[D];
  const T* dp = diag + static_cast<int64_t>(i) * D * D;
#pragma unroll
  for (int e = 0; e < D * D; ++e) dg[e] = dp[e];
  VecIO<T, D>::load(b + o, bi);
  if (MODE == 0) {
#pragma unroll
    for (int a = 0; a < D; ++a) xi[a] = T(0);
  } else {
    VecIO<T, D>::load(x + o, xi);
  }
  T s[D], rhs[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    s[a] = bi[a] - lo[a];
    rhs[a] = s[a] - up[a];
  }
  if (MODE != 2 && s_save) VecIO<T, D>::store(s_save + o, s);
#pragma unroll
  for (int aa = 0; aa < D; ++aa) {
    const int a = (MODE == 2) ? D - 1 - aa : aa;
    T t = rhs[a];
#pragma unroll
    for (int c = 0; c < D; ++c)
      if (c != a) t -= dg[a * D + c] * xi[c];
    xi[a] = t / dg[a * D + a];
  }
  VecIO<T, D>::store(x + o, xi);
}

// r = s - D x - U x (after a forward sweep that saved s).
template <typename T, int D, int K, int GL>
__global__ __launch_bounds__(kBlock) void k_residual_upper_mc(
    int n, Part<T> U, const T* __restrict__ diag, const T* __restrict__ s_save,
    const T* __restrict__ x, T* __restrict__ r) {
  constexpr int DP = Pad<D>::value;
  const int lane = threadIdx.x % GL, slot = lane / K, k = lane % K;
  const int i = xcd_block() * (kBlock / GL) + threadIdx.x / GL;
  if (i >= n) return;
  T acc[D];
#pragma unroll
  for (int a = 0; a < D; ++a) acc[a] = T(0);
  __shared__ PointStage<T, D, K, GL> stg[kBlock / GL];
  mc_part_staged<T, D, K, GL>(U, i, lane, slot, k, x, acc, stg[threadIdx.x / GL]);
#pragma unroll
  for (int a = 0; a < D; ++a) acc[a] = slot_sum<T, K, GL>(acc[a]);
  if (slot != 0) return;
  const int64_t o = (static_cast<int64_t>(i) * K + k) * DP;
  T xi[D], si[D], ri[D];
  VecIO<T, D>::load(x + o, xi);
  VecIO<T, D>::load(s_save + o, si);
  const T* dg = diag + static_cast<int64_t>(i) * D * D;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    T v = si[a] - acc[a];
#pragma unroll
    for (int c = 0; c < D; ++c) v -= dg[a * D + c] * xi[c];
    ri[a] = v;
  }
  VecIO<T, D>::store(r + o, ri);
}

// ---------------------------------------------------------------------------
// Cell levels. Workgroup = one cell: lane group g (GL lanes) sums the
// off-cell part of row g for every column; the cell matrix is staged in LDS;
// then thread k < K runs column k's sequential sweep over the cell's unknowns.
// ---------------------------------------------------------------------------
template <typename T, int D, int K>
struct CellLds {
  static constexpr int NV = CellShape<D>::NV, NU = CellShape<D>::NU;
  T M[NU * NU];
  T lo[NV][K][D];
  T up[NV][K][D];
  RowStage<T, D> stage[NV];   // one per row group
};

template <typename T, int D, int K, int GL>
__device__ __forceinline__ void mc_cell_offcell(int v0, int m, const Part<T>& L, const Part<T>& U,
                                                const T* __restrict__ x, bool want_lo,
                                                bool want_up, CellLds<T, D, K>& sh) {
  // two columns per lane (k and k + K/2) from 8 columns up: a staged block is
  // read from LDS once for both
  constexpr int CPL = K >= 8 ? 2 : 1, KL = K / CPL;
  constexpr int S = GL / KL;
  static_assert(S <= kStage, "slots fit a chunk");
  const int g = threadIdx.x / GL, lane = threadIdx.x % GL, slot = lane / KL, k = lane % KL;
  T lo[CPL * D], up[CPL * D];
#pragma unroll
  for (int a = 0; a < CPL * D; ++a) { lo[a] = T(0); up[a] = T(0); }
  if (g < m) {
    const int i = v0 + g;
    if (want_lo)
      mc_row_product_staged<T, D, K, S, D, GL, kStage, CPL>(L.ptr[i], L.ptr[i + 1], i, lane, slot, k,
                                                            L.col, L.val, L.nnz, x, lo, sh.stage[g]);
    if (want_up)
      mc_row_product_staged<T, D, K, S, D, GL, kStage, CPL>(U.ptr[i], U.ptr[i + 1], i, lane, slot, k,
                                                            U.col, U.val, U.nnz, x, up, sh.stage[g]);
  }
#pragma unroll
  for (int a = 0; a < CPL * D; ++a) {
    if (want_lo) lo[a] = slot_sum<T, KL, GL>(lo[a]);
    if (want_up) up[a] = slot_sum<T, KL, GL>(up[a]);
  }
  if (slot == 0) {
#pragma unroll
    for (int h = 0; h < CPL; ++h) {
#pragma unroll
      for (int a = 0; a < D; ++a) {
        sh.lo[g][k + h * KL][a] = lo[h * D + a];
        sh.up[g][k + h * KL][a] = up[h * D + a];
      }
    }
  }
}

// In-cell sweep of two columns by one wavefront: lane 32h + t owns unknown t of
// column k0 + h; each new value is broadcast to the column's lanes with lane
// reads (the per-column analogue of k_gs_cell's sweep).
template <typename T, int D, int K, int MODE>
__device__ __forceinline__ void mc_cell_sweep_pair(int k0, int v0, int n, const T* __restrict__ Msh,
                                                   const CellLds<T, D, K>& sh,
                                                   const T* __restrict__ b, T* x,
                                                   T* __restrict__ s_save) {
  constexpr int DP = D;   // coarse-level vectors: packed
  constexpr int NU = CellShape<D>::NU;
  static_assert(NU <= 32, "a column's unknowns fit in half a wavefront");
  const int lane = threadIdx.x & 63, h = lane >> 5, t = lane & 31;
  const int k = k0 + h;
  const bool own = t < n && k < K;
  const int row = own ? t / D : 0, a = own ? t % D : 0;
  const int64_t o = (static_cast<int64_t>(v0 + row) * K + (own ? k : 0)) * DP + a;
  T Mrow[NU];
#pragma unroll
  for (int u = 0; u < NU; ++u) Mrow[u] = own ? Msh[u * NU + t] : T(0);
  T xc = T(0), acc = T(0);
  if (own) {
    const T su = b[o] - sh.lo[row][k][a];
    if (MODE != 2 && s_save) s_save[o] = su;
    acc = su - (MODE != 0 ? sh.up[row][k][a] : T(0));
    if (MODE != 0) xc = x[o];
  }
  const T rdg = own_reciprocal<T, NU>(Mrow, t, own);
  if (MODE != 0) {
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      if (u < n) {
        const T x0 = bcast(xc, u), x1 = bcast(xc, 32 + u);
        if (u != t) acc -= Mrow[u] * (h ? x1 : x0);
      }
    }
  }
#pragma unroll
  for (int uu = 0; uu < NU; ++uu) {
    const int u = (MODE == 2) ? NU - 1 - uu : uu;
    if (u < n) {
      T delta = T(0);
      if (t == u && own) {
        const T xn = acc * rdg;
        delta = xn - xc;
        xc = xn;
      }
      const T d0 = bcast(delta, u), d1 = bcast(delta, 32 + u);
      if (t != u) acc -= Mrow[u] * (h ? d1 : d0);
    }
  }
  if (own) x[o] = xc;
}

template <typename T, int D, int K, int GL, int MODE>
__global__ __launch_bounds__(CellShape<D>::NV * GL) void k_gs_cell_mc(
    int cell0, const int* __restrict__ cell_ptr, Part<T> L, Part<T> U,
    const T* __restrict__ cellM, const T* __restrict__ b, T* x, T* __restrict__ s_save) {
  constexpr int NU = CellShape<D>::NU;
  __shared__ CellLds<T, D, K> sh;
  const int c = cell0 + xcd_block();
  const int v0 = cell_ptr[c], m = cell_ptr[c + 1] - v0, n = m * D;
  const T* Mc = cellM + static_cast<int64_t>(c) * NU * NU;
  for (int e = threadIdx.x; e < NU * NU; e += blockDim.x) sh.M[e] = Mc[e];
  mc_cell_offcell<T, D, K, GL>(v0, m, L, U, x, true, MODE != 0, sh);
  __syncthreads();
  // wavefront w sweeps column pairs w, w + waves, ... (all lanes of a wave active)
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int k0 = 2 * w; k0 < K; k0 += 2 * nw)
    mc_cell_sweep_pair<T, D, K, MODE>(k0, v0, n, sh.M, sh, b, x, s_save);
}

// r = s - U x - M x on a cell (after a forward sweep that saved s).
template <typename T, int D, int K, int GL>
__global__ __launch_bounds__(CellShape<D>::NV * GL) void k_cell_residual_mc(
    const int* __restrict__ cell_ptr, Part<T> L, Part<T> U, const T* __restrict__ cellM,
    const T* __restrict__ s_save, const T* __restrict__ x, T* __restrict__ r) {
  constexpr int DP = D;   // coarse-level vectors: packed
  constexpr int NU = CellShape<D>::NU;
  __shared__ CellLds<T, D, K> sh;
  __shared__ T shx[NU][K];
  const int c = xcd_block();
  const int v0 = cell_ptr[c], m = cell_ptr[c + 1] - v0, n = m * D;
  const T* Mc = cellM + static_cast<int64_t>(c) * NU * NU;
  for (int e = threadIdx.x; e < NU * NU; e += blockDim.x) sh.M[e] = Mc[e];
  for (int e = threadIdx.x; e < NU * K; e += blockDim.x) {
    const int u = e / K, k = e % K;
    shx[u][k] = u < n ? x[(static_cast<int64_t>(v0 + u / D) * K + k) * DP + u % D] : T(0);
  }
  mc_cell_offcell<T, D, K, GL>(v0, m, L, U, x, false, true, sh);
  __syncthreads();
  for (int e = threadIdx.x; e < n * K; e += blockDim.x) {
    const int u = e / K, k = e % K;
    const int row = u / D, a = u % D;
    T mx = T(0);
    for (int v = 0; v < n; ++v) mx += sh.M[v * NU + u] * shx[v][k];
    const int64_t o = (static_cast<int64_t>(v0 + row) * K + k) * DP + a;
    r[o] = s_save[o] - sh.up[row][k][a] - mx;
  }
}

// ---------------------------------------------------------------------------
// Transfers: b_c = P^T r and x += P e, lane k of a K-lane group = column k.
// ---------------------------------------------------------------------------
// VF: stride of the fine level's vectors; the coarse level's are packed (D).
template <typename T, int D, int K, int VF>
__global__ __launch_bounds__(kBlock) void k_restrict_mc(int nc, const int* __restrict__ ptr,
                                                        const int* __restrict__ idx,
                                                        const T* __restrict__ w,
                                                        const T* __restrict__ r,
                                                        T* __restrict__ bc) {
  const int k = threadIdx.x % K;
  const int I = xcd_block() * (kBlock / K) + threadIdx.x / K;
  if (I >= nc) return;
  T acc[D];
#pragma unroll
  for (int a = 0; a < D; ++a) acc[a] = T(0);
  for (int p = ptr[I]; p < ptr[I + 1]; ++p) {
    T e[D];
    BlockVecIO<T, D, VF>::load(r + (static_cast<int64_t>(idx[p]) * K + k) * VF, e);
    const T wp = w[p];
#pragma unroll
    for (int a = 0; a < D; ++a) acc[a] += wp * e[a];
  }
  BlockVecIO<T, D, D>::store(bc + (static_cast<int64_t>(I) * K + k) * D, acc);
}

template <typename T, int D, int K, int VF>
__global__ __launch_bounds__(kBlock) void k_prolong_mc(int nf, const int* __restrict__ ptr,
                                                       const int* __restrict__ idx,
                                                       const T* __restrict__ w,
                                                       const T* __restrict__ e, T* x,
                                                       const uint8_t* __restrict__ fixed) {
  const int k = threadIdx.x % K;
  const int i = xcd_block() * (kBlock / K) + threadIdx.x / K;
  if (i >= nf) return;
  const int64_t o = (static_cast<int64_t>(i) * K + k) * VF;
  T xi[D], acc[D];
  BlockVecIO<T, D, VF>::load(x + o, xi);
#pragma unroll
  for (int a = 0; a < D; ++a) acc[a] = T(0);
  for (int p = ptr[i]; p < ptr[i + 1]; ++p) {
    T ev[D];
    BlockVecIO<T, D, D>::load(e + (static_cast<int64_t>(idx[p]) * K + k) * D, ev);
    const T wp = w[p];
#pragma unroll
    for (int a = 0; a < D; ++a) acc[a] += wp * ev[a];
  }
  const int fx = fixed ? fixed[i] : 0;   // constrained components: zero prolongation rows
#pragma unroll
  for (int a = 0; a < D; ++a) xi[a] += ((fx >> a) & 1) ? T(0) : acc[a];
  BlockVecIO<T, D, VF>::store(x + o, xi);
}

// Coarsest solve L L^T e = b per column (FP64, one workgroup; n * K <= kCoarseMax).
// VS: stride of the coarsest level's vectors (padded if it is the fine level).
template <typename T, int D, int K, int VS>
__global__ __launch_bounds__(kBlock) void k_coarse_solve_mc(int n, const double* __restrict__ L,
                                                            const T* __restrict__ b,
                                                            T* __restrict__ x) {
  constexpr int DP = VS;
  __shared__ double y[kCoarseMax];
  const int nk = n * K;
  for (int e = threadIdx.x; e < nk; e += blockDim.x) {
    const int i = e / K, k = e % K;
    y[e] = static_cast<double>(b[((i / D) * K + k) * DP + i % D]);
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    if (threadIdx.x < K) y[j * K + threadIdx.x] /= L[static_cast<int64_t>(j) * n + j];
    __syncthreads();
    for (int e = (j + 1) * K + threadIdx.x; e < nk; e += blockDim.x)
      y[e] -= L[static_cast<int64_t>(e / K) * n + j] * y[j * K + e % K];
    __syncthreads();
  }
  for (int j = n - 1; j >= 0; --j) {
    if (threadIdx.x < K) y[j * K + threadIdx.x] /= L[static_cast<int64_t>(j) * n + j];
    __syncthreads();
    for (int e = threadIdx.x; e < j * K; e += blockDim.x)
      y[e] -= L[static_cast<int64_t>(j) * n + e / K] * y[j * K + e % K];
    __syncthreads();
  }
  for (int e = threadIdx.x; e < nk; e += blockDim.x) {
    const int i = e / K, k = e % K;
    x[((i / D) * K + k) * DP + i % D] = static_cast<T>(y[e]);
  }
}

// Small coarsest levels: x = A_c^{-1} b per column (n <= kCoarseInvMax).
template <typename T, int D, int K, int VS>
__global__ __launch_bounds__(kBlock) void k_coarse_apply_mc(int n, const double* __restrict__ Minv,
                                                            const T* __restrict__ b,
                                                            T* __restrict__ x) {
  __shared__ double y[kCoarseMax];
  const int nk = n * K;
  for (int e = threadIdx.x; e < nk; e += blockDim.x) {
    const int i = e / K, k = e % K;
    y[e] = static_cast<double>(b[((i / D) * K + k) * VS + i % D]);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nk; e += blockDim.x) {
    const int i = e / K, k = e % K;
    const double* row = Minv + static_cast<int64_t>(i) * n;
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += row[j] * y[j * K + k];
    x[((i / D) * K + k) * VS + i % D] = static_cast<T>(s);
  }
}

// ---------------------------------------------------------------------------
// PCG vector kernels over [row][K][DP] (flat grid-stride; the stride is a
// multiple of K*DP, so every thread stays on one column).
// ---------------------------------------------------------------------------
template <int K, int DP>
__device__ __forceinline__ int flat_col(int t) {
  return (t / DP) % K;
}

// per-column scalar updates, one workgroup per column
template <int MODE, int K>
__global__ __launch_bounds__(kBlock) void k_finalize_mc(const double* __restrict__ partial, int np,
                                                        Scalars* sc) {
  __shared__ double sh[kBlock];
  const int k = blockIdx.x;
  Scalars* s = sc + k;
  if (MODE != FIN_NORMF && MODE != FIN_TRUE && s->done) return;
  double v = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) v += partial[static_cast<int64_t>(i) * K + k];
  const double tot = block_sum(v, sh);
  if (threadIdx.x == 0) finalize_scalar<MODE>(tot, s);
}

template <int K, int DP, typename TB>
__global__ __launch_bounds__(kBlock) void k_dot_mc(int64_t n, const double* __restrict__ a,
                                                   const TB* __restrict__ b,
                                                   double* __restrict__ partial) {
  __shared__ double sh[kBlock];
  double v = 0.0;
  for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kBlock)
    v += a[i] * static_cast<double>(b[i]);
  const double s = block_sum_cols<K>(v, sh, [](int t) { return flat_col<K, DP>(t); });
  if (threadIdx.x < K) partial[static_cast<int64_t>(blockIdx.x) * K + threadIdx.x] = s;
}

// r = F - q per column (r may be NULL), partial ||r||^2
template <int K, int DP>
__global__ __launch_bounds__(kBlock) void k_sub_norm_mc(int64_t n, const double* __restrict__ F,
                                                        const double* __restrict__ q,
                                                        double* __restrict__ r,
                                                        double* __restrict__ partial) {
  __shared__ double sh[kBlock];
  double v = 0.0;
  for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kBlock) {
    const double t = F[i] - q[i];
    if (r) r[i] = t;
    v += t * t;
  }
  const double s = block_sum_cols<K>(v, sh, [](int t) { return flat_col<K, DP>(t); });
  if (threadIdx.x < K) partial[static_cast<int64_t>(blockIdx.x) * K + threadIdx.x] = s;
}

// x += alpha_k p; r -= alpha_k q; b0 = (T) r; partial ||r||^2 (running columns)
template <typename T, int K, int DP>
__global__ __launch_bounds__(kBlock) void k_update_xr_mc(int64_t n, const Scalars* __restrict__ sc,
                                                         const double* __restrict__ p,
                                                         const double* __restrict__ q,
                                                         double* __restrict__ x,
                                                         double* __restrict__ r,
                                                         T* __restrict__ b0,
                                                         double* __restrict__ partial) {
  __shared__ double sh[kBlock];
  const int k = flat_col<K, DP>(threadIdx.x);
  const bool run = !sc[k].done;
  const double alpha = sc[k].alpha;
  double v = 0.0;
  if (run) {
    for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * kBlock) {
      x[i] += alpha * p[i];
      const double ri = r[i] - alpha * q[i];
      r[i] = ri;
      if (b0) b0[i] = static_cast<T>(ri);
      v += ri * ri;
    }
  }
  const double s = block_sum_cols<K>(v, sh, [](int t) { return flat_col<K, DP>(t); });
  if (threadIdx.x < K) partial[static_cast<int64_t>(blockIdx.x) * K + threadIdx.x] = s;
}

// p = z + beta_k p (running columns)
template <typename T, int K, int DP>
__global__ __launch_bounds__(kBlock) void k_update_p_mc(int64_t n, const Scalars* __restrict__ sc,
                                                        const T* __restrict__ z,
                                                        double* __restrict__ p) {
  const int k = flat_col<K, DP>(threadIdx.x);
  if (sc[k].done) return;
  const double beta = sc[k].beta;
  for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kBlock)
    p[i] = static_cast<double>(z[i]) + beta * p[i];
}

// columns with F = 0 have x = 0; a zero-guess start of such a column is done
template <int K, int DP>
__global__ __launch_bounds__(kBlock) void k_zero_cols_mc(int64_t n, const Scalars* __restrict__ sc,
                                                         double* __restrict__ x) {
  const int k = flat_col<K, DP>(threadIdx.x);
  if (sc[k].normF != 0.0) return;
  for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kBlock)
    x[i] = 0.0;
}

// per-column start: rtol, and (with an initial guess) stop columns whose
// initial residual already meets it
template <int K>
__global__ void k_start_mc(Scalars* sc, double rtol, int have_x0) {
  const int k = threadIdx.x;
  if (k >= K) return;
  Scalars* s = sc + k;
  s->rtol = rtol;
  if (!(s->normF == s->normF) || s->normF > 1.7976931348623157e308) {
    s->status = 5;
    s->done = 1;
  } else if (s->normF == 0.0) {
    s->done = 1;
  } else if (have_x0 && s->res_true / s->normF < rtol) {
    s->done = 1;
  }
}

// user layout [n_rhs][nv][D], columns c0 .. c0+nc-1 <-> [row][K][DP]
template <int D, int K>
__global__ __launch_bounds__(kBlock) void k_gather_user_mc(int n, const int* __restrict__ map,
                                                           const double* __restrict__ src,
                                                           int64_t nv, int c0, int nc,
                                                           double* __restrict__ dst,
                                                           const uint8_t* __restrict__ fixed) {
  constexpr int DP = Pad<D>::value;
  const int64_t e = blockIdx.x * int64_t(kBlock) + threadIdx.x;
  if (e >= static_cast<int64_t>(n) * K) return;
  const int i = static_cast<int>(e / K), k = static_cast<int>(e % K);
  const int64_t v = map[i];
  const int fx = fixed ? fixed[i] : 0;   // constrained components read as 0
#pragma unroll
  for (int a = 0; a < DP; ++a)
    dst[e * DP + a] = (a < D && k < nc && !((fx >> a) & 1))
                          ? src[(static_cast<int64_t>(c0 + k) * nv + v) * D + a]
                          : 0.0;
}

template <int D, int K>
__global__ __launch_bounds__(kBlock) void k_scatter_user_mc(int n, const int* __restrict__ map,
                                                            const double* __restrict__ src,
                                                            int64_t nv, int c0, int nc,
                                                            double* __restrict__ dst) {
  constexpr int DP = Pad<D>::value;
  const int64_t e = blockIdx.x * int64_t(kBlock) + threadIdx.x;
  if (e >= static_cast<int64_t>(n) * K) return;
  const int i = static_cast<int>(e / K), k = static_cast<int>(e % K);
  if (k >= nc) return;
  const int64_t v = map[i];
#pragma unroll
  for (int a = 0; a < D; ++a) dst[(static_cast<int64_t>(c0 + k) * nv + v) * D + a] = src[e * DP + a];
}

}  // namespace dev
}  // namespace vasmg
