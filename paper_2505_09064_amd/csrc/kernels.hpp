// HIP kernels of the V-ASMG-PCG solve phase for gfx950 (CDNA4, wave64).
//
// Data layout (per level, device numbering = vertices sorted by colour, then
// cell, then canonical index):
//   * the blocks coupling a row to earlier colours (L) and to later colours (U)
//     are two separate CSR matrices, each with ascending columns and values
//     stored component-plane-major, val[(a*D+b)*nnz + k]: lanes walking a row
//     read consecutive addresses, and a sweep or residual that needs only one
//     of the two streams one contiguous array;
//   * fine level: diagonal blocks dense, diag[i*D*D + a*D + b]; coarse levels:
//     the blocks inside a Gauss-Seidel cell (diagonal included) as a dense
//     matrix per cell;
//   * vectors vertex-major with a padded stride DP (2 in 2D, 4 in 3D) so a
//     neighbour's components come in one 8/16-byte (FP32) or 16/32-byte (FP64)
//     load; pad entries are kept at zero.
// A block row is handled by a group of G lanes (G divides 64) that stride over
// its blocks; partial sums are combined with cross-lane shuffles inside the
// group and lane 0 of the group (or wavefront 0 of a cell) finishes the row.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vasmg {
namespace dev {

constexpr int kBlock = 256;

template <int D>
struct Pad {
  static constexpr int value = (D == 3) ? 4 : 2;
};

// One of the two off-diagonal block matrices (L or U) of a level.
template <typename T>
struct Part {
  const int* __restrict__ ptr;   // [n+1]
  const int* __restrict__ col;   // [nnz]
  const T* __restrict__ val;     // [D*D][nnz]
  int64_t nnz;
};

// ---- padded vector loads/stores -------------------------------------------
template <typename T, int D>
struct VecIO;

template <>
struct VecIO<float, 2> {
  static __device__ __forceinline__ void load(const float* p, float* v) {
    const float2 t = *reinterpret_cast<const float2*>(p);
    v[0] = t.x; v[1] = t.y;
  }
  static __device__ __forceinline__ void store(float* p, const float* v) {
    *reinterpret_cast<float2*>(p) = make_float2(v[0], v[1]);
  }
};
template <>
struct VecIO<float, 3> {
  static __device__ __forceinline__ void load(const float* p, float* v) {
    const float4 t = *reinterpret_cast<const float4*>(p);
    v[0] = t.x; v[1] = t.y; v[2] = t.z;
  }
  static __device__ __forceinline__ void store(float* p, const float* v) {
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], 0.0f);
  }
};
template <>
struct VecIO<double, 2> {
  static __device__ __forceinline__ void load(const double* p, double* v) {
    const double2 t = *reinterpret_cast<const double2*>(p);
    v[0] = t.x; v[1] = t.y;
  }
  static __device__ __forceinline__ void store(double* p, const double* v) {
    *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
  }
};
template <>
struct VecIO<double, 3> {
  static __device__ __forceinline__ void load(const double* p, double* v) {
    const double2 t0 = *reinterpret_cast<const double2*>(p);
    const double2 t1 = *reinterpret_cast<const double2*>(p + 2);
    v[0] = t0.x; v[1] = t0.y; v[2] = t1.x;
  }
  static __device__ __forceinline__ void store(double* p, const double* v) {
    *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
    *reinterpret_cast<double2*>(p + 2) = make_double2(v[2], 0.0);
  }
};

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2).
// Renumber them so each XCD walks one contiguous range of rows or cells:
// neighbouring rows then gather the same vector lines through the same L2.
__device__ __forceinline__ int xcd_block() {
  const int g = gridDim.x, b = blockIdx.x;
  const int q = g >> 3, r = g & 7;
  const int k = b & 7, j = b >> 3;
  return (k < r) ? k * (q + 1) + j : r * (q + 1) + (k - r) * q + j;
}

template <typename T, int G>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
  return v;
}

// Block-wide deterministic sum of one value per thread (fixed tree order).
__device__ __forceinline__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Broadcast of lane l's value to the wavefront (l uniform, all lanes active).
__device__ __forceinline__ float bcast(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double bcast(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(b), l);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), l);
  return __longlong_as_double((static_cast<long long>(hi) << 32) |
                              static_cast<unsigned int>(lo));
}

template <typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
  return *p;
}

template <typename T, int D>
__device__ __forceinline__ void block_fma(const T* __restrict__ val, int64_t nnz, int k,
                                          const T* xj, T* acc) {
#pragma unroll
  for (int a = 0; a < D; ++a) {
#pragma unroll
    for (int b = 0; b < D; ++b) acc[a] += ld_stream(val + (a * D + b) * nnz + k) * xj[b];
  }
}

// Off-diagonal block row product over positions [kb, ke): acc += sum A_k x_col(k).
// UN blocks per lane are loaded before any is used (4 in FP32, so a whole row of
// a coarse level is in flight at once; 2 in FP64 to keep the register budget).
template <typename T, int D, int G>
__device__ __forceinline__ void row_product(int kb, int ke, int lane, const int* __restrict__ col,
                                            const T* __restrict__ val, int64_t nnz,
                                            const T* __restrict__ x, T* acc) {
  constexpr int DP = Pad<D>::value;
  constexpr int UN = sizeof(T) == 4 ? 4 : 2;
  int k = kb + lane;
  for (; k + (UN - 1) * G < ke; k += UN * G) {
    int j[UN];
#pragma unroll
    for (int u = 0; u < UN; ++u) j[u] = col[k + u * G];
    T xv[UN][D];
#pragma unroll
    for (int u = 0; u < UN; ++u) VecIO<T, D>::load(x + static_cast<int64_t>(j[u]) * DP, xv[u]);
#pragma unroll
    for (int u = 0; u < UN; ++u) block_fma<T, D>(val, nnz, k + u * G, xv[u], acc);
  }
  for (; k < ke; k += G) {
    const int jj = col[k];
    T xj[D];
    VecIO<T, D>::load(x + static_cast<int64_t>(jj) * DP, xj);
    block_fma<T, D>(val, nnz, k, xj, acc);
  }
}

// Cell levels store every row's L and U blocks padded to whole quads of kQuad
// consecutive blocks (padding: zero blocks pointing at the row itself), so a lane
// takes a quad per step: one 16-byte load of its 4 columns, 4 neighbour
// gathers, and per matrix plane one 16-byte (FP32) or two (FP64) loads. Rows
// and plane strides are multiples of kQuad, so every such load is aligned.
constexpr int kQuad = 4;

template <typename T>
struct Quad;
template <>
struct Quad<float> {
  static __device__ __forceinline__ void load(const float* p, float* v) {
    const float4 t = *reinterpret_cast<const float4*>(p);
    v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
  }
};
template <>
struct Quad<double> {
  static __device__ __forceinline__ void load(const double* p, double* v) {
    const double2 a = *reinterpret_cast<const double2*>(p);
    const double2 b = *reinterpret_cast<const double2*>(p + 2);
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
  }
};

// acc += sum over the quads of positions [kb, ke) (multiples of kQuad).
template <typename T, int D, int G>
__device__ __forceinline__ void quad_product(int kb, int ke, int lane, const int* __restrict__ col,
                                             const T* __restrict__ val, int64_t nnz,
                                             const T* __restrict__ x, T* acc) {
  constexpr int DP = Pad<D>::value;
  for (int q = kb / kQuad + lane; q < ke / kQuad; q += G) {
    const int4 j = reinterpret_cast<const int4*>(col)[q];
    T xv[kQuad][D];
    VecIO<T, D>::load(x + static_cast<int64_t>(j.x) * DP, xv[0]);
    VecIO<T, D>::load(x + static_cast<int64_t>(j.y) * DP, xv[1]);
    VecIO<T, D>::load(x + static_cast<int64_t>(j.z) * DP, xv[2]);
    VecIO<T, D>::load(x + static_cast<int64_t>(j.w) * DP, xv[3]);
#pragma unroll
    for (int a = 0; a < D; ++a) {
#pragma unroll
      for (int b = 0; b < D; ++b) {
        T v[kQuad];
        Quad<T>::load(val + static_cast<int64_t>(a * D + b) * nnz + static_cast<int64_t>(q) * kQuad, v);
        acc[a] += v[0] * xv[0][b] + v[1] * xv[1][b] + v[2] * xv[2][b] + v[3] * xv[3][b];
      }
    }
  }
}

// FP32 takes the quad step; FP64 keeps the per-block step on the same padded
// rows (padding blocks are zeros): a quad of doubles costs more registers than it
// saves in loads (occupancy 3-4 waves per SIMD, measured 20% slower).
template <typename T, int D, int G>
__device__ __forceinline__ void part_quad_product(const Part<T>& p, int i, int lane,
                                                  const T* __restrict__ x, T* acc) {
  if constexpr (sizeof(T) == 4)
    quad_product<T, D, G>(p.ptr[i], p.ptr[i + 1], lane, p.col, p.val, p.nnz, x, acc);
  else
    row_product<T, D, G>(p.ptr[i], p.ptr[i + 1], lane, p.col, p.val, p.nnz, x, acc);
}

template <typename T, int D, int G>
__device__ __forceinline__ void part_product(const Part<T>& p, int i, int lane,
                                             const T* __restrict__ x, T* acc) {
  row_product<T, D, G>(p.ptr[i], p.ptr[i + 1], lane, p.col, p.val, p.nnz, x, acc);
}

// ---------------------------------------------------------------------------
// K1: y = A x (diag + off-diagonal), optional partial dot x.y per workgroup.
// ---------------------------------------------------------------------------
template <typename T, int D, int G, bool DOT>
__global__ __launch_bounds__(kBlock) void k_spmv(int n, Part<T> L, Part<T> U,
                                                 const T* __restrict__ diag,
                                                 const T* __restrict__ x, T* __restrict__ y,
                                                 double* __restrict__ partial,
                                                 const int* __restrict__ done) {
  if (done && *done) return;
  constexpr int DP = Pad<D>::value;
  const int lane = threadIdx.x % G;
  const int i = xcd_block() * (kBlock / G) + threadIdx.x / G;
  double dot = 0.0;
  if (i < n) {
    T acc[D];
#pragma unroll
    for (int a = 0; a < D; ++a) acc[a] = T(0);
    part_product<T, D, G>(L, i, lane, x, acc);
    part_product<T, D, G>(U, i, lane, x, acc);
#pragma unroll
    for (int a = 0; a < D; ++a) acc[a] = group_sum<T, G>(acc[a]);
    if (lane == 0) {
      T xi[D], yi[D];
      VecIO<T, D>::load(x + static_cast<int64_t>(i) * DP, xi);
      const T* dg = diag + static_cast<int64_t>(i) * D * D;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        T s = acc[a];
#pragma unroll
        for (int b = 0; b < D; ++b) s += dg[a * D + b] * xi[b];
        yi[a] = s;
        if (DOT) dot += static_cast<double>(xi[a]) * static_cast<double>(s);
      }
      VecIO<T, D>::store(y + static_cast<int64_t>(i) * DP, yi);
    }
  }
  if (DOT) {
    __shared__ double sh[kBlock];
    const double s = block_sum(dot, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
  }
}

// r = b - A x (full row), used when no saved lower-part sums exist.
template <typename T, int D, int G>
__global__ __launch_bounds__(kBlock) void k_residual_full(
    int n, Part<T> L, Part<T> U, const T* __restrict__ diag, const T* __restrict__ b,
    const T* __restrict__ x, T* __restrict__ r, const int* __restrict__ done) {
  if (done && *done) return;
  constexpr int DP = Pad<D>::value;
  const int lane = threadIdx.x % G;
  const int i = xcd_block() * (kBlock / G) + threadIdx.x / G;
  if (i >= n) return;
  T acc[D];
#pragma unroll
  for (int a = 0; a < D; ++a) acc[a] = T(0);
  part_product<T, D, G>(L, i, lane, x, acc);
  part_product<T, D, G>(U, i, lane, x, acc);
#pragma unroll
  for (int a = 0; a < D; ++a) acc[a] = group_sum<T, G>(acc[a]);
  if (lane == 0) {
    T xi[D], bi[D], ri[D];
    VecIO<T, D>::load(x + static_cast<int64_t>(i) * DP, xi);
    VecIO<T, D>::load(b + static_cast<int64_t>(i) * DP, bi);
    const T* dg = diag + static_cast<int64_t>(i) * D * D;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      T s = bi[a] - acc[a];
#pragma unroll
      for (int c = 0; c < D; ++c) s -= dg[a * D + c] * xi[c];
      ri[a] = s;
    }
    VecIO<T, D>::store(r + static_cast<int64_t>(i) * DP, ri);
  }
}

// ---------------------------------------------------------------------------
// K3: one colour of a point Gauss-Seidel sweep (Algorithm 1 in colour order).
//   MODE 0: forward from a zero guess (only earlier colours are nonzero, so
//           only L is read); saves s_i = b_i - sum_{j<i} A_ij x_j
//   MODE 1: forward from a nonzero guess; saves s_i as well
//   MODE 2: backward (components in reverse order)
// ---------------------------------------------------------------------------
template <typename T, int D, int G, int MODE>
__global__ __launch_bounds__(kBlock) void k_gs_color(
    int row0, int nrows, Part<T> L, Part<T> U, const T* __restrict__ diag,
    const T* __restrict__ b, T* x, T* __restrict__ s_save, const int* __restrict__ done) {
  if (done && *done) return;
  constexpr int DP = Pad<D>::value;
  const int lane = threadIdx.x % G;
  const int g = xcd_block() * (kBlock / G) + threadIdx.x / G;
  if (g >= nrows) return;
  const int i = row0 + g;
  // lane 0 fetches what it needs to finish the row before the row product
  T dg[D * D], xi[D], bi[D];
  if (lane == 0) {
    const T* dp = diag + static_cast<int64_t>(i) * D * D;
#pragma unroll
    for (int e = 0; e < D * D; ++e) dg[e] = dp[e];
    VecIO<T, D>::load(b + static_cast<int64_t>(i) * DP, bi);
    if (MODE == 0) {
#pragma unroll
      for (int a = 0; a < D; ++a) xi[a] = T(0);
    } else {
      VecIO<T, D>::load(x + static_cast<int64_t>(i) * DP, xi);
    }
  }
  T lo[D], up[D];
#pragma unroll
  for (int a = 0; a < D; ++a) { lo[a] = T(0); up[a] = T(0); }
  part_product<T, D, G>(L, i, lane, x, lo);
  if (MODE != 0) part_product<T, D, G>(U, i, lane, x, up);
#pragma unroll
  for (int a = 0; a < D; ++a) {
    lo[a] = group_sum<T, G>(lo[a]);
    if (MODE != 0) up[a] = group_sum<T, G>(up[a]);
  }
  if (lane != 0) return;
  T s[D], rhs[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    s[a] = bi[a] - lo[a];
    rhs[a] = s[a] - up[a];
  }
  if (MODE != 2 && s_save) VecIO<T, D>::store(s_save + static_cast<int64_t>(i) * DP, s);
  if (MODE != 2) {
#pragma unroll
    for (int a = 0; a < D; ++a) {
      T t = rhs[a];
#pragma unroll
      for (int c = 0; c < D; ++c)
        if (c != a) t -= dg[a * D + c] * xi[c];
      xi[a] = t / dg[a * D + a];
    }
  } else {
#pragma unroll
    for (int a = D - 1; a >= 0; --a) {
      T t = rhs[a];
#pragma unroll
      for (int c = 0; c < D; ++c)
        if (c != a) t -= dg[a * D + c] * xi[c];
      xi[a] = t / dg[a * D + a];
    }
  }
  VecIO<T, D>::store(x + static_cast<int64_t>(i) * DP, xi);
}

// K2: r = s - D x - sum_{j > i} A_ij x_j after a forward sweep that saved s.
template <typename T, int D, int G>
__global__ __launch_bounds__(kBlock) void k_residual_upper(
    int n, Part<T> U, const T* __restrict__ diag, const T* __restrict__ s_save,
    const T* __restrict__ x, T* __restrict__ r, const int* __restrict__ done) {
  if (done && *done) return;
  constexpr int DP = Pad<D>::value;
  const int lane = threadIdx.x % G;
  const int i = xcd_block() * (kBlock / G) + threadIdx.x / G;
  if (i >= n) return;
  T acc[D];
#pragma unroll
  for (int a = 0; a < D; ++a) acc[a] = T(0);
  part_product<T, D, G>(U, i, lane, x, acc);
#pragma unroll
  for (int a = 0; a < D; ++a) acc[a] = group_sum<T, G>(acc[a]);
  if (lane == 0) {
    T xi[D], si[D], ri[D];
    VecIO<T, D>::load(x + static_cast<int64_t>(i) * DP, xi);
    VecIO<T, D>::load(s_save + static_cast<int64_t>(i) * DP, si);
    const T* dg = diag + static_cast<int64_t>(i) * D * D;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      T s = si[a] - acc[a];
#pragma unroll
      for (int c = 0; c < D; ++c) s -= dg[a * D + c] * xi[c];
      ri[a] = s;
    }
    VecIO<T, D>::store(r + static_cast<int64_t>(i) * DP, ri);
  }
}

// ---------------------------------------------------------------------------
// Coarse lattice levels: Gauss-Seidel over cells of at most NV = 2^D vertices.
// Device rows of a cell are contiguous ([cell_ptr[c], cell_ptr[c+1])); L and U
// hold only blocks coupling to other cells (earlier / later colours); the blocks
// inside a cell, diagonal included, are a dense NU x NU matrix per cell
// (NU = NV * D, column-major: cellM[c*NU*NU + u*NU + t] = M[t][u]).
// One workgroup handles one cell: lane group g sums the off-cell part of the
// cell's g-th row, then lane t of wavefront 0 owns unknown t (vertex t / D,
// component t % D) for the sequential sweep inside the cell, which broadcasts
// each new value with a shuffle.
// ---------------------------------------------------------------------------
template <int D>
struct CellShape {
  static constexpr int NV = 1 << D;
  static constexpr int NU = NV * D;
};

// Cells per workgroup: one per workgroup when a cell's NV * GR lanes fill a
// wavefront or more (its wavefront 0 runs the in-cell sweep); otherwise as many
// as share one wavefront (2D cells with 4 or 8 lanes per row), each with its own
// lane segment for the off-cell sums and the in-cell sweep.
template <int D, int GR>
struct CellPack {
  static constexpr int CT = (1 << D) * GR;                 // lanes per cell
  static constexpr int CPW = CT >= 64 ? 1 : 64 / CT;
  static constexpr int threads = CT * CPW;
};

// Value of lane u of the calling lane's cell segment (segment = cell slot):
// the wavefront-wide read-lane when one cell owns the wavefront, else a
// shuffle; every lane of the wavefront must call it.
template <int CPW, int CT, typename T>
__device__ __forceinline__ T cell_bcast(T v, int slot, int u) {
  if constexpr (CPW == 1)
    return bcast(v, u);
  else
    return __shfl(v, slot * CT + u, 64);
}

// Reciprocal of the lane's own diagonal entry Mrow[t] (1 for lanes without a
// row), taken once before the sequential in-cell sweep: each of its steps then
// costs a multiply instead of a division on the dependent chain.
template <typename T, int NU>
__device__ __forceinline__ T own_reciprocal(const T* Mrow, int t, bool own) {
  T dg = T(1);
#pragma unroll
  for (int u = 0; u < NU; ++u)
    if (u == t) dg = Mrow[u];
  return own ? T(1) / dg : T(1);
}

// Per-cell block of NV * GR threads: lane group g (GR lanes, inside one
// wavefront) sums the off-cell part of the cell's g-th row; the sums meet in
// LDS; wavefront 0 then runs the sequential sweep over the cell's unknowns.
// On colour-block levels (E, F non-null) the lower sums take E with L and the
// upper sums F with U.
template <typename T, int D, int GR>
__device__ __forceinline__ void cell_offcell_sums(int v0, int m, const Part<T>& L,
                                                  const Part<T>& U, const T* __restrict__ x,
                                                  bool want_lo, bool want_up, T (*sh_lo)[D],
                                                  T (*sh_up)[D], int tc, const Part<T>* E = nullptr,
                                                  const Part<T>* F = nullptr) {
  const int g = tc / GR, gl = tc % GR;
  T lo[D], up[D];
#pragma unroll
  for (int a = 0; a < D; ++a) { lo[a] = T(0); up[a] = T(0); }
  if (g < m) {
    const int i = v0 + g;
    if (want_lo) part_quad_product<T, D, GR>(L, i, gl, x, lo);
    if (want_lo && E) part_quad_product<T, D, GR>(*E, i, gl, x, lo);
    if (want_up) part_quad_product<T, D, GR>(U, i, gl, x, up);
    if (want_up && F) part_quad_product<T, D, GR>(*F, i, gl, x, up);
  }
#pragma unroll
  for (int a = 0; a < D; ++a) {
    if (want_lo) lo[a] = group_sum<T, GR>(lo[a]);
    if (want_up) up[a] = group_sum<T, GR>(up[a]);
  }
  if (gl == 0) {
#pragma unroll
    for (int a = 0; a < D; ++a) {
      sh_lo[g][a] = lo[a];
      sh_up[g][a] = up[a];
    }
  }
  __syncthreads();
}

template <typename T, int D, int GR, int MODE>
__global__ __launch_bounds__((CellPack<D, GR>::threads)) void k_gs_cell(
    int cell0, int ncell, const int* __restrict__ cell_ptr, Part<T> L, Part<T> U,
    const T* __restrict__ cellM, const T* __restrict__ b, T* x, T* __restrict__ s_save,
    const int* __restrict__ done) {
  if (done && *done) return;
  constexpr int DP = Pad<D>::value;
  constexpr int NV = CellShape<D>::NV, NU = CellShape<D>::NU;
  constexpr int CT = CellPack<D, GR>::CT, CPW = CellPack<D, GR>::CPW;
  __shared__ T sh_lo[CPW][NV][D], sh_up[CPW][NV][D];
  const int slot = CPW == 1 ? 0 : threadIdx.x / CT;
  const int t = CPW == 1 ? threadIdx.x : threadIdx.x % CT;
  const int ci = xcd_block() * CPW + slot;
  const bool live = CPW == 1 || ci < ncell;   // the last workgroup may hold fewer cells
  const int c = cell0 + (live ? ci : 0);
  const int v0 = cell_ptr[c], m = live ? cell_ptr[c + 1] - v0 : 0, n = m * D;
  // the sweeping wavefront fetches its part of the in-cell solve first, so these
  // loads overlap the off-cell products
  const bool own = t < n;
  const int k = own ? t / D : 0, a = own ? t % D : 0;
  const int64_t xi = static_cast<int64_t>(v0 + k) * DP + a;
  T Mrow[NU];
  T bt = T(0), xc = T(0);
  if (threadIdx.x < 64) {
    const T* Mc = cellM + static_cast<int64_t>(c) * NU * NU;
#pragma unroll
    for (int u = 0; u < NU; ++u) Mrow[u] = (own && u < n) ? Mc[u * NU + t] : T(0);
    if (own) {
      bt = b[xi];
      if (MODE != 0) xc = x[xi];
    }
  }
  cell_offcell_sums<T, D, GR>(v0, m, L, U, x, true, MODE != 0, sh_lo[slot], sh_up[slot], t);
  if (threadIdx.x >= 64) return;          // wavefront 0 finishes the cell(s)
  const T s_t = own ? bt - sh_lo[slot][k][a] : T(0);
  const T sup = (own && MODE != 0) ? sh_up[slot][k][a] : T(0);
  if (MODE != 2 && s_save && own) s_save[xi] = s_t;
  T acc = s_t - sup;
  const T rdg = own_reciprocal<T, NU>(Mrow, t, own);
  // with one cell per wavefront n is uniform and the guards below are the loop
  // bounds; with several, every lane takes part in each broadcast
  if (MODE != 0) {
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      if (CPW > 1 || u < n) {
        const T xu = cell_bcast<CPW, CT>(xc, slot, u);
        if (u != t && u < n) acc -= Mrow[u] * xu;
      }
    }
  }
  if (MODE != 2) {
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      if (CPW > 1 || u < n) {
        T delta = T(0);
        if (t == u && u < n) {
          const T xn = acc * rdg;
          delta = xn - xc;
          xc = xn;
        }
        delta = cell_bcast<CPW, CT>(delta, slot, u);
        if (t != u && u < n) acc -= Mrow[u] * delta;
      }
    }
  } else {
#pragma unroll
    for (int u = NU - 1; u >= 0; --u) {
      if (CPW > 1 || u < n) {
        T delta = T(0);
        if (t == u && u < n) {
          const T xn = acc * rdg;
          delta = xn - xc;
          xc = xn;
        }
        delta = cell_bcast<CPW, CT>(delta, slot, u);
        if (t != u && u < n) acc -= Mrow[u] * delta;
      }
    }
  }
  if (own) x[xi] = xc;
}

// ---------------------------------------------------------------------------
// Colour-block levels (3D): cells are grouped into colour blocks of up to
// NB = 2^D cells (a colour is given to a block; the cells of a block are swept
// one after the other, in canonical order). A block's device rows are
// contiguous, its cells in canonical order. Besides L and U (blocks to earlier
// / later colours) a row has E and F: blocks to the earlier / later cells of
// its own colour block.
// One workgroup sweeps one colour block, wavefront w its cell w (GR = 64 / NV
// lanes per row):
//   phase A, all wavefronts at once: the products whose operand is final or
//     old for the whole sweep of this colour, from x in HBM before any cell of
//     the block is written: L (earlier colours: final) and, from a nonzero
//     guess, F and U (forward: later cells and colours still old) or E and U
//     (backward: earlier cells old, later colours new). Meanwhile the part the
//     cells need at their turn (forward: E, backward: F) is staged in LDS for
//     the whole block (it is contiguous in every plane), as is the block's x;
//   phase B, cell by cell in sweep order: the turn part's products with the
//     block's iterate in LDS, where the cells swept before hold their new
//     values, then the sequential sweep inside the cell (as k_gs_cell); the new
//     values go to LDS and HBM; a workgroup barrier closes each step.
// The forward sweeps save s = b - L x - E x (final values) for the residual.
// ---------------------------------------------------------------------------
template <int D>
struct BlockShape {
  static constexpr int NB = 1 << D;           // cells per colour block
  static constexpr int GR = 64 / (1 << D);    // lanes per row: one wavefront per cell
  static constexpr int threads = NB * 64;
};

// Entries of the turn part staged in LDS per colour block (a multiple of kQuad;
// entries beyond it are read from HBM at the turn).
template <typename T>
struct BlockStage {
  static constexpr int cap = sizeof(T) == 4 ? 1408 : 704;
};

// acc += products of the turn part's positions [kb, ke) (relative to the
// block's first entry; multiples of kQuad on cell levels) with the block's LDS
// iterate xs (device rows from r0); entries below `staged` come from the LDS
// stage (tcol, tval planes of stride CAP), the rest from the part in HBM.
template <typename T, int D, int G, int CAP>
__device__ __forceinline__ void block_turn_product(int kb, int ke, int lane, const Part<T>& P,
                                                   int base, int staged, const int* tcol,
                                                   const T* tval, const T* xs, int r0, T* acc) {
  constexpr int DP = Pad<D>::value;
  if constexpr (sizeof(T) == 4) {
    for (int q = kb / kQuad + lane; q < ke / kQuad; q += G) {
      const int e = q * kQuad;
      int4 j;
      T v[D * D][kQuad];
      if (e < staged) {
        j = *reinterpret_cast<const int4*>(tcol + e);
#pragma unroll
        for (int pl = 0; pl < D * D; ++pl) Quad<T>::load(tval + pl * CAP + e, v[pl]);
      } else {
        j = reinterpret_cast<const int4*>(P.col + base)[q];
#pragma unroll
        for (int pl = 0; pl < D * D; ++pl)
          Quad<T>::load(P.val + static_cast<int64_t>(pl) * P.nnz + base + e, v[pl]);
      }
      const int jj[kQuad] = {(j.x - r0) * DP, (j.y - r0) * DP, (j.z - r0) * DP, (j.w - r0) * DP};
#pragma unroll
      for (int a = 0; a < D; ++a) {
#pragma unroll
        for (int b = 0; b < D; ++b) {
          const T* vv = v[a * D + b];
          acc[a] += vv[0] * xs[jj[0] + b] + vv[1] * xs[jj[1] + b] + vv[2] * xs[jj[2] + b] +
                    vv[3] * xs[jj[3] + b];
        }
      }
    }
  } else {
    for (int e = kb + lane; e < ke; e += G) {
      const bool st = e < staged;
      const int j = ((st ? tcol[e] : P.col[base + e]) - r0) * DP;
#pragma unroll
      for (int a = 0; a < D; ++a) {
#pragma unroll
        for (int b = 0; b < D; ++b) {
          const int pl = a * D + b;
          const T v = st ? tval[pl * CAP + e] : P.val[static_cast<int64_t>(pl) * P.nnz + base + e];
          acc[a] += v * xs[j + b];
        }
      }
    }
  }
}

// Two workgroups per compute unit (4 waves per SIMD: at most 128 VGPRs).
template <typename T, int D, int MODE>
__global__ __launch_bounds__(BlockShape<D>::threads, 4) void k_gs_block(
    int blk0, const int* __restrict__ block_ptr, const int* __restrict__ cell_ptr, Part<T> L,
    Part<T> U, Part<T> E, Part<T> F, const T* __restrict__ cellM, const T* __restrict__ b, T* x,
    T* __restrict__ s_save) {
  constexpr int DP = Pad<D>::value, DD = D * D;
  constexpr int NV = CellShape<D>::NV, NU = CellShape<D>::NU;
  constexpr int NB = BlockShape<D>::NB, GR = BlockShape<D>::GR;
  constexpr int CAP = BlockStage<T>::cap;
  __shared__ __align__(16) T xs[NB * NV * DP];
  __shared__ __align__(16) int tcol[CAP];
  __shared__ __align__(16) T tval[DD * CAP];
  const Part<T>& TP = MODE == 2 ? F : E;   // the part taken at each cell's turn
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int bk = blk0 + xcd_block();
  const int cb = block_ptr[bk], nc = block_ptr[bk + 1] - cb;
  const int r0 = cell_ptr[cb], nrow = cell_ptr[cb + nc] - r0;
  // stage the block's turn part (contiguous in each plane, 16-byte aligned)
  const int tbase = TP.ptr[r0];
  const int staged = min(TP.ptr[r0 + nrow] - tbase, CAP);
  {
    constexpr int VW = 16 / sizeof(T);   // elements per 16-byte copy
    for (int e = threadIdx.x * 4; e < staged; e += blockDim.x * 4)
      *reinterpret_cast<int4*>(tcol + e) = *reinterpret_cast<const int4*>(TP.col + tbase + e);
    for (int pl = 0; pl < DD; ++pl) {
      const T* src = TP.val + static_cast<int64_t>(pl) * TP.nnz + tbase;
      for (int e = threadIdx.x * VW; e < staged; e += blockDim.x * VW)
        *reinterpret_cast<int4*>(tval + pl * CAP + e) = *reinterpret_cast<const int4*>(src + e);
    }
    for (int e = threadIdx.x; e < nrow * DP; e += blockDim.x)
      xs[e] = MODE != 0 ? x[static_cast<int64_t>(r0) * DP + e] : T(0);
  }
  // this wavefront's cell: the owned unknown t = lane (vertex t / D, component t % D)
  const bool has = w < nc;
  const int c = cb + (has ? w : 0);
  const int v0 = cell_ptr[c], m = has ? cell_ptr[c + 1] - v0 : 0, n = m * D;
  const int t = lane;
  const bool own = t < n;
  const int k = own ? t / D : 0, a = own ? t % D : 0;
  const int64_t xi = static_cast<int64_t>(v0 + k) * DP + a;
  T Mrow[NU];
  const T* Mc = cellM + static_cast<int64_t>(c) * NU * NU;
#pragma unroll
  for (int u = 0; u < NU; ++u) Mrow[u] = (own && u < n) ? Mc[u * NU + t] : T(0);
  const T bt = own ? b[xi] : T(0);
  T xc = (own && MODE != 0) ? x[xi] : T(0);
  // phase A (the turn part's row bounds are loaded now: at the turn only LDS is read)
  const int g = lane / GR, gl = lane % GR;
  const int tkb = g < m ? TP.ptr[v0 + g] - tbase : 0, tke = g < m ? TP.ptr[v0 + g + 1] - tbase : 0;
  T pa[D], pu[D];
#pragma unroll
  for (int q = 0; q < D; ++q) { pa[q] = T(0); pu[q] = T(0); }
  if (g < m) {
    const int i = v0 + g;
    part_quad_product<T, D, GR>(L, i, gl, x, pa);
    if (MODE == 1) {
      part_quad_product<T, D, GR>(F, i, gl, x, pu);
      part_quad_product<T, D, GR>(U, i, gl, x, pu);
    }
    if (MODE == 2) {
      part_quad_product<T, D, GR>(E, i, gl, x, pa);
      part_quad_product<T, D, GR>(U, i, gl, x, pa);
    }
  }
  T my_pa = T(0), my_pu = T(0);
#pragma unroll
  for (int q = 0; q < D; ++q) {   // every lane takes part in each shuffle
    const T s1 = __shfl(group_sum<T, GR>(pa[q]), k * GR, 64);
    const T s2 = MODE == 1 ? __shfl(group_sum<T, GR>(pu[q]), k * GR, 64) : T(0);
    if (q == a) { my_pa = s1; my_pu = s2; }
  }
  const T rdg = own_reciprocal<T, NU>(Mrow, t, own);
  __syncthreads();   // stage and block iterate in LDS
  // phase B: the cells in sweep order
  for (int step = 0; step < nc; ++step) {
    const int kk = MODE == 2 ? nc - 1 - step : step;
    if (w == kk) {
      T pt[D];
#pragma unroll
      for (int q = 0; q < D; ++q) pt[q] = T(0);
      if (g < m)
        block_turn_product<T, D, GR, CAP>(tkb, tke, gl, TP, tbase, staged, tcol, tval, xs, r0, pt);
      T my_pt = T(0);
#pragma unroll
      for (int q = 0; q < D; ++q) {
        const T s1 = __shfl(group_sum<T, GR>(pt[q]), k * GR, 64);
        if (q == a) my_pt = s1;
      }
      T acc;
      if (MODE != 2) {
        const T s_t = own ? bt - my_pa - my_pt : T(0);
        if (s_save && own) s_save[xi] = s_t;
        acc = s_t - my_pu;
      } else {
        acc = own ? bt - my_pa - my_pt : T(0);
      }
      if (MODE != 0) {
#pragma unroll
        for (int u = 0; u < NU; ++u) {
          if (u < n) {
            const T xu = bcast(xc, u);
            if (u != t) acc -= Mrow[u] * xu;
          }
        }
      }
#pragma unroll
      for (int uu = 0; uu < NU; ++uu) {
        const int u = MODE == 2 ? NU - 1 - uu : uu;
        if (u < n) {
          T delta = T(0);
          if (t == u) {
            const T xn = acc * rdg;
            delta = xn - xc;
            xc = xn;
          }
          delta = bcast(delta, u);
          if (t != u) acc -= Mrow[u] * delta;
        }
      }
      if (own) {
        xs[(v0 + k - r0) * DP + a] = xc;
        x[xi] = xc;
      }
    }
    __syncthreads();
  }
}

// out_t = base_t - (off-cell part)_t - (M x)_t on cell levels.
//   KIND 0: residual after a forward sweep: base = saved s, upper range only
//           (U, and F on colour-block levels: s holds b - L x - E x)
//   KIND 1: full residual: base = b, both ranges
//   KIND 2: SpMV: base = 0, both ranges, result negated (y = A x)
//   BLK: a colour-block level, E (with L) and F (with U) taken as well.
template <typename T, int D, int GR, int KIND, bool BLK>
__global__ __launch_bounds__((CellPack<D, GR>::threads)) void k_cell_apply(
    int ncell, const int* __restrict__ cell_ptr, Part<T> L, Part<T> U, Part<T> E, Part<T> F,
    const T* __restrict__ cellM, const T* __restrict__ base, const T* __restrict__ x,
    T* __restrict__ out, const int* __restrict__ done) {
  if (done && *done) return;
  constexpr int DP = Pad<D>::value;
  constexpr int NV = CellShape<D>::NV, NU = CellShape<D>::NU;
  constexpr int CT = CellPack<D, GR>::CT, CPW = CellPack<D, GR>::CPW;
  __shared__ T sh_lo[CPW][NV][D], sh_up[CPW][NV][D];
  const int slot = CPW == 1 ? 0 : threadIdx.x / CT;
  const int t = CPW == 1 ? threadIdx.x : threadIdx.x % CT;
  const int ci = xcd_block() * CPW + slot;
  const bool live = CPW == 1 || ci < ncell;
  const int c = live ? ci : 0;
  const int v0 = cell_ptr[c], m = live ? cell_ptr[c + 1] - v0 : 0, n = m * D;
  // wavefront 0 fetches the in-cell block row, x and the base first
  const bool own = t < n;
  const int k = own ? t / D : 0, a = own ? t % D : 0;
  const int64_t xi = static_cast<int64_t>(v0 + k) * DP + a;
  T Mrow[NU];
  T xt = T(0), bt = T(0);
  if (threadIdx.x < 64) {
    const T* Mc = cellM + static_cast<int64_t>(c) * NU * NU;
#pragma unroll
    for (int u = 0; u < NU; ++u) Mrow[u] = (own && u < n) ? Mc[u * NU + t] : T(0);
    if (own) {
      xt = x[xi];
      if (KIND != 2) bt = base[xi];
    }
  }
  cell_offcell_sums<T, D, GR>(v0, m, L, U, x, KIND != 0, true, sh_lo[slot], sh_up[slot], t,
                              BLK ? &E : nullptr, BLK ? &F : nullptr);
  if (threadIdx.x >= 64) return;
  const T off = own ? (KIND != 0 ? sh_lo[slot][k][a] : T(0)) + sh_up[slot][k][a] : T(0);
  T mx = T(0);
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    if (CPW > 1 || u < n) {
      const T xu = cell_bcast<CPW, CT>(xt, slot, u);
      if (u < n) mx += Mrow[u] * xu;
    }
  }
  if (!own) return;
  if (KIND == 2)
    out[xi] = off + mx;
  else
    out[xi] = bt - off - mx;
}

// ---------------------------------------------------------------------------
// Damped vertex-block Jacobi step: x = omega D^{-1} v (FIRST, from a zero guess,
// v = b) or x += omega D^{-1} v (v = the residual b - A x).
// ---------------------------------------------------------------------------
template <typename T, int D, bool FIRST>
__global__ __launch_bounds__(kBlock) void k_jacobi_step(int n, const T* __restrict__ dinv, T omega,
                                                        const T* __restrict__ v, T* __restrict__ x,
                                                        const int* __restrict__ done) {
  if (done && *done) return;
  constexpr int DP = Pad<D>::value;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  T vi[D], xi[D];
  VecIO<T, D>::load(v + static_cast<int64_t>(i) * DP, vi);
  if (!FIRST) VecIO<T, D>::load(x + static_cast<int64_t>(i) * DP, xi);
  const T* Di = dinv + static_cast<int64_t>(i) * D * D;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    T t = T(0);
#pragma unroll
    for (int b = 0; b < D; ++b) t += Di[a * D + b] * vi[b];
    xi[a] = FIRST ? omega * t : xi[a] + omega * t;
  }
  VecIO<T, D>::store(x + static_cast<int64_t>(i) * DP, xi);
}

// ---------------------------------------------------------------------------
// K4: restriction b_c = P^T r (gather over the CSR of P^T); K5: x += P e.
// ---------------------------------------------------------------------------
// Both transfers are gathers over a scalar CSR (weights shared by the
// components); GT lanes share a row so its entries are loaded together.
template <typename T, int D, int GT>
__device__ __forceinline__ void transfer_row(int pb, int pe, int lane, const int* __restrict__ idx,
                                             const T* __restrict__ w, const T* __restrict__ v,
                                             T* acc) {
  constexpr int DP = Pad<D>::value;
  for (int p = pb + lane; p < pe; p += GT) {
    T e[D];
    VecIO<T, D>::load(v + static_cast<int64_t>(idx[p]) * DP, e);
    const T wp = w[p];
#pragma unroll
    for (int a = 0; a < D; ++a) acc[a] += wp * e[a];
  }
#pragma unroll
  for (int a = 0; a < D; ++a) acc[a] = group_sum<T, GT>(acc[a]);
}

template <typename T, int D, int GT>
__global__ __launch_bounds__(kBlock) void k_restrict(int nc, const int* __restrict__ ptr,
                                                     const int* __restrict__ idx,
                                                     const T* __restrict__ w,
                                                     const T* __restrict__ r, T* __restrict__ bc,
                                                     const int* __restrict__ done) {
  if (done && *done) return;
  constexpr int DP = Pad<D>::value;
  const int lane = threadIdx.x % GT;
  const int I = xcd_block() * (kBlock / GT) + threadIdx.x / GT;
  if (I >= nc) return;
  T acc[D];
#pragma unroll
  for (int a = 0; a < D; ++a) acc[a] = T(0);
  transfer_row<T, D, GT>(ptr[I], ptr[I + 1], lane, idx, w, r, acc);
  if (lane == 0) VecIO<T, D>::store(bc + static_cast<int64_t>(I) * DP, acc);
}

// fixed (optional): constrained components of the fine rows, whose
// prolongation rows are zero.
template <typename T, int D, int GT>
__global__ __launch_bounds__(kBlock) void k_prolong_add(int nf, const int* __restrict__ ptr,
                                                        const int* __restrict__ idx,
                                                        const T* __restrict__ w,
                                                        const T* __restrict__ e, T* x,
                                                        const uint8_t* __restrict__ fixed,
                                                        const int* __restrict__ done) {
  if (done && *done) return;
  constexpr int DP = Pad<D>::value;
  const int lane = threadIdx.x % GT;
  const int i = xcd_block() * (kBlock / GT) + threadIdx.x / GT;
  if (i >= nf) return;
  T xi[D];
  if (lane == 0) VecIO<T, D>::load(x + static_cast<int64_t>(i) * DP, xi);
  T acc[D];
#pragma unroll
  for (int a = 0; a < D; ++a) acc[a] = T(0);
  transfer_row<T, D, GT>(ptr[i], ptr[i + 1], lane, idx, w, e, acc);
  if (lane == 0) {
    const int fx = fixed ? fixed[i] : 0;
#pragma unroll
    for (int a = 0; a < D; ++a) xi[a] += ((fx >> a) & 1) ? T(0) : acc[a];
    VecIO<T, D>::store(x + static_cast<int64_t>(i) * DP, xi);
  }
}

// ---------------------------------------------------------------------------
// K6: coarsest solve L L^T e = b in FP64 (one workgroup; n <= kCoarseMax).
// ---------------------------------------------------------------------------
constexpr int kCoarseMax = 4096;

template <typename T, int D>
__global__ __launch_bounds__(kBlock) void k_coarse_solve(int n, const double* __restrict__ L,
                                                         const T* __restrict__ b, T* __restrict__ x,
                                                         const int* __restrict__ done) {
  if (done && *done) return;
  constexpr int DP = Pad<D>::value;
  __shared__ double y[kCoarseMax];
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    y[i] = static_cast<double>(b[(i / D) * DP + (i % D)]);
  __syncthreads();
  for (int j = 0; j < n; ++j) {           // L y = b, column by column
    if (threadIdx.x == 0) y[j] /= L[static_cast<int64_t>(j) * n + j];
    __syncthreads();
    const double yj = y[j];
    for (int i = j + 1 + threadIdx.x; i < n; i += blockDim.x)
      y[i] -= L[static_cast<int64_t>(i) * n + j] * yj;
    __syncthreads();
  }
  for (int j = n - 1; j >= 0; --j) {      // L^T x = y
    if (threadIdx.x == 0) y[j] /= L[static_cast<int64_t>(j) * n + j];
    __syncthreads();
    const double yj = y[j];
    for (int i = threadIdx.x; i < j; i += blockDim.x)
      y[i] -= L[static_cast<int64_t>(j) * n + i] * yj;
    __syncthreads();
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) x[(i / D) * DP + (i % D)] = static_cast<T>(y[i]);
}

// K6, small coarsest levels (n <= kCoarseInvMax): x = A_c^{-1} b with the inverse
// formed at setup from the same Cholesky factor; one pass instead of 2n
// dependent steps. Row i is one thread's sum in ascending column order.
constexpr int kCoarseInvMax = 256;
template <typename T, int D>
__global__ __launch_bounds__(kBlock) void k_coarse_apply(int n, const double* __restrict__ Minv,
                                                         const T* __restrict__ b, T* __restrict__ x,
                                                         const int* __restrict__ done) {
  if (done && *done) return;
  constexpr int DP = Pad<D>::value;
  __shared__ double y[kCoarseInvMax];
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    y[i] = static_cast<double>(b[(i / D) * DP + (i % D)]);
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double* row = Minv + static_cast<int64_t>(i) * n;
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += row[j] * y[j];
    x[(i / D) * DP + (i % D)] = static_cast<T>(s);
  }
}

// ---------------------------------------------------------------------------
// The bottom of the cycle in one workgroup: the last few cell levels above a
// small coarsest level (smoothing, residual, restriction, prolongation) and the
// coarsest solve by the inverse, which would otherwise take 2 x colours + 3
// launches per level, each too small to fill the chip. The levels' vectors
// live in LDS; each wavefront updates one cell of the current colour (GR =
// 64 / 2^d lanes per row) with the arithmetic of k_gs_cell / k_cell_apply, and
// colours and phases are separated by workgroup barriers. Several levels are
// fused only for the V-cycle (one visit per level); the first level may start
// from a nonzero iterate (second visit of a W-cycle).
// ---------------------------------------------------------------------------
constexpr int kBottomThreads = 512;
constexpr int kBottomLevels = 4;
constexpr int kBottomLds = 56 * 1024;   // dynamic LDS: the levels' vectors and pointer copies

// Pointers that k_bottom reads from its level table (device memory, not kernel
// arguments) are generic to the compiler, which then emits flat loads: counted
// against both the memory and the LDS wait counters, so LDS reads also wait for
// the matrix loads in flight. Its matrix loads go through pointers in the global
// address space instead.
template <typename T>
using gptr = const __attribute__((address_space(1))) T*;
typedef int gint4 __attribute__((ext_vector_type(4)));
typedef float gfloat4 __attribute__((ext_vector_type(4)));
template <typename T>
__device__ __forceinline__ gptr<T> to_global(const T* p) {
  return (gptr<T>)p;
}

template <typename T>
struct BottomLevel {
  int n = 0, ncolors = 0, ncells = 0, nnext = 0;
  const int* color_ptr = nullptr;   // cells of each colour, [ncolors + 1]
  const int* cell_ptr = nullptr;
  Part<T> L{}, U{};
  const T* cellM = nullptr;
  const int *p_ptr = nullptr, *p_idx = nullptr;
  const T* p_w = nullptr;
  const int *pt_ptr = nullptr, *pt_idx = nullptr;
  const T* pt_w = nullptr;
  const uint8_t* fixed = nullptr;   // constrained components (zero prolongation rows), or null
};

template <typename T>
struct BottomArgs {
  int nlev = 0, ncoarse = 0;
  int npre = 1, npost = 1, zero_guess = 1;
  const BottomLevel<T>* lev = nullptr;   // device array [nlev]
  const double* Minv = nullptr;
  const T* b = nullptr;   // first fused level's right-hand side (in)
  T* x = nullptr;         // first fused level's iterate (in unless zero_guess, out)
};

// One level in LDS: right-hand side, iterate, saved s, residual, and copies of
// the colour, cell and row pointers (the sweeps' dependent index loads).
template <typename T>
struct BottomVecs {
  T *b, *x, *s, *r;
  int *color_ptr, *cell_ptr, *Lptr, *Uptr;
};

// LDS elements of one level: four padded vectors (T) and its pointers (int).
__host__ __device__ inline int bottom_vec_elems(int n, int dp) { return 4 * n * dp; }
__host__ __device__ inline int bottom_int_elems(int n, int ncolors, int ncells) {
  return (ncolors + 1) + (ncells + 1) + 2 * (n + 1);
}

// acc += the products of positions [kb, ke) of one part with the LDS iterate x:
// quads of 4 blocks (FP32, one 16-byte load per plane) or single blocks (FP64),
// loaded through global-address-space pointers.
template <typename T, int D, int G>
__device__ __forceinline__ void bottom_part(int kb, int ke, int lane, const int* col, const T* val,
                                            int64_t nnz, const T* x, T* acc) {
  constexpr int DP = Pad<D>::value;
  const gptr<int> gc = to_global(col);
  const gptr<T> gv = to_global(val);
  if constexpr (sizeof(T) == 4) {
    for (int q = kb / kQuad + lane; q < ke / kQuad; q += G) {
      const gint4 j = *reinterpret_cast<gptr<gint4>>(gc + q * kQuad);
      const int jj[kQuad] = {j.x, j.y, j.z, j.w};
#pragma unroll
      for (int a = 0; a < D; ++a) {
#pragma unroll
        for (int b = 0; b < D; ++b) {
          const gfloat4 v = *reinterpret_cast<gptr<gfloat4>>(
              gv + static_cast<int64_t>(a * D + b) * nnz + static_cast<int64_t>(q) * kQuad);
          acc[a] += v.x * x[jj[0] * DP + b] + v.y * x[jj[1] * DP + b] + v.z * x[jj[2] * DP + b] +
                    v.w * x[jj[3] * DP + b];
        }
      }
    }
  } else {
    for (int k = kb + lane; k < ke; k += G) {
      const int j = gc[k];
#pragma unroll
      for (int a = 0; a < D; ++a) {
#pragma unroll
        for (int b = 0; b < D; ++b) acc[a] += gv[static_cast<int64_t>(a * D + b) * nnz + k] * x[j * DP + b];
      }
    }
  }
}

// One cell by one wavefront (MODE as k_gs_cell: 0 zero-guess forward, 1 forward,
// 2 backward); RES: compute r = s - U x - M x instead of a sweep.
template <typename T, int D, int MODE, bool RES>
__device__ __forceinline__ void bottom_cell(const BottomLevel<T>& lv, int c, const BottomVecs<T>& v) {
  constexpr int DP = Pad<D>::value;
  constexpr int NV = CellShape<D>::NV, NU = CellShape<D>::NU;
  constexpr int GR = 64 / NV;
  const int lane = threadIdx.x & 63;
  const int v0 = v.cell_ptr[c], m = v.cell_ptr[c + 1] - v0, n = m * D;
  // the in-cell block row first, so its loads overlap the off-cell products
  const int t = lane;
  const bool own = t < n;
  const int k = own ? t / D : 0, comp = own ? t % D : 0;
  T Mrow[NU];
  const gptr<T> Mc = to_global(lv.cellM) + static_cast<int64_t>(c) * NU * NU;
#pragma unroll
  for (int u = 0; u < NU; ++u) Mrow[u] = (own && u < n) ? Mc[u * NU + t] : T(0);
  const int g = lane / GR, gl = lane % GR;
  T lo[D], up[D];
#pragma unroll
  for (int q = 0; q < D; ++q) { lo[q] = T(0); up[q] = T(0); }
  const bool want_lo = !RES, want_up = RES || MODE != 0;
  if (g < m) {
    const int i = v0 + g;
    if (want_lo) bottom_part<T, D, GR>(v.Lptr[i], v.Lptr[i + 1], gl, lv.L.col, lv.L.val, lv.L.nnz, v.x, lo);
    if (want_up) bottom_part<T, D, GR>(v.Uptr[i], v.Uptr[i + 1], gl, lv.U.col, lv.U.val, lv.U.nnz, v.x, up);
  }
#pragma unroll
  for (int q = 0; q < D; ++q) {
    lo[q] = group_sum<T, GR>(lo[q]);
    up[q] = group_sum<T, GR>(up[q]);
  }
  T my_lo = T(0), my_up = T(0);
#pragma unroll
  for (int q = 0; q < D; ++q) {   // every lane takes part in each shuffle
    const T l1 = __shfl(lo[q], k * GR, 64), u1 = __shfl(up[q], k * GR, 64);
    if (q == comp) { my_lo = l1; my_up = u1; }
  }
  const int xi = (v0 + k) * DP + comp;
  T xc = (own && (MODE != 0 || RES)) ? v.x[xi] : T(0);
  if (RES) {
    T mx = T(0);
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      if (u < n) mx += Mrow[u] * bcast(xc, u);
    }
    if (own) v.r[xi] = v.s[xi] - my_up - mx;
    return;
  }
  const T s_t = own ? v.b[xi] - my_lo : T(0);
  if (MODE != 2 && own) v.s[xi] = s_t;
  T acc = s_t - (MODE != 0 ? my_up : T(0));
  const T rdg = own_reciprocal<T, NU>(Mrow, t, own);
  if (MODE != 0) {
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      if (u < n) {
        const T xu = bcast(xc, u);
        if (u != t) acc -= Mrow[u] * xu;
      }
    }
  }
#pragma unroll
  for (int uu = 0; uu < NU; ++uu) {
    const int u = MODE == 2 ? NU - 1 - uu : uu;
    if (u < n) {
      T delta = T(0);
      if (t == u) {
        const T xn = acc * rdg;
        delta = xn - xc;
        xc = xn;
      }
      delta = bcast(delta, u);
      if (t != u) acc -= Mrow[u] * delta;
    }
  }
  if (own) v.x[xi] = xc;
}

template <typename T, int D, int MODE>
__device__ __forceinline__ void bottom_sweep(const BottomLevel<T>& lv, const BottomVecs<T>& v) {
  const int w = threadIdx.x >> 6, nw = kBottomThreads / 64;
  for (int q = 0; q < lv.ncolors; ++q) {
    const int col = MODE == 2 ? lv.ncolors - 1 - q : q;
    for (int c = v.color_ptr[col] + w; c < v.color_ptr[col + 1]; c += nw)
      bottom_cell<T, D, MODE, false>(lv, c, v);
    __syncthreads();
  }
}

// Gather over a scalar CSR (rows [0, nrows), weights shared by the components)
// from the padded vector src into dst (ADD: dst += ...).
template <typename T, int D, bool ADD, typename TD>
__device__ __forceinline__ void bottom_transfer(int nrows, const int* ptr, const int* idx,
                                                const T* w, const T* src, int sstride, TD* dst,
                                                int dstride, const uint8_t* fixed = nullptr) {
  for (int i = threadIdx.x; i < nrows; i += blockDim.x) {
    T acc[D];
#pragma unroll
    for (int q = 0; q < D; ++q) acc[q] = T(0);
    for (int p = ptr[i]; p < ptr[i + 1]; ++p) {
      const T wp = w[p];
      const T* e = src + idx[p] * sstride;
#pragma unroll
      for (int q = 0; q < D; ++q) acc[q] += wp * e[q];
    }
    const int fx = (ADD && fixed) ? fixed[i] : 0;
#pragma unroll
    for (int q = 0; q < D; ++q) {
      if (ADD)
        dst[i * dstride + q] += ((fx >> q) & 1) ? T(0) : acc[q];
      else
        dst[i * dstride + q] = static_cast<TD>(acc[q]);
    }
  }
}

template <typename T, int D>
__global__ __launch_bounds__(kBottomThreads) void k_bottom(BottomArgs<T> a,
                                                           const int* __restrict__ done) {
  if (done && *done) return;
  constexpr int DP = Pad<D>::value;
  extern __shared__ __align__(16) unsigned char bottom_smem[];
  __shared__ double cy[kCoarseInvMax];
  __shared__ T cx[kCoarseInvMax];
  // LDS: every level's vectors (T), then every level's pointers (int)
  T* base = reinterpret_cast<T*>(bottom_smem);
  int total = 0;
  for (int j = 0; j < a.nlev; ++j) total += bottom_vec_elems(a.lev[j].n, DP);
  int* ibase = reinterpret_cast<int*>(base + total);
  auto vecs = [&](int k) {   // level k's LDS arrays
    int off = 0, ioff = 0;
    for (int j = 0; j < k; ++j) {
      off += bottom_vec_elems(a.lev[j].n, DP);
      ioff += bottom_int_elems(a.lev[j].n, a.lev[j].ncolors, a.lev[j].ncells);
    }
    const BottomLevel<T>& lv = a.lev[k];
    const int len = lv.n * DP;
    int* cp = ibase + ioff;
    int* cl = cp + lv.ncolors + 1;
    int* lp = cl + lv.ncells + 1;
    return BottomVecs<T>{base + off, base + off + len, base + off + 2 * len, base + off + 3 * len,
                         cp, cl, lp, lp + lv.n + 1};
  };
  // zero vectors, pointer copies; first level: b and (second W-cycle visit) x
  // from HBM; deeper levels start at zero
  {
    for (int e = threadIdx.x; e < total; e += blockDim.x) base[e] = T(0);
    for (int k = 0; k < a.nlev; ++k) {
      const BottomLevel<T>& lv = a.lev[k];
      const BottomVecs<T> v = vecs(k);
      for (int e = threadIdx.x; e <= lv.ncolors; e += blockDim.x) v.color_ptr[e] = lv.color_ptr[e];
      for (int e = threadIdx.x; e <= lv.ncells; e += blockDim.x) v.cell_ptr[e] = lv.cell_ptr[e];
      for (int e = threadIdx.x; e <= lv.n; e += blockDim.x) {
        v.Lptr[e] = lv.L.ptr[e];
        v.Uptr[e] = lv.U.ptr[e];
      }
    }
    __syncthreads();
    const BottomVecs<T> v = vecs(0);
    const int len = a.lev[0].n * DP;
    for (int e = threadIdx.x; e < len; e += blockDim.x) {
      v.b[e] = a.b[e];
      if (!a.zero_guess) v.x[e] = a.x[e];
    }
    __syncthreads();
  }
  // down: pre-smoothing, residual r = s - U x - M x, restriction
  for (int k = 0; k < a.nlev; ++k) {
    const BottomLevel<T>& lv = a.lev[k];
    const BottomVecs<T> v = vecs(k);
    for (int it = 0; it < a.npre; ++it) {
      if (it == 0 && (k > 0 || a.zero_guess))
        bottom_sweep<T, D, 0>(lv, v);
      else
        bottom_sweep<T, D, 1>(lv, v);
    }
    const int w = threadIdx.x >> 6, nw = kBottomThreads / 64;
    for (int c = w; c < lv.ncells; c += nw) bottom_cell<T, D, 1, true>(lv, c, v);
    __syncthreads();
    if (k + 1 < a.nlev)
      bottom_transfer<T, D, false, T>(lv.nnext, lv.pt_ptr, lv.pt_idx, lv.pt_w, v.r, DP, vecs(k + 1).b, DP);
    else   // the coarsest right-hand side, rounded to T as in the level vectors
      bottom_transfer<T, D, false, double>(lv.nnext, lv.pt_ptr, lv.pt_idx, lv.pt_w, v.r, DP, cy, D);
    __syncthreads();
  }
  // coarsest: x = A_c^{-1} b, rows in ascending column order (FP64)
  for (int i = threadIdx.x; i < a.ncoarse; i += blockDim.x) {
    const gptr<double> row = to_global(a.Minv) + static_cast<int64_t>(i) * a.ncoarse;
    double s = 0.0;
    for (int j = 0; j < a.ncoarse; ++j) s += row[j] * cy[j];
    cx[i] = static_cast<T>(s);
  }
  __syncthreads();
  // up: prolongation x += P e, post-smoothing
  for (int k = a.nlev - 1; k >= 0; --k) {
    const BottomLevel<T>& lv = a.lev[k];
    const BottomVecs<T> v = vecs(k);
    if (k + 1 < a.nlev)
      bottom_transfer<T, D, true, T>(lv.n, lv.p_ptr, lv.p_idx, lv.p_w, vecs(k + 1).x, DP, v.x, DP,
                                     lv.fixed);
    else
      bottom_transfer<T, D, true, T>(lv.n, lv.p_ptr, lv.p_idx, lv.p_w, cx, D, v.x, DP, lv.fixed);
    __syncthreads();
    for (int it = 0; it < a.npost; ++it) bottom_sweep<T, D, 2>(lv, v);
  }
  const BottomVecs<T> v = vecs(0);
  for (int e = threadIdx.x; e < a.lev[0].n * DP; e += blockDim.x) a.x[e] = v.x[e];
}

// ---------------------------------------------------------------------------
// K7/K8: PCG vector kernels and device-side scalars (FP64, deterministic).
// ---------------------------------------------------------------------------
struct Scalars {
  double rho;       // r^T z of the current direction
  double pq;        // p^T A p
  double alpha, beta;
  double res;       // ||r||
  double normF;     // ||F||
  double rtol;
  double res_true;  // ||F - A x||
  int done;         // 1 = stop (converged or breakdown)
  int status;       // 0 running/converged, 5 breakdown
  int first;        // next beta finalisation is the first one
  int iters;        // products A p so far
};

enum FinMode { FIN_NORMF = 0, FIN_ALPHA = 1, FIN_RES = 2, FIN_BETA = 3, FIN_TRUE = 4 };

// Scalar steps of Algorithm 2 from a finished reduction `tot`.
template <int MODE>
__device__ __forceinline__ void finalize_scalar(double tot, Scalars* s) {
  if (MODE == FIN_NORMF) {
    s->normF = sqrt(tot);
    s->res = s->normF;
    s->done = 0;
    s->status = 0;
    s->first = 1;
    s->iters = 0;
    s->alpha = s->beta = 0.0;
  } else if (MODE == FIN_ALPHA) {
    s->pq = tot;
    if (!(tot > 0.0) || !isfinite(tot)) {
      s->status = 5;
      s->done = 1;
    } else {
      s->alpha = s->rho / tot;
    }
  } else if (MODE == FIN_RES) {
    s->res = sqrt(tot);
    s->iters += 1;
    if (!isfinite(s->res)) {
      s->status = 5;
      s->done = 1;
    } else if (s->res / s->normF < s->rtol) {
      s->done = 1;
    }
  } else if (MODE == FIN_BETA) {
    if (s->first) {
      s->beta = 0.0;
      s->first = 0;
    } else {
      s->beta = tot / s->rho;
    }
    s->rho = tot;
    if (!isfinite(tot)) {
      s->status = 5;
      s->done = 1;
    }
  } else {
    s->res_true = sqrt(tot);
  }
}

template <int MODE>
__global__ __launch_bounds__(1024) void k_finalize(const double* __restrict__ partial, int np,
                                                   Scalars* s) {
  __shared__ double sh[1024];
  if (MODE != FIN_NORMF && MODE != FIN_TRUE && s->done) return;
  double v = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) v += partial[i];
  const double tot = block_sum(v, sh);
  if (threadIdx.x == 0) finalize_scalar<MODE>(tot, s);
}

// partial sums of a.b over a flat vector (grid-stride, fixed grid)
template <typename TB>
__global__ __launch_bounds__(kBlock) void k_dot(int64_t n, const double* __restrict__ a,
                                                const TB* __restrict__ b,
                                                double* __restrict__ partial,
                                                const int* __restrict__ done) {
  if (done && *done) return;
  __shared__ double sh[kBlock];
  double v = 0.0;
  for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kBlock)
    v += a[i] * static_cast<double>(b[i]);
  const double s = block_sum(v, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// x += alpha p; r -= alpha q; partial ||r||^2; b0 = (T) r (V-cycle input)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_update_xr(int64_t n, const Scalars* __restrict__ s,
                                                      const double* __restrict__ p,
                                                      const double* __restrict__ q,
                                                      double* __restrict__ x,
                                                      double* __restrict__ r, T* __restrict__ b0,
                                                      double* __restrict__ partial) {
  __shared__ double sh[kBlock];
  if (s->done) return;
  const double alpha = s->alpha;
  double v = 0.0;
  for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kBlock) {
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    if (b0) b0[i] = static_cast<T>(ri);
    v += ri * ri;
  }
  const double t = block_sum(v, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// p = z + beta p with z = (double) the V-cycle output
template <typename T>
__global__ __launch_bounds__(kBlock) void k_update_p(int64_t n, const Scalars* __restrict__ s,
                                                     const T* __restrict__ z,
                                                     double* __restrict__ p) {
  if (s->done) return;
  const double beta = s->beta;
  for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kBlock)
    p[i] = static_cast<double>(z[i]) + beta * p[i];
}

// point Jacobi z = r / a_ii (a context preconditioner, not the paper's)
template <int D>
__global__ __launch_bounds__(kBlock) void k_jacobi(int n, const double* __restrict__ diag,
                                                   const double* __restrict__ r,
                                                   double* __restrict__ z,
                                                   const int* __restrict__ done) {
  if (done && *done) return;
  constexpr int DP = Pad<D>::value;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
#pragma unroll
  for (int a = 0; a < D; ++a)
    z[static_cast<int64_t>(i) * DP + a] =
        r[static_cast<int64_t>(i) * DP + a] / diag[static_cast<int64_t>(i) * D * D + a * D + a];
}

// flat conversions and fills
template <typename TA, typename TB>
__global__ __launch_bounds__(kBlock) void k_convert(int64_t n, const TA* __restrict__ a,
                                                    TB* __restrict__ b) {
  for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kBlock)
    b[i] = static_cast<TB>(a[i]);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(int64_t n, T* __restrict__ a, T v) {
  for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kBlock)
    a[i] = v;
}

// r = F - q (flat), partial ||r||^2
__global__ __launch_bounds__(kBlock) void k_sub_norm(int64_t n, const double* __restrict__ F,
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
  const double t = block_sum(v, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// user layout [nv][D] <-> device numbering (padded) through a vertex map
// fixed (optional): constrained components of the rows, read as 0.
template <typename TS, typename TD, int D>
__global__ __launch_bounds__(kBlock) void k_gather_user(int n, const int* __restrict__ map,
                                                        const TS* __restrict__ src,
                                                        TD* __restrict__ dst,
                                                        const uint8_t* __restrict__ fixed) {
  constexpr int DP = Pad<D>::value;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int64_t v = map[i];
  const int fx = fixed ? fixed[i] : 0;
#pragma unroll
  for (int a = 0; a < DP; ++a)
    dst[static_cast<int64_t>(i) * DP + a] =
        (a < D && !((fx >> a) & 1)) ? static_cast<TD>(src[v * D + a]) : TD(0);
}

template <typename TS, typename TD, int D>
__global__ __launch_bounds__(kBlock) void k_scatter_user(int n, const int* __restrict__ map,
                                                         const TS* __restrict__ src,
                                                         TD* __restrict__ dst) {
  constexpr int DP = Pad<D>::value;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int64_t v = map[i];
#pragma unroll
  for (int a = 0; a < D; ++a) dst[v * D + a] = static_cast<TD>(src[static_cast<int64_t>(i) * DP + a]);
}

}  // namespace dev
}  // namespace vasmg
