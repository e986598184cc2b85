// Packed solves: several independent problems in one block-diagonal hierarchy,
// each with its own PCG recurrence (Section 2.2, Algorithm 2): its own dot
// products, alpha, beta and stopping test, so every problem runs the iteration
// it would run alone (to rounding) while the V-cycle and the SpMV launches are
// shared. A problem is a segment of the fine level: seg_rows[seg_ptr[s] ..
// seg_ptr[s + 1]) are its device rows, ascending; seg_of_row maps a row back.
// Included by vasmg.hip (uses kBlock, block_sum, Scalars, finalize_scalar).
#pragma once

namespace vasmg {
namespace dev {

// One workgroup per segment: the segment's dot product over its rows (DP
// entries each; DIFF: of a - b with itself), summed in a fixed order, then the
// scalar step MODE of Algorithm 2 on the segment's own scalars. A finished
// segment is skipped except for the norms of the right-hand side and the true
// residual.
template <int MODE, bool DIFF, typename TB>
__global__ __launch_bounds__(kBlock) void k_seg_dot(const int* __restrict__ seg_ptr,
                                                    const int* __restrict__ seg_rows, int DP,
                                                    const double* __restrict__ a,
                                                    const TB* __restrict__ b, Scalars* __restrict__ ss) {
  __shared__ double sh[kBlock];
  const int s = blockIdx.x;
  if (MODE != FIN_NORMF && MODE != FIN_TRUE && ss[s].done) return;
  const int lo = seg_ptr[s], hi = seg_ptr[s + 1];
  double v = 0.0;
  for (int64_t q = static_cast<int64_t>(lo) * DP + threadIdx.x; q < static_cast<int64_t>(hi) * DP;
       q += kBlock) {
    const int64_t i = static_cast<int64_t>(seg_rows[q / DP]) * DP + q % DP;
    if (DIFF) {
      const double t = a[i] - static_cast<double>(b[i]);
      v += t * t;
    } else {
      v += a[i] * static_cast<double>(b[i]);
    }
  }
  const double tot = block_sum(v, sh);
  if (threadIdx.x == 0) finalize_scalar<MODE>(tot, &ss[s]);
}

// After ||F||: rtol, and segments with nothing to solve (F = 0, or not finite:
// breakdown) finish at once.
__global__ void k_seg_start(int nseg, Scalars* __restrict__ ss, double rtol) {
  const int s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= nseg) return;
  ss[s].rtol = rtol;
  const double f = ss[s].normF;
  if (!isfinite(f)) {
    ss[s].status = 5;
    ss[s].done = 1;
  } else if (f == 0.0) {
    ss[s].done = 1;
  }
}

// x += alpha_s p; r -= alpha_s q; b0 = (T) r for the rows of running segments
template <typename T>
__global__ __launch_bounds__(kBlock) void k_seg_update_xr(int64_t n, int DP, const int* __restrict__ seg_of_row,
                                                          const Scalars* __restrict__ ss,
                                                          const double* __restrict__ p,
                                                          const double* __restrict__ q,
                                                          double* __restrict__ x, double* __restrict__ r,
                                                          T* __restrict__ b0) {
  for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock) {
    const Scalars& s = ss[seg_of_row[i / DP]];
    if (s.done) continue;
    const double alpha = s.alpha;
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    if (b0) b0[i] = static_cast<T>(ri);
  }
}

// p = z + beta_s p for the rows of running segments
template <typename T>
__global__ __launch_bounds__(kBlock) void k_seg_update_p(int64_t n, int DP, const int* __restrict__ seg_of_row,
                                                         const Scalars* __restrict__ ss,
                                                         const T* __restrict__ z, double* __restrict__ p) {
  for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock) {
    const Scalars& s = ss[seg_of_row[i / DP]];
    if (s.done) continue;
    p[i] = static_cast<double>(z[i]) + s.beta * p[i];
  }
}

// number of segments still running (one workgroup)
__global__ __launch_bounds__(kBlock) void k_seg_running(int nseg, const Scalars* __restrict__ ss,
                                                        int* __restrict__ running) {
  __shared__ double sh[kBlock];
  double v = 0.0;
  for (int s = threadIdx.x; s < nseg; s += kBlock) v += ss[s].done ? 0.0 : 1.0;
  const double tot = block_sum(v, sh);
  if (threadIdx.x == 0) *running = static_cast<int>(tot);
}

}  // namespace dev
}  // namespace vasmg
