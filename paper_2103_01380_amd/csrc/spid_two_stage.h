// spid_two_stage.h -- device kernels of the modified (two-stage) ID
// (arXiv 2103.01380, Section 3.4.2).  Stage 1 runs the ordinary selection
// and coefficient kernels on temporal windows of every block (a window is a
// column range of the block's sketch); stage 2 runs them on the sketch of the
// concatenated window skeletons, which these kernels gather from the
// resident sketch (the sketch matrix is the same for every column, so no
// pass over A is needed); the last kernel maps the stage-2 pivots back to
// columns of A and forms the coefficients C^1 C^{0'}.
//
// Window w of a block with n columns holds columns [c_w, c_{w+1}),
// c_w = floor(w n / nwin).  Stage-2 slot w * k1 + t holds the t-th stage-1
// pivot of window w; slots past a window's pivot count are zero columns
// (never selected, and they change no other column's projections).
#pragma once

#include "spid_kernels.h"

namespace spid {

__device__ __forceinline__ int ts_window_start(int w, int n, int nwin) {
  return (int)(((int64_t)w * n) / nwin);
}

// window holding column j
__device__ __forceinline__ int ts_window_of(int j, int n, int nwin) {
  int w = (int)(((int64_t)j * nwin) / n);
  while (w > 0 && ts_window_start(w, n, nwin) > j) --w;
  while (w + 1 < nwin && ts_window_start(w + 1, n, nwin) <= j) ++w;
  return w;
}

// Stage-2 sketch: Y2_b(:, w k1 + t) = Y_b(:, c_w + S1_{b,w}[t]) for t < k1_{b,w},
// zero otherwise.  Grid: x covers nwin * k1 * l entries, y strides over blocks.
template <typename TY>
__global__ __launch_bounds__(256) void ts_gather_kernel(
    const BlkInfo* __restrict__ win, const BlkInfo* __restrict__ blk2, int nblocks, int nwin,
    int k1, int l, const int32_t* __restrict__ S1, const int32_t* __restrict__ k1w,
    const TY* __restrict__ Y, TY* __restrict__ Y2) {
  const int64_t total = (int64_t)nwin * k1 * l;
  for (int b = blockIdx.y; b < nblocks; b += gridDim.y) {
    const int64_t y2 = blk2[b].y_off;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * 256) {
      const int slot = (int)(e / l);
      const int r = (int)(e - (int64_t)slot * l);
      const int w = slot / k1, t = slot - w * k1;
      const int64_t wi = (int64_t)b * nwin + w;
      TY v = (TY)0;
      if (t < k1w[wi]) v = Y[win[wi].y_off + (int64_t)S1[wi * k1 + t] * l + r];
      Y2[y2 + (int64_t)slot * l + r] = v;
    }
  }
}

// Final pivots S = I_U(I_1) (columns of A, stage-2 pivot order), k, status
// (the stage-2 selection's, as on the compact union of the stage-1 pivots),
// and P(:, j) = C^1(:, slots of window w) C_w(:, j - c_w) for column j of
// window w; rows past k are zero.  A window with a non-finite sketch makes
// the block NONFINITE with k = 0.  One workgroup per block.
static __global__ __launch_bounds__(256) void ts_combine_kernel(
    const BlkInfo* __restrict__ blks, const BlkInfo* __restrict__ win,
    const BlkInfo* __restrict__ blk2, int nwin, int k1, int k_max,
    const int32_t* __restrict__ S1, const int32_t* __restrict__ k1w,
    const int32_t* __restrict__ st1, const double* __restrict__ P1,
    const int32_t* __restrict__ S2, const int32_t* __restrict__ k2,
    const int32_t* __restrict__ st2, const double* __restrict__ P2, double* __restrict__ P,
    int32_t* __restrict__ S_ws, int32_t* __restrict__ k_ws, int32_t* __restrict__ st_ws) {
  __shared__ int bad_s, union_s;
  const int b = blockIdx.x;
  const BlkInfo bi = blks[b];
  const int n = bi.n;
  if (threadIdx.x == 0) {
    int bad = 0, nu = 0;
    for (int w = 0; w < nwin; ++w) {
      if (st1[(int64_t)b * nwin + w] == 2) bad = 1;
      nu += k1w[(int64_t)b * nwin + w];
    }
    bad_s = bad;
    union_s = nu;
  }
  __syncthreads();
  const int kk = bad_s ? 0 : k2[b];
  for (int s = threadIdx.x; s < k_max; s += 256) {
    int v = -1;
    if (s < kk) {
      const int slot = S2[(int64_t)b * k_max + s];
      const int w = slot / k1, t = slot - w * k1;
      v = ts_window_start(w, n, nwin) + S1[((int64_t)b * nwin + w) * k1 + t];
    }
    S_ws[(int64_t)b * k_max + s] = v;
  }
  if (threadIdx.x == 0) {
    k_ws[b] = kk;
    // Stage 2 runs on nwin * k1 slots, the ones past a window's pivot count
    // zero.  Having taken every stage-1 pivot, it meets a zero pivot and
    // reports RANK_DEFICIENT; on the compact union of the stage-1 skeletons
    // (whose size caps the selection) the same pivots end the selection with
    // OK, and that is the status reported.
    int st = bad_s ? 2 : st2[b];
    if (st == 1 && kk > 0 && kk == union_s) st = 0;
    st_ws[b] = st;
  }
  const double* __restrict__ P2b = P2 + blk2[b].p_off;
  for (int64_t e = threadIdx.x; e < (int64_t)n * k_max; e += 256) {
    const int j = (int)(e / k_max), s = (int)(e - (int64_t)j * k_max);
    double acc = 0.0;
    if (s < kk) {
      const int w = ts_window_of(j, n, nwin);
      const int64_t wi = (int64_t)b * nwin + w;
      const double* __restrict__ cw =
          P1 + win[wi].p_off + (int64_t)(j - ts_window_start(w, n, nwin)) * k1;
      const int kw = k1w[wi];
      for (int t = 0; t < kw; ++t) acc += P2b[(int64_t)(w * k1 + t) * k_max + s] * cw[t];
    }
    P[bi.p_off + (int64_t)j * k_max + s] = acc;
  }
}

}  // namespace spid
