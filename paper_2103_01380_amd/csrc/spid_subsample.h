// spid_subsample.h -- device kernels of the deterministic coarse-grid sketch
// (arXiv 2103.01380, Section 2): the sketch is the row subsample
// B = A(J,:) of a coarse grid (Algorithm 2, SubID), the selection runs on B,
// and the single-pass approximation M B(:,S) C interpolates the coarse
// skeleton back to the fine grid (equation (single_ID), Algorithm 3) with a
// trilinear M (Section 5.2).
//
// Grid convention: block b stacks nf fields, each on an nx x ny x nz
// structured grid, fine row f*nx*ny*nz + x + nx*(y + ny*z).  Coarse
// coordinates per direction are 0, s, 2s, ... below the point count
// (ceil(N/s) points); coarse rows use the same ordering.  A fine point at or
// past the last coarse coordinate of a direction takes that coordinate's
// value (the grid is not extended).
#pragma once

#include "spid_kernels.h"

namespace spid {

struct GridInfo {
  int32_t nx, ny, nz, nf;  // fine points per direction, fields
  int32_t sx, sy, sz;      // subsampling interval per direction
  int32_t cx, cy, cz;      // coarse points per direction
  int32_t mc;              // coarse rows of the block, nf * cx * cy * cz
  int32_t pad;
  int64_t cs_off;          // element offset of the block's coarse skeleton (mc x k_max)
};

// fine row of coarse row r
__device__ __forceinline__ int64_t coarse_to_fine(const GridInfo& g, int r) {
  const int cxyz = g.cx * g.cy * g.cz;
  const int f = r / cxyz;
  int p = r - f * cxyz;
  const int tx = p % g.cx;
  p /= g.cx;
  const int ty = p % g.cy;
  const int tz = p / g.cy;
  return (int64_t)f * g.nx * g.ny * g.nz + (int64_t)tx * g.sx +
         (int64_t)g.nx * ((int64_t)ty * g.sy + (int64_t)g.ny * tz * g.sz);
}

// linear weights of fine coordinate x between coarse points t*s, t < nc
__device__ __forceinline__ void lin_weights(int x, int s, int nc, int& t0, int& t1, double& w0,
                                            double& w1) {
  const int t = x / s;
  if (t >= nc - 1) {
    t0 = t1 = nc - 1;
    w0 = 1.0;
    w1 = 0.0;
  } else {
    const double frac = (double)(x - t * s) / (double)s;
    t0 = t;
    t1 = t + 1;
    w0 = 1.0 - frac;
    w1 = frac;
  }
}

// ---------------------------------------------------------------------------
// Sketch update of the coarse-grid sketch: Y_b(r, j) = A_b(J_b[r], j) for
// r < mc_b and 0 for mc_b <= r < l (zero rows change no sum of the
// selection), columns [j0, min(j1, n_b)).  One thread per sketch entry, rows
// fastest (coalesced sketch writes; the reads are the subsample's stride).
// Grid: x covers l * (j1 - j0) entries, y strides over blocks.
// ---------------------------------------------------------------------------
template <typename TA>
__global__ __launch_bounds__(256) void subsample_kernel(const BlkInfo* __restrict__ blks,
                                                        const GridInfo* __restrict__ grids,
                                                        int nblocks, int l, int j0, int j1,
                                                        double* __restrict__ Y) {
  for (int b = blockIdx.y; b < nblocks; b += gridDim.y) {
    const int n = blks[b].n;
    const int je = min(j1, n);
    if (je <= j0) continue;
    const int64_t lda = blks[b].lda;
    const int64_t y_off = blks[b].y_off;
    gptr<TA> __restrict__ A = (gptr<TA>)blks[b].A;
    const GridInfo g = grids[b];
    const int64_t total = (int64_t)l * (je - j0);
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * 256) {
      const int jj = (int)(e / l);
      const int r = (int)(e - (int64_t)jj * l);
      const int j = j0 + jj;
      double v = 0.0;
      if (r < g.mc) v = (double)A[(int64_t)j * lda + coarse_to_fine(g, r)];
      Y[y_off + (int64_t)j * l + r] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// Column selection of tall sketches (Section 2, Algorithm 1 mgsqr on B; the
// coarse grid can have far more rows than registers and LDS hold): the
// working copy W of the block's sketch lives in global memory (L2-resident
// for the block being processed), one workgroup per block, one wave per
// column with the rows over the lanes (coalesced), so every
// dot product and norm is a wave reduction (16 waves per workgroup, four
// row loads per lane in flight).  Same steps, stopping rules and
// outputs as the register kernels: pivot = largest residual norm (ties to
// the lowest index), q = W(:,p)/||W(:,p)|| (stored over W(:,p)), one
// Gram-Schmidt sweep, norms recomputed.
// ---------------------------------------------------------------------------
constexpr int kTallThreads = 1024;
constexpr int kTallUnroll = 4;   // independent row loads per lane in flight
constexpr int kTallMaxN = 1024;

// RPL > 0 (l <= 64 RPL): each wave keeps the pivot column q and the column
// it updates in registers, so a column is read once and written once per
// step; RPL = 0: any l, two streaming passes per column.
template <int RPL>
__global__ __launch_bounds__(kTallThreads) void select_tall_kernel(
    const BlkInfo* __restrict__ blks, int l, int k_max, double tol, double rank_floor,
    const double* __restrict__ Y, double* __restrict__ W, double* __restrict__ R,
    int32_t* __restrict__ S_ws, int32_t* __restrict__ k_ws, int32_t* __restrict__ st_ws) {
  __shared__ double nu[kTallMaxN];
  __shared__ unsigned char used[kTallMaxN];
  __shared__ double red_v[kTallThreads / kWave];
  __shared__ int red_i[kTallThreads / kWave];
  constexpr int NWV = kTallThreads / kWave;
  const int b = blockIdx.x;
  const BlkInfo bi = blks[b];
  const int n = bi.n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double* __restrict__ Yb = Y + bi.y_off;
  double* __restrict__ Wb = W + bi.y_off;
  double* __restrict__ Rb = R + bi.r_off;

  int bad = 0;
  for (int j = wave; j < n; j += NWV) {
    double acc = 0.0;
    for (int r0 = lane; r0 < l; r0 += kTallUnroll * kWave) {
      double v[kTallUnroll];
#pragma unroll
      for (int u = 0; u < kTallUnroll; ++u) {
        const int r = r0 + u * kWave;
        v[u] = r < l ? Yb[(int64_t)j * l + r] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kTallUnroll; ++u) {
        const int r = r0 + u * kWave;
        if (r < l) Wb[(int64_t)j * l + r] = v[u];
        if (!isfinite(v[u])) bad = 1;
        acc += v[u] * v[u];
      }
    }
    acc = wave_sum(acc);
    if (lane == 0) {
      nu[j] = acc;
      used[j] = 0;
    }
  }
  const int any_bad = __syncthreads_or(bad);

  // ||Y||_F^2 and the largest initial column norm
  double fs = 0.0, fm = 0.0;
  for (int j = tid; j < n; j += kTallThreads) {
    fs += nu[j];
    fm = fmax(fm, nu[j]);
  }
  fs = wave_sum(fs);
  fm = wave_max(fm);
  if (lane == 0) red_v[wave] = fs;
  __syncthreads();
  double F2 = 0.0;
  for (int v = 0; v < NWV; ++v) F2 += red_v[v];
  __syncthreads();
  if (lane == 0) red_v[wave] = fm;
  __syncthreads();
  double nu0max = 0.0;
  for (int v = 0; v < NWV; ++v) nu0max = fmax(nu0max, red_v[v]);
  __syncthreads();

  int kcap = k_max;
  if (kcap > l) kcap = l;
  if (kcap > n) kcap = n;
  int status = 0, taken = 0;
  if (any_bad) {
    status = 2;
  } else {
    for (int s = 0; s < kcap; ++s) {
      double bv = -1.0;
      int bj = 0x7fffffff;
      for (int j = tid; j < n; j += kTallThreads)
        if (!used[j] && nu[j] > bv) {   // ascending j: ties keep the lowest index
          bv = nu[j];
          bj = j;
        }
      wave_argmax(bv, bj);
      if (lane == 0) {
        red_v[wave] = bv;
        red_i[wave] = bj;
      }
      __syncthreads();
      double best = red_v[0];
      int p = red_i[0];
      for (int x = 1; x < NWV; ++x)
        if (red_v[x] > best || (red_v[x] == best && red_i[x] < p)) {
          best = red_v[x];
          p = red_i[x];
        }
      __syncthreads();
      if (!(best > 0.0)) {
        status = 1;
        break;
      }
      if (rank_floor > 0.0 && best <= rank_floor * rank_floor * nu0max) {
        status = 1;
        break;
      }
      if (wave == 0) {
        double pn = 0.0;
        for (int r0 = lane; r0 < l; r0 += kTallUnroll * kWave) {
          double v[kTallUnroll];
#pragma unroll
          for (int u = 0; u < kTallUnroll; ++u) {
            const int r = r0 + u * kWave;
            v[u] = r < l ? Wb[(int64_t)p * l + r] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < kTallUnroll; ++u) pn += v[u] * v[u];
        }
        const double rss = sqrt(wave_sum(pn));
        for (int r = lane; r < l; r += kWave) Wb[(int64_t)p * l + r] /= rss;
        if (lane == 0) {
          Rb[(int64_t)s * n + p] = rss;
          S_ws[(int64_t)b * k_max + s] = p;
          used[p] = 1;
          nu[p] = 0.0;
        }
      }
      __syncthreads();
      taken = s + 1;
      const double* __restrict__ q = Wb + (int64_t)p * l;
      if constexpr (RPL > 0) {
        double qr[RPL];
#pragma unroll
        for (int u = 0; u < RPL; ++u) {
          const int r = lane + u * kWave;
          qr[u] = r < l ? q[r] : 0.0;
        }
        for (int j = wave; j < n; j += NWV) {
          if (used[j]) continue;   // uniform over the wave
          double* __restrict__ wj = Wb + (int64_t)j * l;
          double wv[RPL];
          double d = 0.0;
#pragma unroll
          for (int u = 0; u < RPL; ++u) {
            const int r = lane + u * kWave;
            wv[u] = r < l ? wj[r] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < RPL; ++u) d += qr[u] * wv[u];
          d = wave_sum(d);
          double a2 = 0.0;
#pragma unroll
          for (int u = 0; u < RPL; ++u) {
            const int r = lane + u * kWave;
            const double v = wv[u] - d * qr[u];
            if (r < l) wj[r] = v;
            a2 += v * v;
          }
          a2 = wave_sum(a2);
          if (lane == 0) {
            Rb[(int64_t)s * n + j] = d;
            nu[j] = a2;
          }
        }
      } else {
      for (int j = wave; j < n; j += NWV) {
        if (used[j]) continue;   // uniform over the wave
        double* __restrict__ wj = Wb + (int64_t)j * l;
        double d = 0.0;
        for (int r0 = lane; r0 < l; r0 += kTallUnroll * kWave) {
          double qv[kTallUnroll], wv[kTallUnroll];
#pragma unroll
          for (int u = 0; u < kTallUnroll; ++u) {
            const int r = r0 + u * kWave;
            qv[u] = r < l ? q[r] : 0.0;
            wv[u] = r < l ? wj[r] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < kTallUnroll; ++u) d += qv[u] * wv[u];
        }
        d = wave_sum(d);
        double a2 = 0.0;
        for (int r0 = lane; r0 < l; r0 += kTallUnroll * kWave) {
          double qv[kTallUnroll], wv[kTallUnroll];
#pragma unroll
          for (int u = 0; u < kTallUnroll; ++u) {
            const int r = r0 + u * kWave;
            qv[u] = r < l ? q[r] : 0.0;
            wv[u] = r < l ? wj[r] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < kTallUnroll; ++u) {
            const int r = r0 + u * kWave;
            const double v = wv[u] - d * qv[u];
            if (r < l) wj[r] = v;
            a2 += v * v;
          }
        }
        a2 = wave_sum(a2);
        if (lane == 0) {
          Rb[(int64_t)s * n + j] = d;
          nu[j] = a2;
        }
      }
      }
      __syncthreads();
      if (tol > 0.0) {
        double rest = 0.0;
        for (int j = tid; j < n; j += kTallThreads)
          if (!used[j]) rest += nu[j];
        rest = wave_sum(rest);
        if (lane == 0) red_v[wave] = rest;
        __syncthreads();
        double tot = 0.0;
        for (int v = 0; v < NWV; ++v) tot += red_v[v];
        __syncthreads();
        if (sqrt(tot) <= tol * sqrt(F2)) break;
        if (s == kcap - 1) status = 3;
      }
    }
  }
  if (tid == 0) {
    k_ws[b] = taken;
    st_ws[b] = status;
  }
  for (int s = taken + tid; s < k_max; s += kTallThreads) S_ws[(int64_t)b * k_max + s] = -1;
}

// ---------------------------------------------------------------------------
// Column selection of a few very tall sketches (the single-partition case):
// the same mgsqr steps as select_tall_kernel, with every block's rows split
// into chunks of kSplitRows so that many workgroups share one block.  One
// step is three launches: the pivot (one workgroup per block: fixed-order
// sums of the chunk partial norms, stopping rules, argmax), the dot products
// (per chunk: that chunk's rows of q = W(:,p)/r_pp are formed in place, then
// partial q.W(:,j)), and the update (per chunk: fixed-order sum of the
// partial dots, W(:,j) -= d_j q, partial norms).  A block that has stopped
// makes the later launches return at once; the host launches k steps plus
// one final pivot launch (which applies the last tolerance test).
// State per block (SplitState) and partial sums live in the workspace.
// ---------------------------------------------------------------------------
constexpr int kSplitRows = 256;
constexpr int kSplitThreads = 1024;  // 16 waves: columns of a chunk in flight at once

struct SplitState {
  double F2, nu0max, rss;
  int32_t p, done, k, status;
};

// clears the per-block non-finite flags before split_init_kernel
static __global__ void split_clear_kernel(int nblocks, int32_t* __restrict__ bad) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nblocks) bad[b] = 0;
}

// copy of the sketch, non-finite check, partial column norms of each chunk
static __global__ __launch_bounds__(kSplitThreads) void split_init_kernel(
    const BlkInfo* __restrict__ blks, int l, const double* __restrict__ Y, double* __restrict__ W,
    const int64_t* __restrict__ poff, double* __restrict__ pnorm, int32_t* __restrict__ bad) {
  const int b = blockIdx.y, c = blockIdx.x;
  const int nch = (l + kSplitRows - 1) / kSplitRows;
  if (c >= nch) return;
  const BlkInfo bi = blks[b];
  const int n = bi.n;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r0 = c * kSplitRows, r1 = min(l, r0 + kSplitRows);
  int nonfinite = 0;
  for (int j = wave; j < n; j += kSplitThreads / kWave) {
    double acc = 0.0;
    for (int r = r0 + lane; r < r1; r += kWave) {
      const double v = Y[bi.y_off + (int64_t)j * l + r];
      W[bi.y_off + (int64_t)j * l + r] = v;
      if (!isfinite(v)) nonfinite = 1;
      acc += v * v;
    }
    acc = wave_sum(acc);
    if (lane == 0) pnorm[poff[b] + (int64_t)c * n + j] = acc;
  }
  if (__any(nonfinite) && lane == 0) bad[b] = 1;   // only ever set: no ordering needed
}

// pivot of step s (s == kcap_b: the final tolerance test only)
static __global__ __launch_bounds__(kSplitThreads) void split_pivot_kernel(
    const BlkInfo* __restrict__ blks, int l, int k_max, double tol, double rank_floor, int s,
    const int64_t* __restrict__ poff, const double* __restrict__ pnorm,
    unsigned char* __restrict__ used, SplitState* __restrict__ st, const int32_t* __restrict__ bad,
    double* __restrict__ R, int32_t* __restrict__ S_ws, int32_t* __restrict__ k_ws,
    int32_t* __restrict__ st_ws) {
  __shared__ double nu[kTallMaxN];
  __shared__ double red_v[kSplitThreads / kWave];
  __shared__ int red_i[kSplitThreads / kWave];
  constexpr int NWV = kSplitThreads / kWave;
  const int b = blockIdx.x;
  const BlkInfo bi = blks[b];
  const int n = bi.n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  SplitState& S = st[b];
  if (s > 0 && S.done) return;                          // uniform
  unsigned char* __restrict__ ub = used + (int64_t)b * kTallMaxN;
  const int nch = (l + kSplitRows - 1) / kSplitRows;
  int kcap = k_max;
  if (kcap > l) kcap = l;
  if (kcap > n) kcap = n;
  auto finish = [&](int k, int status) {
    if (tid == 0) {
      S.done = 1;
      S.k = k;
      S.status = status;
      k_ws[b] = k;
      st_ws[b] = status;
    }
    for (int t = k + tid; t < k_max; t += kSplitThreads) S_ws[(int64_t)b * k_max + t] = -1;
  };
  if (s == 0) {
    if (tid == 0) S.done = 0;
    for (int j = tid; j < n; j += kSplitThreads) ub[j] = 0;
    if (bad[b]) {
      finish(0, 2);
      return;
    }
  }
  // nu_j of the live columns: fixed-order sums of the chunk partials
  for (int j = tid; j < n; j += kSplitThreads) {
    double v = 0.0;
    if (s == 0 || !ub[j])
      for (int c = 0; c < nch; ++c) v += pnorm[poff[b] + (int64_t)c * n + j];
    nu[j] = v;
  }
  __syncthreads();
  double fs = 0.0, fm = 0.0;
  for (int j = tid; j < n; j += kSplitThreads) {
    fs += nu[j];
    fm = fmax(fm, nu[j]);
  }
  fs = wave_sum(fs);
  fm = wave_max(fm);
  if (lane == 0) red_v[wave] = fs;
  __syncthreads();
  double tot = 0.0;
  for (int v = 0; v < NWV; ++v) tot += red_v[v];
  __syncthreads();
  if (lane == 0) red_v[wave] = fm;
  __syncthreads();
  double mx = 0.0;
  for (int v = 0; v < NWV; ++v) mx = fmax(mx, red_v[v]);
  __syncthreads();
  double F2, nu0max;
  if (s == 0) {
    F2 = tot;
    nu0max = mx;
    if (tid == 0) {
      S.F2 = tot;
      S.nu0max = mx;
    }
  } else {
    F2 = S.F2;
    nu0max = S.nu0max;
    if (tol > 0.0 && sqrt(tot) <= tol * sqrt(F2)) {   // after the previous step's update
      finish(s, 0);
      return;
    }
  }
  if (s >= kcap) {
    finish(kcap, tol > 0.0 ? 3 : 0);
    return;
  }
  double bv = -1.0;
  int bj = 0x7fffffff;
  for (int j = tid; j < n; j += kSplitThreads)
    if (!ub[j] && nu[j] > bv) {   // ascending j: ties keep the lowest index
      bv = nu[j];
      bj = j;
    }
  wave_argmax(bv, bj);
  if (lane == 0) {
    red_v[wave] = bv;
    red_i[wave] = bj;
  }
  __syncthreads();
  double best = red_v[0];
  int p = red_i[0];
  for (int x = 1; x < NWV; ++x)
    if (red_v[x] > best || (red_v[x] == best && red_i[x] < p)) {
      best = red_v[x];
      p = red_i[x];
    }
  if (!(best > 0.0) || (rank_floor > 0.0 && best <= rank_floor * rank_floor * nu0max)) {
    finish(s, 1);
    return;
  }
  if (tid == 0) {
    const double rss = sqrt(best);
    S.p = p;
    S.rss = rss;
    R[bi.r_off + (int64_t)s * n + p] = rss;
    S_ws[(int64_t)b * k_max + s] = p;
    ub[p] = 1;
  }
}

// dot products of step s: chunk rows of q formed in place, partial q.W(:,j)
static __global__ __launch_bounds__(kSplitThreads) void split_dot_kernel(
    const BlkInfo* __restrict__ blks, int l, const int64_t* __restrict__ poff,
    const SplitState* __restrict__ st, const unsigned char* __restrict__ used,
    double* __restrict__ W, double* __restrict__ pdot) {
  const int b = blockIdx.y, c = blockIdx.x;
  const int nch = (l + kSplitRows - 1) / kSplitRows;
  if (c >= nch || st[b].done) return;
  const BlkInfo bi = blks[b];
  const int n = bi.n;
  const int p = st[b].p;
  const double rss = st[b].rss;
  const unsigned char* __restrict__ ub = used + (int64_t)b * kTallMaxN;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r0 = c * kSplitRows, r1 = min(l, r0 + kSplitRows);
  double* __restrict__ q = W + bi.y_off + (int64_t)p * l;
  __shared__ double qs[kSplitRows];
  for (int r = r0 + threadIdx.x; r < r1; r += kSplitThreads) {
    const double v = q[r] / rss;
    q[r] = v;
    qs[r - r0] = v;
  }
  __syncthreads();
  for (int j = wave; j < n; j += kSplitThreads / kWave) {
    if (ub[j]) continue;   // the pivot and earlier pivots (uniform over the wave)
    double d = 0.0;
    for (int r = r0 + lane; r < r1; r += kWave) d += qs[r - r0] * W[bi.y_off + (int64_t)j * l + r];
    d = wave_sum(d);
    if (lane == 0) pdot[poff[b] + (int64_t)c * n + j] = d;
  }
}

// update of step s: d_j in a fixed order, W(:,j) -= d_j q on the chunk rows,
// chunk partial norms; chunk 0 records R(s, j)
static __global__ __launch_bounds__(kSplitThreads) void split_update_kernel(
    const BlkInfo* __restrict__ blks, int l, int s, const int64_t* __restrict__ poff,
    const SplitState* __restrict__ st, const unsigned char* __restrict__ used,
    const double* __restrict__ pdot, double* __restrict__ W, double* __restrict__ pnorm,
    double* __restrict__ R) {
  const int b = blockIdx.y, c = blockIdx.x;
  const int nch = (l + kSplitRows - 1) / kSplitRows;
  if (c >= nch || st[b].done) return;
  const BlkInfo bi = blks[b];
  const int n = bi.n;
  const int p = st[b].p;
  const unsigned char* __restrict__ ub = used + (int64_t)b * kTallMaxN;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r0 = c * kSplitRows, r1 = min(l, r0 + kSplitRows);
  __shared__ double qs[kSplitRows];
  for (int r = r0 + threadIdx.x; r < r1; r += kSplitThreads)
    qs[r - r0] = W[bi.y_off + (int64_t)p * l + r];
  __syncthreads();
  for (int j = wave; j < n; j += kSplitThreads / kWave) {
    if (ub[j]) continue;
    double d = 0.0;
    for (int x = 0; x < nch; ++x) d += pdot[poff[b] + (int64_t)x * n + j];
    double a2 = 0.0;
    for (int r = r0 + lane; r < r1; r += kWave) {
      const int64_t e = bi.y_off + (int64_t)j * l + r;
      const double v = W[e] - d * qs[r - r0];
      W[e] = v;
      a2 += v * v;
    }
    a2 = wave_sum(a2);
    if (lane == 0) {
      pnorm[poff[b] + (int64_t)c * n + j] = a2;
      if (c == 0) R[bi.r_off + (int64_t)s * n + j] = d;
    }
  }
}

// ---------------------------------------------------------------------------
// Single-pass error (equation (single_ID), Algorithm 3) on the FP64 matrix
// cores: Ahat(rows, cols) = K(rows, :) P(:, cols) with the interpolated
// skeleton K = M B(:,S) as the A operand of v_mfma_f64_16x16x4 (16 rows x 4
// selected columns per k-step, each entry an 8-point trilinear stencil over
// the coarse sketch, which stays in L2), P as the B operand, and the
// residual A - Ahat accumulated per lane.  Same tiling as the error pass of
// spid_reconstruct (row permutation inside a 16-row tile so that lane (g, c)
// owns rows 4g..4g+3 of column c; work item = it.nsub sub-tiles of
// 4 * 16 * MTR rows; coefficients staged in LDS pcap columns at a time) but
// over every column: the interpolated skeleton does not reproduce A on the
// selected columns.  Dynamic LDS: pcap * 4 * KS doubles.
// ---------------------------------------------------------------------------
template <typename TA, int KS, int MTR, bool VEC>
__global__ __launch_bounds__(kRcThreads) void interp_mfma_kernel(
    const BlkInfo* __restrict__ blks, const GridInfo* __restrict__ grids,
    const RcItem* __restrict__ items, XcdSplit xs, int l, int k_max, int pcap,
    const int32_t* __restrict__ S_ws, const int32_t* __restrict__ k_ws,
    const double* __restrict__ Y, const double* __restrict__ P, double* __restrict__ part) {
  // [pcap][kp + 1]: the odd stride puts the 16 columns one MFMA reads on
  // different banks (a stride of kp, a multiple of 16 doubles, is one bank)
  extern __shared__ __attribute__((aligned(16))) double p_lds[];
  __shared__ double red[8];
  constexpr int kp = 4 * KS;
  constexpr int kSub = 4 * 16 * MTR;
  const int item = xcd_item(xs);
  if (item < 0) return;
  const RcItem it = items[item];
  const BlkInfo bi = blks[it.blk];
  const GridInfo gr = grids[it.blk];
  const int n = bi.n;
  const int k = k_ws[it.blk];
  const int32_t* __restrict__ S = S_ws + (int64_t)it.blk * k_max;
  gptr<TA> __restrict__ A = (gptr<TA>)bi.A;
  const double* __restrict__ Pb = P + bi.p_off;
  const double* __restrict__ Yb = Y + bi.y_off;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, c16 = lane & 15;
  const int arow = 4 * (c16 & 3) + (c16 >> 2);
  const int64_t pts = (int64_t)gr.nx * gr.ny * gr.nz;
  const int cxyz = gr.cx * gr.cy * gr.cz;
  double a2 = 0.0, e2 = 0.0;

  for (int c0 = 0; c0 < n; c0 += pcap) {
    const int cc = min(pcap, n - c0);
    const int ntile = (cc + 15) / 16;
    for (int e = tid; e < ntile * 16 * kp; e += kRcThreads) {
      const int q = e / kp, t = e - q * kp;
      const bool ok = q < cc && t < k_max;
      const double x = Pb[(int64_t)(c0 + min(q, cc - 1)) * k_max + min(t, k_max - 1)];
      p_lds[q * (kp + 1) + t] = ok ? x : 0.0;   // P rows k..k_max-1 are zero
    }
    __syncthreads();
    for (int rs = 0; rs < it.nsub; ++rs) {
      const int64_t rbase = it.i0 + (int64_t)rs * kSub + (int64_t)wave * 16 * MTR;
      double as[MTR][KS];
#pragma unroll
      for (int mt = 0; mt < MTR; ++mt) {
        const int64_t i = rbase + 16 * mt + arow;
        const bool row = i < bi.m;
        int idx[8];
        double w[8];
        {
          const int64_t ii = row ? i : 0;
          const int f = (int)(ii / pts);
          const int64_t pp = ii - f * pts;
          const int x = (int)(pp % gr.nx);
          const int y = (int)((pp / gr.nx) % gr.ny);
          const int z = (int)(pp / ((int64_t)gr.nx * gr.ny));
          int tx0, tx1, ty0, ty1, tz0, tz1;
          double wx0, wx1, wy0, wy1, wz0, wz1;
          lin_weights(x, gr.sx, gr.cx, tx0, tx1, wx0, wx1);
          lin_weights(y, gr.sy, gr.cy, ty0, ty1, wy0, wy1);
          lin_weights(z, gr.sz, gr.cz, tz0, tz1, wz0, wz1);
          const int fb = f * cxyz;
#pragma unroll
          for (int c = 0; c < 8; ++c) {
            const int a = c >> 2, bb = (c >> 1) & 1, d = c & 1;
            idx[c] = fb + (d ? tx1 : tx0) + gr.cx * ((bb ? ty1 : ty0) + gr.cy * (a ? tz1 : tz0));
            w[c] = (a ? wz1 : wz0) * (bb ? wy1 : wy0) * (d ? wx1 : wx0);
          }
        }
        // stencils gathered without branches (entries outside the block or
        // past k read the first selected column, then are zeroed), so the
        // loads overlap
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          as[mt][s] = 0.0;
          if (4 * s >= k) continue;   // uniform: k-steps past the selected columns are never read
          const int t = 4 * s + g;
          const double* __restrict__ col = Yb + (int64_t)S[t < k ? t : 0] * l;
          double gv[8];
#pragma unroll
          for (int c = 0; c < 8; ++c) gv[c] = col[idx[c]];
          double v = 0.0;
#pragma unroll
          for (int c = 0; c < 8; ++c) v += w[c] * gv[c];
          as[mt][s] = (t < k && row) ? v : 0.0;
        }
      }
      for (int tq = 0; tq < ntile; ++tq) {
        const int q = 16 * tq + c16;
        const bool cok = q < cc;
        gptr<TA> colp = A + (int64_t)(c0 + (cok ? q : cc - 1)) * bi.lda;
        double av[MTR][4];
#pragma unroll
        for (int mt = 0; mt < MTR; ++mt)
          rc_load4<TA, VEC>(colp, rbase + 16 * mt + 4 * g, bi.m, cok, av[mt]);
        const double* pc = p_lds + q * (kp + 1) + g;
        f64x4 acc[MTR];
#pragma unroll
        for (int mt = 0; mt < MTR; ++mt) acc[mt] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          if (4 * s >= k) break;    // uniform: k-steps past the selected columns are zero
          const double pv = pc[4 * s];
#pragma unroll
          for (int mt = 0; mt < MTR; ++mt) acc[mt] = mfma_f64(as[mt][s], pv, acc[mt]);
        }
#pragma unroll
        for (int mt = 0; mt < MTR; ++mt)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const double r = av[mt][v] - acc[mt][v];
            e2 += r * r;
            a2 += av[mt][v] * av[mt][v];
          }
      }
    }
    __syncthreads();
  }

  e2 = wave_sum(e2);
  a2 = wave_sum(a2);
  if (lane == 0) {
    red[wave] = e2;
    red[4 + wave] = a2;
  }
  __syncthreads();
  if (tid == 0) {
    part[2 * (int64_t)item] = red[0] + red[1] + red[2] + red[3];
    part[2 * (int64_t)item + 1] = red[4] + red[5] + red[6] + red[7];
  }
}

// Coarse skeleton B_b(:, S_b) (what Algorithm 3 stores): mc_b x k_max
// column-major in the A dtype at grids[b].cs_off; columns >= k_b untouched.
template <typename TA>
__global__ __launch_bounds__(256) void coarse_skeleton_kernel(
    const BlkInfo* __restrict__ blks, const GridInfo* __restrict__ grids, int nblocks, int l,
    int k_max, const int32_t* __restrict__ S_ws, const int32_t* __restrict__ k_ws,
    const double* __restrict__ Y, TA* __restrict__ out) {
  for (int b = blockIdx.y; b < nblocks; b += gridDim.y) {
    const int k = k_ws[b];
    const int mc = grids[b].mc;
    const int64_t cs = grids[b].cs_off;
    const int64_t y_off = blks[b].y_off;
    const int64_t total = (int64_t)mc * k;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * 256) {
      const int t = (int)(e / mc);
      const int r = (int)(e - (int64_t)t * mc);
      out[cs + (int64_t)t * mc + r] =
          (TA)Y[y_off + (int64_t)S_ws[(int64_t)b * k_max + t] * l + r];
    }
  }
}

}  // namespace spid
