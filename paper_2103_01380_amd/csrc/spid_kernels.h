// spid_kernels.h -- gfx950 kernels of the sketched column ID.
//
//   sketch_kernel     Y_b(:, cols) = Omega_b A_b(:, cols) on the matrix cores,
//                     Omega regenerated per 32-row chunk into LDS.
//   sketch_reduce     fixed-order sum of split-K partial sketches (per block,
//                     or per group of blocks for one-snapshot updates).
//   select_step_kernel pivoted modified Gram-Schmidt on the sketch, one
//                     workgroup per block, sketch columns in registers (groups
//                     of lanes holding four columns), one barrier per step.
//   coeffs_kernel     back-substitution R11 x = R12(:, j) in row blocks of 16
//                     (diagonal solves in registers, updates on the FP64 matrix
//                     cores), identity columns (and the split-bfloat16
//                     coefficients of the mixed error pass).
//   recon_mfma_kernel streaming residual ||A - A(:,S) P||^2 per row tile, the
//                     product A(:,S) P on the FP64 matrix cores.
//   recon_reduce      fixed-order per-block sums of the row-tile partials.
#pragma once

#include <type_traits>

#include "spid_device.h"

namespace spid {

// Per-block table in the workspace (filled at create / bind).
struct BlkInfo {
  const void* A;      // device address of block b (column-major)
  int64_t lda;        // leading dimension (elements)
  int64_t m;          // rows
  int64_t y_off;      // element offset of Y_b (l x n column-major)
  int64_t r_off;      // element offset of R_b (k_max x n row-major)
  int64_t p_off;      // element offset of P_b (k_max x n column-major)
  int64_t sk_off;     // element offset of the skeleton (m x k_max)
  int64_t part_off;   // element offset of the split-K partials (nsplit x l x n)
  int32_t n;          // columns
  int32_t nsplit;     // K splits of the sketch (1: written straight to Y)
  int32_t vec_ok;     // 1 if column starts are 16-byte aligned
  int32_t pad;
};

// One sketch work item: block, 64*TN-column tile, K range [r0, r1).
struct SkItem {
  int32_t blk;        // block (stream items: the first block of the group)
  int32_t c0;         // first column (stream items: first position in the block order)
  int32_t split;      // index of the K range
  int32_t gsize;      // stream items: blocks in the group
  int64_t r0, r1;     // rows [r0, r1)
  int32_t gnsplit;    // stream items: K ranges of the group
  int32_t pad;
  int64_t gpart;      // stream items: element offset of the group's partial sketches
};

// One reconstruction work item: block, rows [i0, i0 + 256).
struct RcItem {
  int32_t blk;
  int32_t nsub;       // row sub-tiles of this item
  int64_t i0;         // first row
};

constexpr int kSkThreads = 256;   // 4 waves
constexpr int kKC = 32;           // rows per sketch chunk
constexpr int kOmStride = kKC + 2;  // LDS row stride (doubles) of the Omega tile

// Loads of A for the sketch kernels.  Full chunks use straight-line loads
// (no branches: the column is clamped to a valid one and the values of an
// invalid column are zeroed by selection), so the compiler can keep the
// prefetched chunk in flight with partial vmcnt waits; only the ragged last
// chunk of a work item takes the checked path.
//
// A lane reads NP pieces of W consecutive rows of one column, piece p
// starting at row + p * STEP.  The four lanes sharing a column (g = 0..3)
// start at row + W g, so every load instruction of a 16-column group reads
// one contiguous run of 4 W elements per column.  VEC: aligned column starts
// (16 bytes) and W-aligned rows, so the pieces are 8- or 16-byte vectors.
template <typename TA, int NP, int W, int STEP, bool VEC, typename TO>
__device__ __forceinline__ void load_pieces_full(gptr<TA> __restrict__ cb, int64_t row, bool ok,
                                                 TO out[NP * W]) {
  constexpr int kBytes = W * (int)sizeof(TA);
#pragma unroll
  for (int pc = 0; pc < NP; ++pc) {
    gptr<TA> p = cb + row + pc * STEP;
    if constexpr (VEC && kBytes % 16 == 0 && sizeof(TA) == 8) {
#pragma unroll
      for (int h = 0; h < W / 2; ++h) {
        const f64x2 v = __builtin_nontemporal_load((gptr<f64x2>)p + h);
        out[W * pc + 2 * h] = ok ? (TO)v[0] : (TO)0;
        out[W * pc + 2 * h + 1] = ok ? (TO)v[1] : (TO)0;
      }
    } else if constexpr (VEC && kBytes % 16 == 0 && sizeof(TA) == 4) {
#pragma unroll
      for (int h = 0; h < W / 4; ++h) {
        const f32x4 v = __builtin_nontemporal_load((gptr<f32x4>)p + h);
#pragma unroll
        for (int e = 0; e < 4; ++e) out[W * pc + 4 * h + e] = ok ? (TO)v[e] : (TO)0;
      }
    } else if constexpr (VEC && kBytes == 8 && sizeof(TA) == 4) {
      const f32x2 v = __builtin_nontemporal_load((gptr<f32x2>)p);
      out[2 * pc] = ok ? (TO)v[0] : (TO)0;
      out[2 * pc + 1] = ok ? (TO)v[1] : (TO)0;
    } else if constexpr (sizeof(TA) == 4 && W == 4) {
      // element-aligned vector load through the caches (see load_line)
      const f32x4u v = *(gptr<f32x4u>)p;
#pragma unroll
      for (int e = 0; e < 4; ++e) out[W * pc + e] = ok ? (TO)v[e] : (TO)0;
    } else if constexpr (sizeof(TA) == 8 && W % 2 == 0) {
#pragma unroll
      for (int h = 0; h < W / 2; ++h) {
        const f64x2u v = *((gptr<f64x2u>)p + h);
        out[W * pc + 2 * h] = ok ? (TO)v[0] : (TO)0;
        out[W * pc + 2 * h + 1] = ok ? (TO)v[1] : (TO)0;
      }
    } else {
#pragma unroll
      for (int e = 0; e < W; ++e) {
        const TA v = __builtin_nontemporal_load(p + e);
        out[W * pc + e] = ok ? (TO)v : (TO)0;
      }
    }
  }
}

// The same for a ragged chunk: rows at or past `rend` read as zero.
template <typename TA, int NP, int W, int STEP, typename TO>
__device__ __forceinline__ void load_pieces_tail(gptr<TA> __restrict__ cb, int64_t row,
                                                 int64_t rend, bool ok, TO out[NP * W]) {
#pragma unroll
  for (int pc = 0; pc < NP; ++pc)
#pragma unroll
    for (int e = 0; e < W; ++e) {
      const int64_t r = row + pc * STEP + e;
      out[W * pc + e] = (ok && r < rend) ? (TO)cb[r] : (TO)0;
    }
}

// ---------------------------------------------------------------------------
// Omega chunk generation into LDS: rows 0..l-1 of columns k0..k0+31 of the
// sketch matrix (pair q -> rows 2q, 2q+1).  Rows l..MT*16-1 stay zero.
// ---------------------------------------------------------------------------
// bfloat16 Omega chunk: entries rounded to nearest-even bfloat16 through the
// cheap exact path of omega_pair_rounded.
template <int STRIDE, int NTHR>
__device__ __forceinline__ void gen_omega_chunk_bf16(__bf16* __restrict__ om, int l, uint64_t seed,
                                                     uint32_t bkey, int64_t k0, int tid) {
  const int npairs = (l + 1) >> 1;
  for (int e = tid; e < npairs * kKC; e += NTHR) {
    const int q = e / kKC, kk = e - q * kKC;
    float z0, z1;
    omega_pair_rounded<0>(seed, bkey, (uint32_t)(k0 + kk), (uint32_t)q, z0, z1);
    om[(2 * q) * STRIDE + kk] = to_bf16(z0);
    if (2 * q + 1 < l) om[(2 * q + 1) * STRIDE + kk] = to_bf16(z1);
  }
}

template <typename TO, int STRIDE, int NTHR, typename CVT>
__device__ __forceinline__ void gen_omega_chunk(TO* __restrict__ om, int l, uint64_t seed,
                                                uint32_t bkey, int64_t k0, int tid, CVT cvt) {
  const int npairs = (l + 1) >> 1;
  for (int e = tid; e < npairs * kKC; e += NTHR) {
    const int q = e / kKC, kk = e - q * kKC;
    const double2 z = omega_pair(seed, bkey, (uint32_t)(k0 + kk), (uint32_t)q);
    om[(2 * q) * STRIDE + kk] = cvt(z.x);
    if (2 * q + 1 < l) om[(2 * q + 1) * STRIDE + kk] = cvt(z.y);
  }
}

// Shared double-precision Omega, regenerated once per update: chunk c (A rows
// 32c..32c+31), Omega row r: 32 doubles at ((c * MT*16 + r) * 32), the
// chunk's LDS row without its padding; rows l.. zero.  A work item copies its
// chunks into LDS (copy_omega_chunk_f64) instead of generating them.
template <typename TD>   // double
__global__ __launch_bounds__(256) void omega_table_f64_kernel(int l, int MT, int64_t ncols,
                                                              uint64_t seed, TD* __restrict__ tab) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)MT * 8 * ncols) return;
  const int q = (int)(e / ncols);
  const int64_t i = e - (int64_t)q * ncols;
  double2 z = make_double2(0.0, 0.0);
  if (2 * q < l) z = omega_pair(seed, 0u, (uint32_t)i, (uint32_t)q);
  if (2 * q + 1 >= l) z.y = 0.0;
  const int64_t base = (i >> 5) * MT * 16 * kKC + (i & 31);
  tab[base + (int64_t)(2 * q) * kKC] = z.x;
  tab[base + (int64_t)(2 * q + 1) * kKC] = z.y;
}

template <int STRIDE, int NTHR>
__device__ __forceinline__ void copy_omega_chunk_f64(double* __restrict__ om, int MT,
                                                     const double* __restrict__ tab, int64_t k0,
                                                     int tid) {
  const f64x2* __restrict__ src = reinterpret_cast<const f64x2*>(tab + (k0 / kKC) * MT * 16 * kKC);
  for (int e = tid; e < MT * 16 * (kKC / 2); e += NTHR) {
    const int r = e / (kKC / 2), c2 = e - r * (kKC / 2);
    const f64x2 v = src[e];
    om[r * STRIDE + 2 * c2] = v[0];
    om[r * STRIDE + 2 * c2 + 1] = v[1];
  }
}

// ---------------------------------------------------------------------------
// Common set-up of a sketch work item: the lane's columns (clamped to a valid
// column, with a validity flag), the updated column window, the Omega key.
// ---------------------------------------------------------------------------
template <typename TA, int TN>
struct SkLane {
  gptr<TA> cb[TN];    // column starts (clamped)
  bool ok[TN];        // column inside the block and inside [j0, j1)
  int col[TN];
};

template <typename TA, int TN>
__device__ __forceinline__ bool sk_setup(const BlkInfo& bi, const SkItem& it, int cwave, int r16,
                                         int span, int j0, int j1, SkLane<TA, TN>& ln) {
  const int clo = max(j0, 0), chi = min(j1, bi.n);
  if (it.c0 >= chi || it.c0 + span <= clo) return false;   // whole tile outside (uniform)
  gptr<TA> A = (gptr<TA>)bi.A;
#pragma unroll
  for (int u = 0; u < TN; ++u) {
    const int col = cwave + 16 * u + r16;
    ln.col[u] = col;
    ln.ok[u] = col >= clo && col < chi;
    ln.cb[u] = A + (int64_t)(ln.ok[u] ? col : clo) * bi.lda;
  }
  return true;
}

// One-snapshot update of many blocks (stream mode): the MFMA column
// dimension runs over the blocks of a group instead of one block's columns,
// so Y_b(:, j) = Omega(:, rows) A_b(rows, j) for every block of the group is
// one matrix product with a shared Omega chunk (blocks of a group have equal
// m_b; Omega keyed by (seed, r, i) only).  Lane column `local` is block
// perm[it.c0 + local], snapshot j.
template <typename TA, int TN>
__device__ __forceinline__ void sk_setup_stream(const BlkInfo* __restrict__ blks,
                                                const int32_t* __restrict__ perm,
                                                const SkItem& it, int cw, int r16, int j,
                                                SkLane<TA, TN>& ln) {
#pragma unroll
  for (int u = 0; u < TN; ++u) {
    const int local = cw + 16 * u + r16;
    const bool valid = local < it.gsize;
    const BlkInfo& bb = blks[perm[it.c0 + (valid ? local : 0)]];
    const bool ok = valid && j < bb.n;
    ln.col[u] = local;
    ln.ok[u] = ok;
    ln.cb[u] = (gptr<TA>)bb.A + (int64_t)(ok ? j : 0) * bb.lda;
  }
}

// Output offset of lane column u in the sketch (or its partial buffer).
template <typename TA, int TN, int GCAP, bool ST>
__device__ __forceinline__ int64_t sk_out_offset(const BlkInfo* __restrict__ blks,
                                                 const int32_t* __restrict__ perm,
                                                 const BlkInfo& bi, const SkItem& it,
                                                 const SkLane<TA, TN>& ln, int u, int l, int j) {
  if constexpr (ST) {
    if (it.gnsplit == 1) return blks[perm[it.c0 + ln.col[u]]].y_off + (int64_t)j * l;
    return it.gpart + ((int64_t)it.split * GCAP + ln.col[u]) * l;
  } else {
    const int64_t base = (bi.nsplit == 1) ? bi.y_off : bi.part_off + (int64_t)it.split * bi.n * l;
    return base + (int64_t)ln.col[u] * l;
  }
}

// ---------------------------------------------------------------------------
// Sketch, double precision: Y = Omega A on v_mfma_f64_16x16x4.
// Workgroup = NW waves; wave w owns columns c0 + 16*TN*w + [0, 16*TN); every
// wave covers all MT*16 sketch rows.  Per 32-row chunk each lane holds rows
// 8h + 2g + e (h = 0..3, e = 0..1, g = lane/16) of one column per 16-column
// tile, so each load instruction reads 64 contiguous bytes per column, and
// eight MFMA k-steps consume them (step 2h+e pairs that A row with the same
// Omega column).
// Software pipeline over the full chunks (two register buffers, two LDS
// buffers): while chunk c's MFMAs run, chunk c+1's loads are in flight and the
// workgroup generates chunk c+1's Omega; one LDS-only barrier per chunk.  The
// ragged last chunk is handled after the loop.
// ---------------------------------------------------------------------------
template <typename TA, int MT, int TN, int NW, bool VEC, bool ST>
__global__ __launch_bounds__(64 * NW) void sketch_f64_kernel(
    const BlkInfo* __restrict__ blks, const SkItem* __restrict__ items, int l, uint64_t seed,
    int omega_per_block, int j0, int j1, const int32_t* __restrict__ perm, int jst,
    const double* __restrict__ omtab, double* __restrict__ Y, double* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) double om[2][MT * 16 * kOmStride];
  const SkItem it = items[blockIdx.x];
  const BlkInfo bi = blks[it.blk];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, r16 = lane & 15;
  const int cwave = it.c0 + wave * 16 * TN;
  SkLane<TA, TN> ln;
  if constexpr (ST) {
    sk_setup_stream<TA, TN>(blks, perm, it, wave * 16 * TN, r16, jst, ln);
  } else {
    if (!sk_setup<TA, TN>(bi, it, cwave, r16, NW * 16 * TN, j0, j1, ln)) return;
  }
  const uint32_t bkey = omega_per_block ? (uint32_t)(it.blk + 1) : 0u;
  auto ident = [](double x) { return x; };
  // a chunk of Omega into LDS: copied from the update's table (shared Omega)
  // or generated (Omega keyed per block); uniform branch
  auto fill_om = [&](double* __restrict__ omb, int64_t k0) {
    if (omtab) copy_omega_chunk_f64<kOmStride, 64 * NW>(omb, MT, omtab, k0, tid);
    else gen_omega_chunk<double, kOmStride, 64 * NW>(omb, l, seed, bkey, k0, tid, ident);
  };
  // the table path split in two, so that its loads are issued before the A
  // prefetch of the same step and their wait leaves that prefetch in flight
  constexpr int kOmPieces = MT * 16 * (kKC / 2);   // 16-byte pieces of a chunk
  constexpr int kOmPer = (kOmPieces + 64 * NW - 1) / (64 * NW);
  f64x2 omr[kOmPer];
  auto om_load = [&](int64_t k0) {
    const f64x2* __restrict__ src = reinterpret_cast<const f64x2*>(omtab + (k0 / kKC) * MT * 16 * kKC);
#pragma unroll
    for (int i = 0; i < kOmPer; ++i) {
      const int e = tid + i * 64 * NW;
      if (e < kOmPieces) omr[i] = src[e];
    }
  };
  auto om_store = [&](double* __restrict__ omb) {
#pragma unroll
    for (int i = 0; i < kOmPer; ++i) {
      const int e = tid + i * 64 * NW;
      if (e < kOmPieces) {
        const int r = e / (kKC / 2), c2 = e - r * (kKC / 2);
        *reinterpret_cast<f64x2*>(omb + r * kOmStride + 2 * c2) = omr[i];
      }
    }
  };

  for (int e = tid; e < 2 * MT * 16 * kOmStride; e += 64 * NW) (&om[0][0])[e] = 0.0;

  f64x4 acc[MT][TN];
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int u = 0; u < TN; ++u) acc[t][u] = f64x4{0.0, 0.0, 0.0, 0.0};

  auto load_full = [&](int64_t k0, double (&a)[TN][8]) {
#pragma unroll
    for (int u = 0; u < TN; ++u)
      load_pieces_full<TA, 4, 2, 8, VEC>(ln.cb[u], k0 + 2 * g, ln.ok[u], a[u]);
  };
  auto mfma_chunk = [&](const double* __restrict__ omb, double (&a)[TN][8]) {
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      double ov[8];
      const double* orow = omb + (16 * t + r16) * kOmStride + 2 * g;
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const f64x2 pv = *reinterpret_cast<const f64x2*>(orow + 8 * h);
        ov[2 * h] = pv[0];
        ov[2 * h + 1] = pv[1];
      }
#pragma unroll
      for (int s = 0; s < 8; ++s)
#pragma unroll
        for (int u = 0; u < TN; ++u) acc[t][u] = mfma_f64(ov[s], a[u][s], acc[t][u]);
    }
  };

  const int64_t nfull = (it.r1 - it.r0) / kKC;
  const int64_t klast = it.r0 + (nfull - 1) * kKC;      // start of the last full chunk
  double a0[TN][8], a1[TN][8];
  __syncthreads();                                      // zero fill before generation
  if (nfull > 0) {
    load_full(it.r0, a0);
    fill_om(om[0], it.r0);
  }
  lds_barrier();
  // one pipeline step: prefetch (clamped: redundant on the last chunk), Omega of
  // the next chunk, MFMAs of this chunk
  auto step = [&](double (&cur)[TN][8], double (&nxt)[TN][8], int b, int64_t k0) {
    const int64_t k1 = min(k0 + kKC, klast);
    if (omtab) {
      om_load(k1);
      load_full(k1, nxt);
      mfma_chunk(om[b], cur);
      om_store(om[b ^ 1]);
    } else {
      load_full(k1, nxt);
      fill_om(om[b ^ 1], k1);
      mfma_chunk(om[b], cur);
    }
    lds_barrier();
  };
  int64_t c = 0;
  for (; c + 2 <= nfull; c += 2) {
    step(a0, a1, 0, it.r0 + c * kKC);
    step(a1, a0, 1, it.r0 + (c + 1) * kKC);
  }
  if (c < nfull) step(a0, a1, 0, it.r0 + c * kKC);
  // ragged last chunk
  const int64_t kt = it.r0 + nfull * kKC;
  if (kt < it.r1) {
    const int b = (int)(nfull & 1);
    fill_om(om[b], kt);
#pragma unroll
    for (int u = 0; u < TN; ++u)
      load_pieces_tail<TA, 4, 2, 8>(ln.cb[u], kt + 2 * g, it.r1, ln.ok[u], a0[u]);
    lds_barrier();
    mfma_chunk(om[b], a0);
  }
  // epilogue: lane holds rows 16t + g + 4v of column cwave + 16u + r16
  const bool direct = ST ? it.gnsplit == 1 : bi.nsplit == 1;
  double* dst = direct ? Y : part;
#pragma unroll
  for (int u = 0; u < TN; ++u) {
    if (!ln.ok[u]) continue;
    const int64_t ob = sk_out_offset<TA, TN, NW * 16 * TN, ST>(blks, perm, bi, it, ln, u, l, jst);
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * t + g + 4 * v;
        if (row < l) dst[ob + row] = acc[t][u][v];
      }
  }
}

// ---------------------------------------------------------------------------
// Loads of A in whole 128-byte lines.  A load instruction whose lanes read
// only 64 contiguous bytes of each column (four lanes per column, the MFMA
// operand layout) streams at about 5.4 TB/s on MI355X; one whose eight lanes
// per column read a whole 128-byte line reaches about 7 TB/s.  So a wave
// loads each 32-row chunk of its 16-column tiles as two instructions per
// tile: instruction h covers columns 8h..8h+7 of the tile, lane
// (c8 = lane / 8, p = lane % 8) reading rows 4p..4p+3 of column 8h + c8
// (FP64 A: rows 2p, 2p+1 and 16+2p, 17+2p, two 16-byte loads), and passes
// them through a wave-private LDS tile into the MFMA operand layout.  No
// barrier: a wave's LDS operations run in order.
//
// The staged column is one 128-byte line whose eight 16-byte pieces are
// permuted: piece q of column c sits at position q ^ line_swz(c).  Both the
// writes (eight lanes per column) and the operand reads (sixteen columns,
// one piece each) then touch distinct banks in every group of 8 lanes (32
// banks) and of 16 lanes (64 banks).
// ---------------------------------------------------------------------------
constexpr int kLineSt = kKC;   // floats per staged column

__device__ __forceinline__ int line_swz(int col) { return ((col >> 1) ^ (col << 2)) & 7; }

__device__ __forceinline__ float* line_piece(float* st, int col, int q) {
  return st + col * kLineSt + 4 * (q ^ line_swz(col));
}

template <typename TA, int TN>
struct SkLines {
  gptr<TA> cb[TN][2];   // load column starts (an invalid column: a valid stand-in)
};

// lane's load columns of a batch item: tile u, instruction h -> column
// cwave + 16 u + 8 h + lane / 8
template <typename TA, int TN>
__device__ __forceinline__ void sk_lines(const BlkInfo& bi, int cwave, int lane, int j0, int j1,
                                         SkLines<TA, TN>& ld) {
  const int clo = max(j0, 0), chi = min(j1, bi.n);
  gptr<TA> A = (gptr<TA>)bi.A;
#pragma unroll
  for (int u = 0; u < TN; ++u)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int col = cwave + 16 * u + 8 * h + (lane >> 3);
      const bool ok = col >= clo && col < chi;
      ld.cb[u][h] = A + (int64_t)(ok ? col : clo) * bi.lda;
    }
}

// the same for a one-snapshot item (column = block perm[c0 + local], snapshot j)
template <typename TA, int TN>
__device__ __forceinline__ void sk_lines_stream(const BlkInfo* __restrict__ blks,
                                                const int32_t* __restrict__ perm, const SkItem& it,
                                                int cw, int lane, int j, SkLines<TA, TN>& ld) {
#pragma unroll
  for (int u = 0; u < TN; ++u)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int local = cw + 16 * u + 8 * h + (lane >> 3);
      const bool valid = local < it.gsize;
      const BlkInfo& bb = blks[perm[it.c0 + (valid ? local : 0)]];
      const bool ok = valid && j < bb.n;
      ld.cb[u][h] = (gptr<TA>)bb.A + (int64_t)(ok ? j : 0) * bb.lda;
    }
}

// One line piece: rows row + 4p .. +3 (FP64: row + 2p, +1, row + 16 + 2p, +1)
// of a full chunk, straight-line loads.  An invalid column reads its clamped
// stand-in unmasked: an MFMA output column depends on its own input column
// only, and invalid output columns are never stored.
template <typename TA, bool VEC>
__device__ __forceinline__ void load_line(gptr<TA> __restrict__ cb, int64_t row, int p,
                                          float (&x)[4]) {
  // VEC: 16-byte aligned column starts, streaming (non-temporal) loads.
  // Otherwise element-aligned vector loads through the caches: a chunk of a
  // column that does not start on a 128-byte line shares its first and last
  // lines with the neighbouring chunks, which then hit in L2 instead of being
  // fetched twice.
  if constexpr (sizeof(TA) == 4) {
    if constexpr (VEC) {
      const f32x4 v = __builtin_nontemporal_load((gptr<f32x4>)(cb + row + 4 * p));
#pragma unroll
      for (int e = 0; e < 4; ++e) x[e] = v[e];
    } else {
      const f32x4u v = *(gptr<f32x4u>)(cb + row + 4 * p);
#pragma unroll
      for (int e = 0; e < 4; ++e) x[e] = v[e];
    }
  } else {
    if constexpr (VEC) {
      const f64x2 v0 = __builtin_nontemporal_load((gptr<f64x2>)(cb + row + 2 * p));
      const f64x2 v1 = __builtin_nontemporal_load((gptr<f64x2>)(cb + row + 16 + 2 * p));
      x[0] = (float)v0[0];
      x[1] = (float)v0[1];
      x[2] = (float)v1[0];
      x[3] = (float)v1[1];
    } else {
      const f64x2u v0 = *(gptr<f64x2u>)(cb + row + 2 * p);
      const f64x2u v1 = *(gptr<f64x2u>)(cb + row + 16 + 2 * p);
      x[0] = (float)v0[0];
      x[1] = (float)v0[1];
      x[2] = (float)v1[0];
      x[3] = (float)v1[1];
    }
  }
}

// ragged chunk (cb = column start, row and rend absolute): rows at or past
// rend read row 0 and are zeroed (no branches, so the loads overlap)
template <typename TA>
__device__ __forceinline__ void load_line_tail(gptr<TA> __restrict__ cb, int64_t row, int64_t rend,
                                               int p, float (&x)[4]) {
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int64_t r = sizeof(TA) == 4 ? row + 4 * p + e : row + 16 * (e >> 1) + 2 * p + (e & 1);
    const float v = (float)cb[r < rend ? r : 0];
    x[e] = r < rend ? v : 0.0f;
  }
}

// a lane's piece into column col of the wave's tile
template <typename TA>
__device__ __forceinline__ void stage_line(float* __restrict__ st, int col, int p,
                                           const float (&x)[4]) {
  if constexpr (sizeof(TA) == 4) {
    *reinterpret_cast<f32x4*>(line_piece(st, col, p)) = f32x4{x[0], x[1], x[2], x[3]};
  } else {
    // rows 2p, 2p+1 (piece p / 2) and 16 + 2p, 17 + 2p (piece 4 + p / 2)
    *reinterpret_cast<f32x2*>(line_piece(st, col, p >> 1) + 2 * (p & 1)) = f32x2{x[0], x[1]};
    *reinterpret_cast<f32x2*>(line_piece(st, col, 4 + (p >> 1)) + 2 * (p & 1)) = f32x2{x[2], x[3]};
  }
}

// ---------------------------------------------------------------------------
// Sketch, bfloat16 (FP32 accumulation): Omega rounded to nearest-even
// bfloat16; A split into `terms` bfloat16 terms in registers
// (hi = bf16(a), lo = bf16(a - hi), lo2 = bf16(a - hi - lo));
// v_mfma_f32_16x16x32_bf16.  The k-values of lane (g, r16) are rows
// 8g..8g+7 of the chunk, of its column r16 (from the staged lines) and of
// Omega row 16t + r16.
//
// Omega shared by all blocks (TAB): regenerated once per sketch update by
// omega_table_kernel into a small table (l x max m_b, resident in L2) already
// in MFMA operand order (16 bytes per lane and tile, one coalesced load per
// tile), instead of once per work item and chunk; software-pipelined with A
// in registers, the waves run without barriers.  Omega keyed per block (!TAB): regenerated
// per 32-row chunk into LDS, double-buffered like A, one LDS-only barrier per
// chunk.  The ragged last chunk is handled after the loop.
// ---------------------------------------------------------------------------
// Table entry of Omega row r, column i (sketch-matrix column = A row): chunk
// i / 32, tile r / 16, lane 16 g + r % 16 with g = (i % 32) / 8, element i % 8;
// 8 bfloat16 per lane.
__host__ __device__ constexpr int64_t omega_tab_index(int MT, int r, int64_t i) {
  return (((i >> 5) * MT + (r >> 4)) * 64 + 16 * ((i & 31) >> 3) + (r & 15)) * 8 + (i & 7);
}

// The table: MT*16 rows (rows l.. zero) x ncols columns (a multiple of 32),
// one thread per pair of rows and column, values of omega_pair_rounded.
template <int KIND>
__global__ __launch_bounds__(256) void omega_table_kernel(int l, int MT, int64_t ncols,
                                                          uint64_t seed, __bf16* __restrict__ tab) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)MT * 8 * ncols) return;
  const int q = (int)(e / ncols);
  const int64_t i = e - (int64_t)q * ncols;
  float z0 = 0.0f, z1 = 0.0f;
  if (2 * q < l) omega_pair_rounded<KIND>(seed, 0u, (uint32_t)i, (uint32_t)q, z0, z1);
  if (2 * q + 1 >= l) z1 = 0.0f;
  tab[omega_tab_index(MT, 2 * q, i)] = to_bf16(z0);
  tab[omega_tab_index(MT, 2 * q + 1, i)] = to_bf16(z1);
}

template <typename TA, int MT, int TN, int NW, bool VEC, bool ST, bool TAB>
__global__ __launch_bounds__(64 * NW) void sketch_bf16_kernel(
    const BlkInfo* __restrict__ blks, const SkItem* __restrict__ items, int l, uint64_t seed,
    int omega_per_block, int j0, int j1, const int32_t* __restrict__ perm, int jst, int terms,
    const bf16x8* __restrict__ omtab, float* __restrict__ Y, float* __restrict__ part) {
  constexpr int kS = kKC + 8;   // LDS row stride of the generated Omega (bf16, 80 bytes)
  __shared__ __attribute__((aligned(16))) __bf16 om[2][TAB ? 8 : MT * 16 * kS];
  __shared__ __attribute__((aligned(16))) float stage_all[NW * TN * 16 * kLineSt];
  const SkItem it = items[blockIdx.x];
  const BlkInfo bi = blks[it.blk];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, r16 = lane & 15, p8 = lane & 7;
  const int cwave = it.c0 + wave * 16 * TN;
  SkLane<TA, TN> ln;      // output columns (lane column r16 of each tile)
  SkLines<TA, TN> ld;     // load columns
  if constexpr (ST) {
    sk_setup_stream<TA, TN>(blks, perm, it, wave * 16 * TN, r16, jst, ln);
    sk_lines_stream<TA, TN>(blks, perm, it, wave * 16 * TN, lane, jst, ld);
  } else {
    if (!sk_setup<TA, TN>(bi, it, cwave, r16, NW * 16 * TN, j0, j1, ln)) return;
    sk_lines<TA, TN>(bi, cwave, lane, j0, j1, ld);
  }
  const uint32_t bkey = omega_per_block ? (uint32_t)(it.blk + 1) : 0u;
  float* __restrict__ st = stage_all + wave * TN * 16 * kLineSt;

  if constexpr (!TAB)
    for (int e = tid; e < 2 * MT * 16 * kS; e += 64 * NW) (&om[0][0])[e] = (__bf16)0.0f;

  f32x4 acc[MT][TN];
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int u = 0; u < TN; ++u) acc[t][u] = f32x4{0.f, 0.f, 0.f, 0.f};

  auto load_full = [&](int64_t k0, float (&a)[TN][2][4]) {
#pragma unroll
    for (int u = 0; u < TN; ++u)
#pragma unroll
      for (int h = 0; h < 2; ++h) load_line<TA, VEC>(ld.cb[u][h], k0, p8, a[u][h]);
  };
  auto load_tail = [&](int64_t k0, float (&a)[TN][2][4]) {
#pragma unroll
    for (int u = 0; u < TN; ++u)
#pragma unroll
      for (int h = 0; h < 2; ++h)
        load_line_tail<TA>(ld.cb[u][h], k0, it.r1, p8, a[u][h]);
  };
  // lines -> LDS -> operand layout (rows 8g..8g+7 of column r16 of each tile)
  auto transpose = [&](const float (&a)[TN][2][4], float (&b)[TN][8]) {
#pragma unroll
    for (int u = 0; u < TN; ++u)
#pragma unroll
      for (int h = 0; h < 2; ++h) stage_line<TA>(st, 16 * u + 8 * h + (lane >> 3), p8, a[u][h]);
#pragma unroll
    for (int u = 0; u < TN; ++u) {
      const f32x4 lo = *reinterpret_cast<const f32x4*>(line_piece(st, 16 * u + r16, 2 * g));
      const f32x4 hi = *reinterpret_cast<const f32x4*>(line_piece(st, 16 * u + r16, 2 * g + 1));
      b[u][0] = lo[0];
      b[u][1] = lo[1];
      b[u][2] = lo[2];
      b[u][3] = lo[3];
      b[u][4] = hi[0];
      b[u][5] = hi[1];
      b[u][6] = hi[2];
      b[u][7] = hi[3];
    }
  };
  // A split into `terms` (1..3) bfloat16 terms and the MFMAs of every term.
  // Each pair of values is rounded by one packed conversion; the terms'
  // values are read back from its halves by shifts, and the last term forms
  // no remainder (uniform branches on the term count).
  auto split_mfma = [&](const bf16x8 (&oa)[MT], const float (&a)[TN][2][4]) {
    float b[TN][8];
    transpose(a, b);
#pragma unroll
    for (int u = 0; u < TN; ++u) {
      float rem[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) rem[e] = b[u][e];
#pragma unroll
      for (int h = 0; h < 3; ++h) {
        if (h >= terms) break;
        uint32_t w[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) w[e] = pack_bf16x2(rem[2 * e], rem[2 * e + 1]);
        if (h + 1 < terms) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            rem[2 * e] -= __uint_as_float(w[e] << 16);
            rem[2 * e + 1] -= __uint_as_float(w[e] & 0xffff0000u);
          }
        }
        const bf16x8 bt = __builtin_bit_cast(bf16x8, i32x4{(int)w[0], (int)w[1], (int)w[2],
                                                            (int)w[3]});
#pragma unroll
        for (int t = 0; t < MT; ++t) acc[t][u] = mfma_bf16(oa[t], bt, acc[t][u]);
      }
    }
  };
  auto mfma_chunk = [&](const __bf16* __restrict__ omb, const float (&a)[TN][2][4]) {
    bf16x8 oa[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t)
      oa[t] = *reinterpret_cast<const bf16x8*>(omb + (16 * t + r16) * kS + 8 * g);
    split_mfma(oa, a);
  };

  const int64_t nfull = (it.r1 - it.r0) / kKC;
  const int64_t klast = it.r0 + (nfull - 1) * kKC;
  const int64_t kt = it.r0 + nfull * kKC;
  float a0[TN][2][4], a1[TN][2][4];
  if constexpr (TAB) {
    const bf16x8* __restrict__ ot = omtab + lane;
    auto load_om = [&](int64_t k0, bf16x8 (&o)[MT]) {
#pragma unroll
      for (int t = 0; t < MT; ++t) o[t] = ot[((k0 >> 5) * MT + t) * 64];
    };
    bf16x8 o0[MT], o1[MT];
    if (nfull > 0) {
      load_full(it.r0, a0);
      load_om(it.r0, o0);
    }
    auto step = [&](float (&cur)[TN][2][4], float (&nxt)[TN][2][4], bf16x8 (&ocur)[MT],
                    bf16x8 (&onxt)[MT], int64_t k0) {
      const int64_t k1 = min(k0 + kKC, klast);
      load_full(k1, nxt);
      load_om(k1, onxt);
      split_mfma(ocur, cur);
    };
    int64_t c = 0;
    for (; c + 2 <= nfull; c += 2) {
      step(a0, a1, o0, o1, it.r0 + c * kKC);
      step(a1, a0, o1, o0, it.r0 + (c + 1) * kKC);
    }
    if (c < nfull) step(a0, a1, o0, o1, it.r0 + c * kKC);
    if (kt < it.r1) {
      load_om(kt, o0);
      load_tail(kt, a0);
      split_mfma(o0, a0);
    }
  } else {
    __syncthreads();
    if (nfull > 0) {
      load_full(it.r0, a0);
      gen_omega_chunk_bf16<kS, 64 * NW>(om[0], l, seed, bkey, it.r0, tid);
    }
    lds_barrier();
    auto step = [&](float (&cur)[TN][2][4], float (&nxt)[TN][2][4], int b, int64_t k0) {
      const int64_t k1 = min(k0 + kKC, klast);
      load_full(k1, nxt);
      gen_omega_chunk_bf16<kS, 64 * NW>(om[b ^ 1], l, seed, bkey, k1, tid);
      mfma_chunk(om[b], cur);
      lds_barrier();
    };
    int64_t c = 0;
    for (; c + 2 <= nfull; c += 2) {
      step(a0, a1, 0, it.r0 + c * kKC);
      step(a1, a0, 1, it.r0 + (c + 1) * kKC);
    }
    if (c < nfull) step(a0, a1, 0, it.r0 + c * kKC);
    if (kt < it.r1) {
      const int b = (int)(nfull & 1);
      gen_omega_chunk_bf16<kS, 64 * NW>(om[b], l, seed, bkey, kt, tid);
      load_tail(kt, a0);
      lds_barrier();
      mfma_chunk(om[b], a0);
    }
  }
  const bool direct = ST ? it.gnsplit == 1 : bi.nsplit == 1;
  float* dst = direct ? Y : part;
#pragma unroll
  for (int u = 0; u < TN; ++u) {
    if (!ln.ok[u]) continue;
    const int64_t ob = sk_out_offset<TA, TN, NW * 16 * TN, ST>(blks, perm, bi, it, ln, u, l, jst);
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * t + 4 * g + v;
        if (row < l) dst[ob + row] = acc[t][u][v];
      }
  }
}

// ---------------------------------------------------------------------------
// Sketch, OCP fp8 e4m3 (FP32 accumulation) on
// v_mfma_scale_f32_16x16x128_f8f6f4.  Omega is the double-precision normal
// rounded to nearest-even e4m3 (|Omega| < 448, scale 1).  A chunk is 128 rows
// (one MFMA k-step); every 32 consecutive rows of a column form one scaling
// block: per split term its power of two 2^E (max|residual| * 2^-E < 256) is
// agreed between the two lanes holding its halves, passed as the E8M0 operand
// scale of the product, the residual * 2^-E is rounded to e4m3 and what it
// represented is subtracted.  Omega is double-buffered in LDS as bytes.
// ---------------------------------------------------------------------------
constexpr int kKC8 = 128;
constexpr int kOm8Stride = kKC8 + 16;   // bytes per Omega row in LDS

// position of chunk row kk (0..127) in an Omega row of the chunk (the k
// layout below)
__host__ __device__ constexpr int fp8_kpos(int kk) {
  return (kk & ~63) | (((kk >> 2) & 3) << 4) | (((kk >> 4) & 3) << 2) | (kk & 3);
}

// Shared e4m3 Omega for the one-snapshot updates, regenerated once per update,
// in the f8f6f4 A-operand order of sketch_fp8_stream_kernel: chunk c (A rows
// 128c..), tile t, lane 16 g + r (Omega row 16t + r), 32 bytes: k = 16g..16g+15
// then 64+16g..64+16g+15 of the chunk, k = the A row within the chunk.  Rows
// l.. zero.  One thread per pair of Omega rows and A row.
__host__ __device__ constexpr int64_t omega_tab8_index(int MT, int r, int64_t i) {
  return (((i >> 7) * MT + (r >> 4)) * 64 + 16 * ((i >> 4) & 3) + (r & 15)) * 32 +
         16 * ((i >> 6) & 1) + (i & 15);
}

template <typename TB>   // uint8_t
__global__ __launch_bounds__(256) void omega_table_e4m3_kernel(int l, int MT, int64_t ncols,
                                                               uint64_t seed, TB* __restrict__ tab) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)MT * 8 * ncols) return;
  const int q = (int)(e / ncols);
  const int64_t i = e - (int64_t)q * ncols;
  float z0 = 0.0f, z1 = 0.0f;
  if (2 * q < l) omega_pair_rounded<1>(seed, 0u, (uint32_t)i, (uint32_t)q, z0, z1);
  if (2 * q + 1 >= l) z1 = 0.0f;
  tab[omega_tab8_index(MT, 2 * q, i)] = (TB)to_e4m3_byte(z0);
  tab[omega_tab8_index(MT, 2 * q + 1, i)] = (TB)to_e4m3_byte(z1);
}

template <int NTHR>
__device__ __forceinline__ void gen_omega_chunk_e4m3(uint8_t* __restrict__ om, int l,
                                                     uint64_t seed, uint32_t bkey, int64_t k0,
                                                     int tid) {
  const int npairs = (l + 1) >> 1;
  for (int e = tid; e < npairs * kKC8; e += NTHR) {
    const int q = e / kKC8, kk = e - q * kKC8;
    float z0, z1;
    omega_pair_rounded<1>(seed, bkey, (uint32_t)(k0 + kk), (uint32_t)q, z0, z1);
    // chunk row kk = 64 h + 16 w + 4 g + x sits at k = 64 h + 16 g + 4 w + x
    const int kpos = fp8_kpos(kk);
    om[(2 * q) * kOm8Stride + kpos] = (uint8_t)to_e4m3_byte(z0);
    if (2 * q + 1 < l) om[(2 * q + 1) * kOm8Stride + kpos] = (uint8_t)to_e4m3_byte(z1);
  }
}

// The f8f6f4 16x16x128 operand layout (checked on the device): lane group g
// = lane/16 holds k = 16g..16g+15 in bytes 0..15 and k = 64+16g..64+16g+15 in
// bytes 16..31; the E8M0 scale of K block kb (k = 32kb..32kb+31) for row or
// column c is taken from lane c + 16 kb.  Chunk row r = 64h + 16w + 4g + x
// is placed at k = 64h + 16g + 4w + x, so lane g's sixteen k-values of a half
// are rows 4g..4g+3 of each 16-row group (64 contiguous bytes per column and
// load instruction); Omega is stored in LDS at the same k positions.

// Power-of-two exponent E with amax * 2^-E < 256 (<= 448, the e4m3 maximum);
// -127 for an all-zero block.
__device__ __forceinline__ int fp8_block_exp(float amax) {
  if (!(amax > 0.0f)) return -127;
  int ex;
  frexpf(amax, &ex);   // amax < 2^ex
  return max(ex - 8, -127);
}

// The split terms of a lane's 32 values (two 16-value halves, each in its own
// 32-row K block).  Term h of a K block is taken at the power of two
// 2^(E - 4h), E from the block maximum (amax * 2^-E < 256): rounding to e4m3
// leaves at most 1/16 of a value's own binade, so every later residual times
// 2^-(E - 4h) stays below 256 too and no term saturates.  fp8_block_scales
// finds E for the lane's two halves (the block maxima are combined over the
// two lanes holding each block) and the exponent of the K block g that this
// lane's scale operand supplies to the MFMA; fp8_term forms one term: e4m3
// bytes packed 4 per int (v_cvt_scalef32_pk_fp8_f32: x / 2^E' rounded to
// nearest even) and, unless it is the last term, what it represents
// (v_cvt_scalef32_pk_f32_fp8: byte * 2^E') taken off the residual.
struct Fp8Scales {
  int e_first, e_second;   // exponents of the lane's two K blocks
  int e_g;                 // exponent of K block g (the lane's MFMA scale)
};

__device__ __forceinline__ Fp8Scales fp8_block_scales(const float res[32], int g) {
  float h0 = 0.0f, h1 = 0.0f;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    h0 = fmaxf(h0, fabsf(res[e]));
    h1 = fmaxf(h1, fabsf(res[16 + e]));
  }
  // block maxima: first halves of lane groups {0,1} -> block 0, {2,3} -> block 1,
  // second halves {0,1} -> block 2, {2,3} -> block 3
  h0 = fmaxf(h0, __shfl_xor(h0, 16, kWave));
  h1 = fmaxf(h1, __shfl_xor(h1, 16, kWave));
  const float o0 = __shfl_xor(h0, 32, kWave);
  const float o1 = __shfl_xor(h1, 32, kWave);
  const bool lo_pair = g < 2;
  const float b0 = lo_pair ? h0 : o0, b1 = lo_pair ? o0 : h0;
  const float b2 = lo_pair ? h1 : o1, b3 = lo_pair ? o1 : h1;
  Fp8Scales sc;
  sc.e_first = fp8_block_exp(lo_pair ? b0 : b1);
  sc.e_second = fp8_block_exp(lo_pair ? b2 : b3);
  sc.e_g = fp8_block_exp(g == 0 ? b0 : (g == 1 ? b1 : (g == 2 ? b2 : b3)));
  return sc;
}

__device__ __forceinline__ i32x8 fp8_term(float res[32], const Fp8Scales& sc, int h,
                                          bool rem_needed) {
  typedef short s16x2 __attribute__((ext_vector_type(2)));
  i32x8 out;
#pragma unroll
  for (int hh = 0; hh < 2; ++hh) {
    const float scale = ldexpf(1.0f, max((hh ? sc.e_second : sc.e_first) - 4 * h, -127));
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int e = 16 * hh + 4 * w;
      s16x2 pk = s16x2{0, 0};
      pk = __builtin_amdgcn_cvt_scalef32_pk_fp8_f32(pk, res[e], res[e + 1], scale, false);
      pk = __builtin_amdgcn_cvt_scalef32_pk_fp8_f32(pk, res[e + 2], res[e + 3], scale, true);
      out[4 * hh + w] = __builtin_bit_cast(int, pk);
    }
    if (rem_needed) {
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const int e = 16 * hh + 4 * w;
        const f32x2 q0 = __builtin_amdgcn_cvt_scalef32_pk_f32_fp8(out[4 * hh + w], scale, false);
        const f32x2 q1 = __builtin_amdgcn_cvt_scalef32_pk_f32_fp8(out[4 * hh + w], scale, true);
        res[e] -= q0[0];
        res[e + 1] -= q0[1];
        res[e + 2] -= q1[0];
        res[e + 3] -= q1[1];
      }
    }
  }
  return out;
}

// E8M0 scale byte of term h for the lane's K block g
__device__ __forceinline__ int fp8_scale_byte(const Fp8Scales& sc, int h) {
  return max(sc.e_g - 4 * h, -127) + 127;
}

template <typename TA, int MT, int TN, int NW, bool VEC, bool ST>
__global__ __launch_bounds__(64 * NW) void sketch_fp8_kernel(
    const BlkInfo* __restrict__ blks, const SkItem* __restrict__ items, int l, uint64_t seed,
    int omega_per_block, int j0, int j1, const int32_t* __restrict__ perm, int jst, int terms,
    float* __restrict__ Y, float* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) uint8_t om[2][MT * 16 * kOm8Stride];
  const SkItem it = items[blockIdx.x];
  const BlkInfo bi = blks[it.blk];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, r16 = lane & 15;
  const int cwave = it.c0 + wave * 16 * TN;
  SkLane<TA, TN> ln;
  if constexpr (ST) {
    sk_setup_stream<TA, TN>(blks, perm, it, wave * 16 * TN, r16, jst, ln);
  } else {
    if (!sk_setup<TA, TN>(bi, it, cwave, r16, NW * 16 * TN, j0, j1, ln)) return;
  }
  const uint32_t bkey = omega_per_block ? (uint32_t)(it.blk + 1) : 0u;

  for (int e = tid; e < 2 * MT * 16 * kOm8Stride; e += 64 * NW) (&om[0][0])[e] = 0;

  f32x4 acc[MT][TN];
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int u = 0; u < TN; ++u) acc[t][u] = f32x4{0.f, 0.f, 0.f, 0.f};

  // the lane's two 16-row runs: k0 + 16g and k0 + 64 + 16g
  auto load_full = [&](int64_t k0, float (&a)[TN][32]) {
#pragma unroll
    for (int u = 0; u < TN; ++u) {
      load_pieces_full<TA, 4, 4, 16, VEC>(ln.cb[u], k0 + 4 * g, ln.ok[u], a[u]);
      load_pieces_full<TA, 4, 4, 16, VEC>(ln.cb[u], k0 + 64 + 4 * g, ln.ok[u], a[u] + 16);
    }
  };
  auto mfma_chunk = [&](const uint8_t* __restrict__ omb, float (&a)[TN][32]) {
    i32x8 oa[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      const uint8_t* orow = omb + (16 * t + r16) * kOm8Stride;
      const i32x4 lo = *reinterpret_cast<const i32x4*>(orow + 16 * g);
      const i32x4 hi = *reinterpret_cast<const i32x4*>(orow + 64 + 16 * g);
      oa[t] = i32x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    }
#pragma unroll
    for (int u = 0; u < TN; ++u) {
      const Fp8Scales sc = fp8_block_scales(a[u], g);
      for (int h = 0; h < terms; ++h) {
        const i32x8 bt = fp8_term(a[u], sc, h, h + 1 < terms);
        const int sb = fp8_scale_byte(sc, h);
#pragma unroll
        for (int t = 0; t < MT; ++t) acc[t][u] = mfma_fp8_scaled(oa[t], bt, acc[t][u], 127, sb);
      }
    }
  };

  const int64_t nfull = (it.r1 - it.r0) / kKC8;
  const int64_t klast = it.r0 + (nfull - 1) * kKC8;
  float a0[TN][32], a1[TN][32];
  __syncthreads();
  if (nfull > 0) {
    load_full(it.r0, a0);
    gen_omega_chunk_e4m3<64 * NW>(om[0], l, seed, bkey, it.r0, tid);
  }
  lds_barrier();
  auto step = [&](float (&cur)[TN][32], float (&nxt)[TN][32], int b, int64_t k0) {
    const int64_t k1 = min(k0 + kKC8, klast);
    load_full(k1, nxt);
    gen_omega_chunk_e4m3<64 * NW>(om[b ^ 1], l, seed, bkey, k1, tid);
    mfma_chunk(om[b], cur);
    lds_barrier();
  };
  int64_t c = 0;
  for (; c + 2 <= nfull; c += 2) {
    step(a0, a1, 0, it.r0 + c * kKC8);
    step(a1, a0, 1, it.r0 + (c + 1) * kKC8);
  }
  if (c < nfull) step(a0, a1, 0, it.r0 + c * kKC8);
  const int64_t kt = it.r0 + nfull * kKC8;
  if (kt < it.r1) {
    const int b = (int)(nfull & 1);
    gen_omega_chunk_e4m3<64 * NW>(om[b], l, seed, bkey, kt, tid);
#pragma unroll
    for (int u = 0; u < TN; ++u) {
      load_pieces_tail<TA, 4, 4, 16>(ln.cb[u], kt + 4 * g, it.r1, ln.ok[u], a0[u]);
      load_pieces_tail<TA, 4, 4, 16>(ln.cb[u], kt + 64 + 4 * g, it.r1, ln.ok[u], a0[u] + 16);
    }
    lds_barrier();
    mfma_chunk(om[b], a0);
  }
  const bool direct = ST ? it.gnsplit == 1 : bi.nsplit == 1;
  float* dst = direct ? Y : part;
#pragma unroll
  for (int u = 0; u < TN; ++u) {
    if (!ln.ok[u]) continue;
    const int64_t ob = sk_out_offset<TA, TN, NW * 16 * TN, ST>(blks, perm, bi, it, ln, u, l, jst);
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * t + 4 * g + v;
        if (row < l) dst[ob + row] = acc[t][u][v];
      }
  }
}

// ---------------------------------------------------------------------------
// One-snapshot FP8 update (FP32 data).  A work item is `cnt` groups of up to
// 128 equal-m blocks (stream items first, first + stride, ...); wave w takes
// blocks 16w..16w+15 of a group, column j of each, over all of K (no K split,
// so no partial sketches and no reduction launch).  Per 128-row chunk the
// wave loads its 16 columns as whole 128-byte lines (8 lanes per column: four
// lines x two halves of 8 columns), passes them through its LDS tile into the
// f8f6f4 B-operand layout (lane (g, c): rows 16g..16g+15 and 64+16g..64+16g+15
// of column c, k = the row), and reads its Omega operands from the update's
// table (omega_table_e4m3_kernel: 32 bytes per lane and tile, L2-resident)
// ahead of the next chunk's lines, so that waiting for Omega does not wait
// for them.  No barriers.
//
// A staged column is 128 floats (512 bytes, 32 pieces of 16); piece q sits at
// (q & 16) | ((q & 15) ^ s(c)) with s(c) = 8 (c & 1) + c / 2 (c < 16): the 16
// columns of a read and the two columns of every 16-lane write phase then hit
// distinct banks.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int fp8_piece_pos(int q, int col) {
  return (q & 16) | ((q & 15) ^ (((col & 1) << 3) | ((col >> 1) & 7)));
}

template <int MT, int NW, bool VEC>
__global__ __launch_bounds__(64 * NW) void sketch_fp8_stream_kernel(
    const BlkInfo* __restrict__ blks, const SkItem* __restrict__ sitems,
    const int32_t* __restrict__ ritems, int l, const i32x4* __restrict__ omtab,
    const int32_t* __restrict__ perm, int jst, int terms, float* __restrict__ Y) {
  __shared__ __attribute__((aligned(16))) float stage_all[NW * 16 * kKC8];
  const int first = ritems[3 * blockIdx.x], cnt = ritems[3 * blockIdx.x + 1];
  const int stride = ritems[3 * blockIdx.x + 2];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, r16 = lane & 15, p8 = lane & 7, c8 = lane >> 3;
  float* __restrict__ st = stage_all + wave * 16 * kKC8;
  const i32x4* __restrict__ ot = omtab + 2 * lane;
  for (int gi = 0; gi < cnt; ++gi) {
    const SkItem it = sitems[first + gi * stride];
    SkLane<float, 1> ln;   // output column: block perm[c0 + 16 wave + r16]
    sk_setup_stream<float, 1>(blks, perm, it, wave * 16, r16, jst, ln);
    SkLines<float, 1> ld;  // load columns: blocks 16 wave + 8 h + c8
    sk_lines_stream<float, 1>(blks, perm, it, wave * 16, lane, jst, ld);
    f32x4 acc[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    // lines L = 0..3 of half h: rows k0 + 32 L + 4 p8 .. +3 of load column h
    auto load_full = [&](int64_t k0, float (&x)[2][4][4]) {
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int L = 0; L < 4; ++L) load_line<float, VEC>(ld.cb[0][h], k0 + 32 * L, p8, x[h][L]);
    };
    auto load_tail = [&](int64_t k0, float (&x)[2][4][4]) {
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int L = 0; L < 4; ++L)
          load_line_tail<float>(ld.cb[0][h], k0 + 32 * L, it.r1, p8, x[h][L]);
    };
    auto load_om = [&](int64_t k0, i32x8 (&o)[MT]) {
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        const i32x4* q = ot + ((k0 >> 7) * MT + t) * 128;
        const i32x4 lo = q[0], hi = q[1];
        o[t] = i32x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
      }
    };
    // stage the chunk's lines, read back the operand layout, split and multiply
    auto chunk = [&](const float (&x)[2][4][4], const i32x8 (&oa)[MT]) {
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int L = 0; L < 4; ++L) {
          const int col = 8 * h + c8;
          *reinterpret_cast<f32x4*>(st + col * kKC8 + 4 * fp8_piece_pos(8 * L + p8, col)) =
              f32x4{x[h][L][0], x[h][L][1], x[h][L][2], x[h][L][3]};
        }
      float a[32];
#pragma unroll
      for (int hf = 0; hf < 2; ++hf)
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          const f32x4 v = *reinterpret_cast<const f32x4*>(
              st + r16 * kKC8 + 4 * fp8_piece_pos(16 * hf + 4 * g + w, r16));
#pragma unroll
          for (int e = 0; e < 4; ++e) a[16 * hf + 4 * w + e] = v[e];
        }
      const Fp8Scales sc = fp8_block_scales(a, g);
      for (int h = 0; h < terms; ++h) {
        const i32x8 bt = fp8_term(a, sc, h, h + 1 < terms);
        const int sb = fp8_scale_byte(sc, h);
#pragma unroll
        for (int t = 0; t < MT; ++t) acc[t] = mfma_fp8_scaled(oa[t], bt, acc[t], 127, sb);
      }
    };
    const int64_t nfull = (it.r1 - it.r0) / kKC8;
    const int64_t klast = it.r0 + (nfull - 1) * kKC8;
    const int64_t kt = it.r0 + nfull * kKC8;
    float x0[2][4][4], x1[2][4][4];
    i32x8 oa[MT];
    if (nfull > 0) load_full(it.r0, x0);
    auto step = [&](const float (&cur)[2][4][4], float (&nxt)[2][4][4], int64_t k0) {
      load_om(k0, oa);                            // before the next lines: waited for first
      load_full(min(k0 + kKC8, klast), nxt);
      chunk(cur, oa);
    };
    int64_t c = 0;
    for (; c + 2 <= nfull; c += 2) {
      step(x0, x1, it.r0 + c * kKC8);
      step(x1, x0, it.r0 + (c + 1) * kKC8);
    }
    if (c < nfull) step(x0, x1, it.r0 + c * kKC8);
    if (kt < it.r1) {
      load_om(kt, oa);
      load_tail(kt, x0);
      chunk(x0, oa);
    }
    if (ln.ok[0]) {
      const BlkInfo bi = blks[it.blk];
      const int64_t ob = sk_out_offset<float, 1, NW * 16, true>(blks, perm, bi, it, ln, 0, l, jst);
#pragma unroll
      for (int t = 0; t < MT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 16 * t + 4 * g + v;
          if (row < l) Y[ob + row] = acc[t][v];
        }
    }
  }
}

// ---------------------------------------------------------------------------
// Split-K reduction: Y_b(:, j) = sum over splits s (ascending) of the
// partials, for the blocks listed in `split_blocks`, columns [j0, j1).
// grid = (ceil(l*maxn / 256), number of split blocks)
// ---------------------------------------------------------------------------
template <typename TY>
__global__ __launch_bounds__(256) void sketch_reduce_kernel(const BlkInfo* __restrict__ blks,
                                                            const int32_t* __restrict__ split_blocks,
                                                            int l, int j0, int j1,
                                                            TY* __restrict__ Y,
                                                            const TY* __restrict__ part) {
  const int b = split_blocks[blockIdx.y];
  const BlkInfo bi = blks[b];
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t total = (int64_t)l * bi.n;
  if (e >= total) return;
  const int col = (int)(e / l);
  if (col < j0 || col >= j1) return;
  const TY* p = part + bi.part_off + e;
  TY s = 0;
  for (int sp = 0; sp < bi.nsplit; ++sp) s += p[(int64_t)sp * total];
  Y[bi.y_off + e] = s;
}

// ---------------------------------------------------------------------------
// Stream-mode split-K reduction for snapshot j: for each listed group head
// (grid.y) and each (block of the group, sketch row) pair, sum the group's
// partials over its K ranges in ascending order into Y_b(:, j).
// ---------------------------------------------------------------------------
template <typename TY>
__global__ __launch_bounds__(256) void sketch_stream_reduce_kernel(
    const BlkInfo* __restrict__ blks, const int32_t* __restrict__ perm,
    const SkItem* __restrict__ items, const int32_t* __restrict__ heads, int l, int gcap, int j,
    TY* __restrict__ Y, const TY* __restrict__ part) {
  const SkItem it = items[heads[blockIdx.y]];
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)it.gsize * l) return;
  const int c = (int)(e / l), r = (int)(e - (int64_t)c * l);
  const BlkInfo bb = blks[perm[it.c0 + c]];
  if (j >= bb.n) return;
  TY s = 0;
  for (int sp = 0; sp < it.gnsplit; ++sp) s += part[it.gpart + ((int64_t)sp * gcap + c) * l + r];
  Y[bb.y_off + (int64_t)j * l + r] = s;
}

// ---------------------------------------------------------------------------
// Column selection with one barrier per step.  A group of LPC lanes holds CPL
// sketch columns, each lane RPT consecutive rows of all of them (RPT * LPC >=
// l, rows past l zero), so a lane reads only its RPT rows of the pivot column
// and uses each of them on CPL columns; dot products and norms are summed over
// the group's lanes by DPP moves.  In every step each wave finds its best live
// column (largest residual norm^2, lowest index on ties) and that column's
// lanes write its rows to the wave's slot in LDS beside the candidate; after
// the barrier the per-wave candidates are reduced across lanes (entries of
// absent waves never win) and every lane reads its rows of the pivot column
// from the winning wave's slot.  Slots and candidates are double buffered by
// step parity: the writes of step s + 1 go to the buffer last read in step
// s - 1, which every lane finished before the barrier of step s, so one
// barrier per step suffices.  The pivot column is used unscaled:
// R(s, j) = <w_p, w_j> / r_ss and w_j -= (R(s, j) / r_ss) w_p, the modified
// Gram-Schmidt step of Algorithm 1 with q = w_p / r_ss folded into two
// products with 1 / r_ss, where r_ss^2 is the pivot's residual norm^2 summed
// by its group from its rows as they are published (the same sum as a
// recomputed norm; it is also the value the waves' candidates are compared
// by).  The other residual norms are downdated, nu_j -= R(s, j)^2, as in the pivoted QR of
// Golub and Van Loan, and recomputed from the column when the downdated value
// falls below kNormRecompute of the last computed one; the downdate then errs
// by at most a few hundred units of rounding of that larger value, so the
// pivot choice can differ from one with norms recomputed every step only
// where two candidates' norms agree to about 1e-12 of the largest.  The
// tolerance test
// after step s (Remark 2.1) runs at the start of step s + 1 on per-wave sums of
// the live residual norms published with the candidates (after the last step,
// in one more round), so it ends the selection at the same step.
// ---------------------------------------------------------------------------
// sum over the LPC lanes of a group (LPC = 1, 2, 4, 8 or 16 consecutive lanes);
// every lane of the group gets the same value (the pairings are symmetric and
// addition is commutative)
template <int CTRL>
__device__ __forceinline__ double dpp_add(double v) {
  // every pattern used reads a lane of the same row, so no lane is out of
  // bounds and the moves need no initial value
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, true);
  return v + __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                              (unsigned)lo));
}

template <int LPC>
__device__ __forceinline__ double group_sum(double v) {
  if constexpr (LPC >= 2) v = dpp_add<0xB1>(v);    // quad_perm [1,0,3,2]
  if constexpr (LPC >= 4) v = dpp_add<0x4E>(v);    // quad_perm [2,3,0,1]
  if constexpr (LPC >= 8) v = dpp_add<0x141>(v);   // row_half_mirror
  if constexpr (LPC >= 16) v = dpp_add<0x140>(v);  // row_mirror
  return v;
}

__device__ __forceinline__ double readfirstlane_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)b);
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                          (unsigned)lo));
}

constexpr double kNormRecompute = 1e-3;

// two workgroups per CU at 256 threads, one at 512 or 768 (two or three waves per SIMD)
template <typename TY, int RPT, int LPC, int CPL, int MAXTHR>
__global__ __launch_bounds__(MAXTHR) __attribute__((amdgpu_waves_per_eu(MAXTHR == 768 ? 3 : 2)))
void select_step_kernel(
    const BlkInfo* __restrict__ blks, int l, int k_max, double tol, double rank_floor,
    const TY* __restrict__ Y, double* __restrict__ R, int32_t* __restrict__ S_ws,
    int32_t* __restrict__ k_ws, int32_t* __restrict__ st_ws) {
  static_assert(RPT % 2 == 0 && (LPC == 1 || LPC == 2 || LPC == 4 || LPC == 8), "shape");
  constexpr int LCOL = RPT * LPC;
  constexpr int NWMAX = MAXTHR / kWave;
  __shared__ __attribute__((aligned(16))) double slot[2][NWMAX][LCOL];
  __shared__ double cand_v[2][NWMAX];
  __shared__ double cand_r[2][NWMAX];
  __shared__ int cand_i[2][NWMAX];
  const int b = blockIdx.x;
  const BlkInfo bi = blks[b];
  const int n = bi.n;
  const int tid = threadIdx.x;
  const int lane = tid & 63, nwaves = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: LDS slot addresses in scalars
  const int h = tid % LPC;                 // row slice of the lane
  const int j0 = (tid / LPC) * CPL;        // first column of the lane's group
  const int r0 = h * RPT;
  const TY* __restrict__ Yb = Y + bi.y_off;
  double* __restrict__ Rb = R + bi.r_off;

  double w[CPL][RPT];
  double nu[CPL];    // residual norm^2 (downdated)
  // last computed residual norm^2 of each column (only compared with), in LDS
  // by group: it is read once per step
  __shared__ __attribute__((aligned(16))) float nref_s[MAXTHR / LPC][CPL];
  float* __restrict__ nref = nref_s[tid / LPC];
  // a column past n or already selected carries nu = -1 (never the argmax,
  // left out of the sums) and nref = -inf (never recomputed)
  int bad = 0;
#pragma unroll
  for (int c = 0; c < CPL; ++c) {
    const int j = j0 + c;
    const bool in = j < n;
    double s0 = 0.0, s1 = 0.0;
    // every load from a valid address (the block's first entry for rows and
    // columns outside it) and the value selected after, so that the loads
    // are all in flight together
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const bool ok = in && r0 + i < l;
      const TY raw = Yb[ok ? (int64_t)j * l + r0 + i : 0];
      w[c][i] = ok ? (double)raw : 0.0;
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const double v = w[c][i];
      if (!isfinite(v)) bad = 1;
      if (i & 1) s1 += v * v;
      else s0 += v * v;
    }
    const double ns = group_sum<LPC>(s0 + s1);
    nu[c] = in ? ns : -1.0;
    if (h == 0) nref[c] = in ? (float)ns : -INFINITY;
  }
  // candidate entries of waves that do not exist never win and add nothing
  for (int e = tid; e < 2 * NWMAX; e += blockDim.x) {
    (&cand_v[0][0])[e] = -1.0;
    (&cand_i[0][0])[e] = 0x7fffffff;
    (&cand_r[0][0])[e] = 0.0;
  }
  const int any_bad = __syncthreads_or(bad);
  // Frobenius norm^2 and largest column norm^2 of the sketch (each column
  // once), through buffer 1, which step 1 writes only after the barrier of step 0
  {
    double fs = 0.0, fm = 0.0;
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      fs += h == 0 ? fmax(nu[c], 0.0) : 0.0;
      fm = fmax(fm, nu[c]);
    }
    fs = wave_sum(fs);
    fm = wave_max(fm);
    if (lane == 0) {
      cand_r[1][wave] = fs;
      cand_v[1][wave] = fm;
    }
  }
  __syncthreads();
  double F2 = 0.0, nu0max = 0.0;
  for (int v = 0; v < nwaves; ++v) {
    F2 += cand_r[1][v];
    nu0max = fmax(nu0max, cand_v[1][v]);
  }
  // equal on every lane: held in scalar registers through the steps
  F2 = readfirstlane_f64(F2);
  nu0max = readfirstlane_f64(nu0max);
  const double tol_f = readfirstlane_f64(tol * sqrt(F2));
  const double floor2 = readfirstlane_f64(rank_floor * rank_floor * nu0max);

  int kcap = k_max;
  if (kcap > l) kcap = l;
  if (kcap > n) kcap = n;
  int status = 0, taken = 0;
  bool ran_out = false;   // the loop ended at kcap without a stop
  auto live_sum = [&]() {  // sum of the live residual norms of the lane's group (once)
    double t = 0.0;
#pragma unroll
    for (int c = 0; c < CPL; ++c) t += h == 0 ? fmax(nu[c], 0.0) : 0.0;
    return wave_sum(t);
  };
  if (any_bad) {
    status = 2;   // SPID_BLOCK_NONFINITE
  } else {
    int s = 0;
    for (; s < kcap; ++s) {
      const int buf = s & 1;
      // the lane's best live column, then the wave's
      double bv = -1.0;
      int bj = 0x7fffffff, bc = 0;
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        const bool take = nu[c] > bv;   // ties keep the lower column
        bv = take ? nu[c] : bv;
        bj = take ? j0 + c : bj;
        bc = take ? c : bc;
      }
      const int my_j = bj;
      wave_argmax_uniform(bv, bj);
      double rw = 0.0;
      if (tol > 0.0 && s > 0) rw = live_sum();
      if ((my_j == bj) & (bj != 0x7fffffff)) {
        // the lanes of the wave's winning column publish their rows of it;
        // they form one group, so its slot in the group is uniform
        // and its residual norm^2 summed from those rows, which replaces the
        // downdated value as the candidate's
        const int bcu = __builtin_amdgcn_readfirstlane(bc);
        double e0 = 0.0, e1 = 0.0;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
          if (c != bcu) continue;
#pragma unroll
          for (int i = 0; i < RPT; i += 2) {
            *reinterpret_cast<f64x2*>(&slot[buf][wave][r0 + i]) = f64x2{w[c][i], w[c][i + 1]};
            e0 += w[c][i] * w[c][i];
            e1 += w[c][i + 1] * w[c][i + 1];
          }
          __builtin_amdgcn_sched_barrier(0);
        }
        const double pn = group_sum<LPC>(e0 + e1);
        if (h == 0) {
          cand_v[buf][wave] = pn;
          cand_i[buf][wave] = bj;
        }
      }
      if (lane == 0) {
        if (bj == 0x7fffffff) {   // no live column in the wave
          cand_v[buf][wave] = -1.0;
          cand_i[buf][wave] = bj;
        }
        cand_r[buf][wave] = rw;
      }
      // orders LDS only: the R stores of the previous step stay in flight
      lds_barrier();
      // lane v < NWMAX takes wave v's candidate (entries past the last wave
      // hold -1 / 0); the argmax over those 16 lanes, then lane 0's result is
      // the block's, uniform in scalar registers
      double best;
      int p;
      {
        // the lane index is recomputed from an opaque copy every step, so
        // the candidate addresses are not held (or spilled) across the steps
        int ln = lane;
        asm volatile("" : "+v"(ln));
        double cv = ln < NWMAX ? cand_v[buf][ln] : -1.0;
        int ci = ln < NWMAX ? cand_i[buf][ln] : 0x7fffffff;
        argmax_dpp_level<0xB1>(cv, ci);
        argmax_dpp_level<0x4E>(cv, ci);
        argmax_dpp_level<0x141>(cv, ci);
        argmax_dpp_level<0x140>(cv, ci);
        best = readfirstlane_f64(cv);
        p = __builtin_amdgcn_readfirstlane(ci);
      }
      if (tol > 0.0 && s > 0) {
        int ln = lane;
        asm volatile("" : "+v"(ln));
        double cr = ln < NWMAX ? cand_r[buf][ln] : 0.0;
        cr = group_sum<16>(cr);
        if (sqrt(readfirstlane_f64(cr)) <= tol_f) break;
      }
      if (!(best > 0.0)) {
        status = 1;   // SPID_BLOCK_RANK_DEFICIENT
        break;
      }
      if (rank_floor > 0.0 && best <= floor2) {
        status = 1;
        break;
      }
      const int pw = ((p / CPL) * LPC) >> 6;   // the wave holding column p
      const double rss = sqrt(best);
      const double inv_rss = 1.0 / rss;
#pragma unroll
      for (int c = 0; c < CPL; ++c)
        if (j0 + c == p) {
          nu[c] = -1.0;
          if (h == 0) nref[c] = -INFINITY;
        }
      if (h == 0 && p >= j0 && p < j0 + CPL) {
        Rb[(int64_t)s * n + p] = rss;
        S_ws[(int64_t)b * k_max + s] = p;
      }
      taken = s + 1;
      // the lane's rows of the pivot column, held for both passes
      double q[RPT];
      const double* __restrict__ qs = &slot[buf][pw][r0];
#pragma unroll
      for (int i = 0; i < RPT; i += 2) {
        const f64x2 qa = *reinterpret_cast<const f64x2*>(qs + i);
        q[i] = qa[0];
        q[i + 1] = qa[1];
      }
      // per column: its product with the pivot, R(s, j), the update and the
      // downdated norm (one column at a time: bounded registers)
      bool need[CPL];
      bool any_need = false;
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        double d0 = 0.0, d1 = 0.0;
#pragma unroll
        for (int i = 0; i < RPT; i += 2) {
          d0 += q[i] * w[c][i];
          d1 += q[i + 1] * w[c][i + 1];
        }
        // (columns already selected hold a residue of rounding size; their
        // entries of R below the diagonal are never read)
        const double d = group_sum<LPC>(d0 + d1) * inv_rss;
        if (h == 0 && j0 + c < n) Rb[(int64_t)s * n + j0 + c] = d;
        const double coef = d * inv_rss;
#pragma unroll
        for (int i = 0; i < RPT; ++i) w[c][i] -= coef * q[i];
        // group-uniform: nu, nref and d are equal on the group's lanes
        const double nd = nu[c] - d * d;
        need[c] = nd < kNormRecompute * (double)nref[c];
        any_need |= need[c];
        nu[c] = nd;
        __builtin_amdgcn_sched_barrier(0);
      }
      // recomputation, skipped by the whole wave when no column needs it
      if (__builtin_amdgcn_ballot_w64(any_need) != 0) {
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
          double a0 = 0.0, a1 = 0.0;
#pragma unroll
          for (int i = 0; i < RPT; i += 2) {
            a0 += w[c][i] * w[c][i];
            a1 += w[c][i + 1] * w[c][i + 1];
          }
          const double np = group_sum<LPC>(a0 + a1);
          nu[c] = need[c] ? np : nu[c];
          if (need[c] && h == 0) nref[c] = (float)np;
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
    ran_out = s == kcap;
  }
  if (ran_out && tol > 0.0) {
    // tolerance after the last step: one more round of per-wave sums
    const int buf = kcap & 1;
    const double rw = live_sum();
    if (lane == 0) cand_r[buf][wave] = rw;
    lds_barrier();
    double tot = 0.0;
    for (int v = 0; v < nwaves; ++v) tot += cand_r[buf][v];
    if (!(sqrt(tot) <= tol_f)) status = 3;   // SPID_BLOCK_TOL_NOT_MET
  }
  if (tid == 0) {
    k_ws[b] = taken;
    st_ws[b] = status;
  }
  for (int t = taken + tid; t < k_max; t += blockDim.x) S_ws[(int64_t)b * k_max + t] = -1;
}

// ---------------------------------------------------------------------------
// Column selection for sketches too large for registers alone: thread t owns
// column t; rows [0, RR) of its sketch column live in registers, rows
// [RR, l) in LDS laid out row-major over the threads ([r - RR][t], so a
// wave's accesses are consecutive).  Per step: block argmax of the residual
// norms by wave butterfly and LDS (ties to the lowest index), the owner
// publishes q = w_p / ||w_p|| in LDS, every column is orthogonalised against
// q and its norm recomputed.  Dynamic LDS: (l - RR) * blockDim doubles.
// ---------------------------------------------------------------------------
template <typename TY, int RR, int MAXTHR>
__global__ __launch_bounds__(MAXTHR) void select_hybrid_kernel(
    const BlkInfo* __restrict__ blks, int l, int k_max, double tol, double rank_floor,
    const TY* __restrict__ Y, double* __restrict__ R, int32_t* __restrict__ S_ws,
    int32_t* __restrict__ k_ws, int32_t* __restrict__ st_ws) {
  extern __shared__ double wl[];          // [(l - RR)][nthr]
  __shared__ double q_lds[128];
  __shared__ double red_v[16];
  __shared__ int red_i[16];
  __shared__ double bc_rss;
  const int b = blockIdx.x;
  const BlkInfo bi = blks[b];
  const int n = bi.n;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, nwaves = nthr >> 6;
  const int lr = l > RR ? l - RR : 0;     // rows held in LDS
  const TY* __restrict__ Yb = Y + bi.y_off;
  double* __restrict__ Rb = R + bi.r_off;
  const int j = tid;
  bool live = j < n;

  double w[RR];
  int bad = 0;
  double nu;
  {
    // loads from valid addresses (the block's first entry outside it), values
    // selected after, so that the loads are in flight together
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < RR; ++r) {
      const bool ok = live && r < l;
      const TY raw = Yb[ok ? (int64_t)j * l + r : 0];
      w[r] = ok ? (double)raw : 0.0;
    }
#pragma unroll
    for (int r = 0; r < RR; ++r) {
      if (!isfinite(w[r])) bad = 1;
      acc += w[r] * w[r];
    }
#pragma unroll 8
    for (int r = 0; r < lr; ++r) {
      const TY raw = Yb[live ? (int64_t)j * l + RR + r : 0];
      const double v = live ? (double)raw : 0.0;
      if (!isfinite(v)) bad = 1;
      wl[r * nthr + tid] = v;
      acc += v * v;
    }
    nu = live ? acc : 0.0;
  }
  for (int e = tid; e < 128; e += nthr) q_lds[e] = 0.0;
  const int any_bad = __syncthreads_or(bad);

  double fs = wave_sum(nu), fm = wave_max(nu);
  if (lane == 0) red_v[wave] = fs;
  __syncthreads();
  double F2 = 0.0;
  for (int v = 0; v < nwaves; ++v) F2 += red_v[v];
  __syncthreads();
  if (lane == 0) red_v[wave] = fm;
  __syncthreads();
  double nu0max = 0.0;
  for (int v = 0; v < nwaves; ++v) nu0max = fmax(nu0max, red_v[v]);
  __syncthreads();

  int kcap = k_max;
  if (kcap > l) kcap = l;
  if (kcap > n) kcap = n;
  int status = 0, taken = 0;
  if (any_bad) {
    status = 2;
  } else {
    for (int s = 0; s < kcap; ++s) {
      double bv = live ? nu : -1.0;
      int bj = live ? j : 0x7fffffff;
      wave_argmax(bv, bj);
      if (lane == 0) {
        red_v[wave] = bv;
        red_i[wave] = bj;
      }
      lds_barrier();
      // every wave reduces the per-wave winners itself (ties to the lowest index); the
      // next write of red_v comes after the pivot barrier below
      double best = lane < nwaves ? red_v[lane] : -1.0;
      int p = lane < nwaves ? red_i[lane] : 0x7fffffff;
      wave_argmax(best, p);
      if (!(best > 0.0)) {
        status = 1;
        break;
      }
      if (rank_floor > 0.0 && best <= rank_floor * rank_floor * nu0max) {
        status = 1;
        break;
      }
      if (j == p) {
        double pn = 0.0;
#pragma unroll
        for (int r = 0; r < RR; ++r) {
          pn += w[r] * w[r];
          q_lds[r] = w[r];
        }
        for (int r = 0; r < lr; ++r) {
          const double v = wl[r * nthr + tid];
          pn += v * v;
          q_lds[RR + r] = v;
        }
        const double rss = sqrt(pn);
        bc_rss = rss;
        Rb[(int64_t)s * n + p] = rss;
        live = false;
        nu = 0.0;
      }
      if (tid == 0) S_ws[(int64_t)b * k_max + s] = p;
      lds_barrier();
      if (tid < RR + lr) q_lds[tid] = q_lds[tid] / bc_rss;
      lds_barrier();
      taken = s + 1;
      double d = 0.0;
#pragma unroll
      for (int r0 = 0; r0 < RR; r0 += 8) {
#pragma unroll
        for (int r = r0; r < r0 + 8 && r < RR; ++r) d += q_lds[r] * w[r];
        __builtin_amdgcn_sched_barrier(0);
      }
      for (int r = 0; r < lr; ++r) d += q_lds[RR + r] * wl[r * nthr + tid];
      if (live) Rb[(int64_t)s * n + j] = d;
      d = live ? d : 0.0;
      double a2 = 0.0;
#pragma unroll
      for (int r0 = 0; r0 < RR; r0 += 8) {
#pragma unroll
        for (int r = r0; r < r0 + 8 && r < RR; ++r) {
          const double qr =
              __hip_atomic_load(q_lds + r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          w[r] -= d * qr;
          a2 += w[r] * w[r];
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      for (int r = 0; r < lr; ++r) {
        double v = wl[r * nthr + tid];
        v -= d * q_lds[RR + r];
        wl[r * nthr + tid] = v;
        a2 += v * v;
      }
      nu = live ? a2 : 0.0;
      if (tol > 0.0) {
        const double rest = wave_sum(nu);
        if (lane == 0) red_v[wave] = rest;
        lds_barrier();
        double tot = 0.0;
        for (int v = 0; v < nwaves; ++v) tot += red_v[v];
        if (sqrt(tot) <= tol * sqrt(F2)) {
          lds_barrier();
          break;
        }
        if (s == kcap - 1) status = 3;
      }
      lds_barrier();
    }
  }
  if (tid == 0) {
    k_ws[b] = taken;
    st_ws[b] = status;
  }
  for (int s = taken + tid; s < k_max; s += nthr) S_ws[(int64_t)b * k_max + s] = -1;
}

// Copy per-block selection results to the caller's arrays.
static __global__ void select_export_kernel(int nblocks, int k_max, const int32_t* __restrict__ S_ws,
                                     const int32_t* __restrict__ k_ws,
                                     const int32_t* __restrict__ st_ws, int32_t* d_k,
                                     int32_t* d_S, int32_t* d_status) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (d_S && e < (int64_t)nblocks * k_max) d_S[e] = S_ws[e];
  if (e < nblocks) {
    if (d_k) d_k[e] = k_ws[e];
    if (d_status) d_status[e] = st_ws[e];
  }
}

// ---------------------------------------------------------------------------
// Coefficients: P_b(:, S[t]) = e_t, and for every other column j the
// solution of R11 x = R12(:, j) (Section 2, Algorithm 1), FP64, by block
// back-substitution in row blocks of 16.  One workgroup of kCoThreads per
// block: the non-skeleton columns are listed in ascending order in LDS (the
// order the error pass uses) and R11 is staged in LDS, padded to KB * 16 rows
// and columns with the identity past k (the padded unknowns come out as exact
// zeros and add exact zeros to the real rows).  The inverse of each 16 x 16
// diagonal block of R11 is formed once per workgroup (back-substitution on
// the unit vectors, one lane per column).  A wave takes 16 non-skeleton
// columns at a time, their right-hand sides R12(:, j) held as KB accumulator
// tiles of the FP64 matrix cores (16 rows each); from the last row block up,
// the block's unknowns are its inverse times its right-hand side and are
// taken off every row block above by products with R11, both on the matrix
// cores.  Its error is that of a triangular solve, at most a small multiple
// of the unit roundoff times the condition number of R11 (a diagonal block's
// condition number is at most that of R11).  When `pt` is given (mixed
// error pass on FP32 data) the wave also writes the three bfloat16 terms
// (hi, mid, lo: 24 significant bits) of its columns' negated coefficients and
// the compact column list, so the error pass stages them by plain copies.
// Layouts: cols[col_off + q], pt[(col_off + q) * 3 * KP + term * KP + 8 pi + v]
// = term of -P(rcbf_sel(pi / 4, pi % 4, v), column q) with col_off = y_off / l
// (the block's first column in the batch), KP = 32 KS32 = 32 ceil(KB / 2).
// ---------------------------------------------------------------------------
// Order of the split coefficient terms (mixed error pass): slot v of the
// 16-byte piece 4 ks + g of a term holds coefficient row rcbf_sel(ks, g, v),
// and the error pass gathers selected column rcbf_sel(ks, g, v) into the same
// slot of its MFMA operand (the sum over the selected columns, permuted
// alike on both sides).  Rows 16 r + g + 4 u (u < 4) are accumulator slots of
// tile r in the coefficients kernel, so its lanes write whole pieces.
__host__ __device__ constexpr int rcbf_sel(int ks, int g, int v) {
  return 32 * ks + 16 * (v >> 2) + g + 4 * (v & 3);
}
constexpr int kCoThreads = 256;
constexpr int kCoSld = 17;    // row stride of a wave's 16 x 16 staging tile (doubles)

// LDS of coeffs_kernel<KB>: R11 padded to 16 KB rows, row stride 16 KB + 1
__host__ __device__ constexpr size_t coeffs_lds_bytes(int KB) {
  return sizeof(double) * (size_t)(16 * KB) * (16 * KB + 1);
}


// three workgroups per CU fit the LDS up to KB = 4 (one for KB = 6)
template <int KB>
__global__ __launch_bounds__(kCoThreads) __attribute__((amdgpu_waves_per_eu(KB <= 4 ? 3 : 1))) void coeffs_kernel(
    const BlkInfo* __restrict__ blks, int l, int k_max, const double* __restrict__ R,
    const int32_t* __restrict__ S_ws, const int32_t* __restrict__ k_ws, double* __restrict__ P,
    __bf16* __restrict__ pt, int KP, int32_t* __restrict__ cols_out, int32_t* __restrict__ ncols_out) {
  constexpr int KM = 16 * KB;          // padded rank
  constexpr int LD = KM + 1;           // R11 row stride in LDS (odd: spreads the banks)
  extern __shared__ double r11[];      // [KM][LD]
  __shared__ double tinv[KB][16 * kCoSld];   // inverses of the diagonal 16 x 16 blocks
  __shared__ int s_sh[KM];
  __shared__ int cols[1024];
  __shared__ unsigned char is_sel[1024];
  __shared__ int wcount[kCoThreads / 64];
  const int b = blockIdx.x;
  const BlkInfo bi = blks[b];
  const int n = bi.n;
  const int k = k_ws[b];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int32_t* S = S_ws + (int64_t)b * k_max;
  const double* Rb = R + bi.r_off;
  double* Pb = P + bi.p_off;
  for (int j = tid; j < n; j += kCoThreads) is_sel[j] = 0;
  if (tid < KM) s_sh[tid] = tid < k ? S[tid] : 0;
  __syncthreads();
  if (tid < k) is_sel[s_sh[tid]] = 1;
  {
    // R11 with the identity past k: every load issued before the LDS stores
    constexpr int NE = (KM * KM + kCoThreads - 1) / kCoThreads;
    double v[NE];
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      const int e = tid + q * kCoThreads;
      const int s2 = e / KM, t = e - s2 * KM;
      const bool in = e < KM * KM && s2 < k && t < k && t >= s2;
      v[q] = Rb[in ? (int64_t)s2 * n + s_sh[t] : 0];
      v[q] = in ? v[q] : (s2 == t ? 1.0 : 0.0);
    }
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      const int e = tid + q * kCoThreads;
      const int s2 = e / KM, t = e - s2 * KM;
      if (e < KM * KM) r11[s2 * LD + t] = v[q];
    }
  }
  __syncthreads();
  // the inverse of every diagonal block (one column per lane, by
  // back-substitution on the unit vectors; zero below the diagonal)
  for (int B = wave; B < KB; B += kCoThreads / 64) {
    if (lane < 16) {
      double x[16];
#pragma unroll
      for (int i = 15; i >= 0; --i) {
        const double* rr = r11 + (16 * B + i) * LD + 16 * B;
        double a = i == lane ? 1.0 : 0.0;
#pragma unroll
        for (int t = i + 1; t < 16; ++t) a -= rr[t] * x[t];
        x[i] = a / rr[i];
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) tinv[B][i * kCoSld + lane] = x[i];
    }
  }
  // compact list of the non-skeleton columns (ascending)
  int ncols = 0;
  for (int base = 0; base < n; base += kCoThreads) {
    const int j = base + tid;
    const bool keep = j < n && !is_sel[j];
    const uint64_t bal = __ballot(keep);
    const int before = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wcount[wave] = __popcll(bal);
    __syncthreads();
    int off = ncols;
    for (int v = 0; v < wave; ++v) off += wcount[v];
    if (keep) cols[off + before] = j;
    int tot = 0;
    for (int v = 0; v < kCoThreads / 64; ++v) tot += wcount[v];
    ncols += tot;
    __syncthreads();
  }
  const int64_t col_off = bi.y_off / l;
  if (pt && tid == 0) ncols_out[b] = ncols;
  // skeleton columns: exact unit vectors
  for (int e = tid; e < k * k_max; e += kCoThreads) {
    const int t = e / k_max, u = e - t * k_max;
    Pb[(int64_t)s_sh[t] * k_max + u] = (u == t) ? 1.0 : 0.0;
  }
  const int c16 = lane & 15, g4 = lane >> 4;
  const int ntiles = (ncols + 15) / 16;
  // right-hand sides R12(:, j) of a tile: tile r, slot v holds row 16 r + g4 +
  // 4 v; loaded from valid addresses with the values selected after, one
  // tile ahead, so that the loads of the next tile are in flight during this
  // tile's products and are issued before its stores (a wait for them then
  // covers no store)
  auto load_rhs = [&](int tile, f64x4 (&b)[KB]) {
    const int cq = tile * 16 + c16;
    const bool cok = cq < ncols;
    const int j = cok ? cols[cq] : 0;
#pragma unroll
    for (int r = 0; r < KB; ++r)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * r + g4 + 4 * v;
        const bool ok = cok && row < k;
        const double x = Rb[ok ? (int64_t)row * n + j : 0];
        b[r][v] = ok ? x : 0.0;
      }
  };
  f64x4 nxt[KB];
  if (wave < ntiles) load_rhs(wave, nxt);
  for (int tile = wave; tile < ntiles; tile += kCoThreads / 64) {
    const int cq = tile * 16 + c16;          // compact index of the lane's column
    const bool cok = cq < ncols;
    const int j = cok ? cols[cq] : 0;
    f64x4 acc[KB];
#pragma unroll
    for (int r = 0; r < KB; ++r) acc[r] = nxt[r];
    if (tile + kCoThreads / 64 < ntiles) load_rhs(tile + kCoThreads / 64, nxt);
    // From the last row block up: x_B = inv(R11_BB) b_B, then the rows above
    // lose R11(rows r, columns of B) x_B, all on the matrix cores.  Slot v of
    // the accumulator layout (row g4 + 4 v) is the B operand of k-step v
    // (row 4 v + g4), so the solved block feeds the products as it stands.
    // the operands are read from LDS in every tile (an opaque offset keeps
    // the compiler from holding all of them in registers across tiles)
    int lo = 0;
    asm volatile("" : "+v"(lo));
#pragma unroll
    for (int B = KB - 1; B >= 0; --B) {
      f64x4 xb = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int qk = 0; qk < 4; ++qk)
        xb = mfma_f64(tinv[B][lo + c16 * kCoSld + 4 * qk + g4], acc[B][qk], xb);
      acc[B] = xb;
#pragma unroll
      for (int r = 0; r < B; ++r)
#pragma unroll
        for (int qk = 0; qk < 4; ++qk) {
          const double a = -r11[lo + (16 * r + c16) * LD + 16 * B + 4 * qk + g4];
          acc[r] = mfma_f64(a, acc[B][qk], acc[r]);
        }
    }
    if (!cok) continue;
    // P(:, j): rows below k_max (rows past k are exact zeros)
    double* pc = Pb + (int64_t)j * k_max;
#pragma unroll
    for (int r = 0; r < KB; ++r)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * r + g4 + 4 * v;
        if (row < k_max) pc[row] = acc[r][v];
      }
    if (pt) {
      if (g4 == 0) cols_out[col_off + cq] = j;
      // three bfloat16 terms of every coefficient (rows past 16 KB zero up to
      // KP), in 16-byte pieces: piece pi = 4 rho + g4 of a term holds rows
      // 32 rho + 16 (v / 4) + g4 + 4 (v % 4), v < 8 -- accumulator slots
      // v % 4 of tiles 2 rho and 2 rho + 1 of this lane -- so every lane
      // writes whole pieces.  The error pass gathers its selected columns in
      // the same order (sum over the selected columns permuted alike).
      __bf16* o = pt + (col_off + cq) * 3 * KP;
#pragma unroll
      for (int rho = 0; rho < (KB + 1) / 2; ++rho) {
        bf16x8 th, tm, tl;
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          // row rcbf_sel(rho, g4, v) = 16 r + g4 + 4 (v % 4): slot v % 4 of tile r
          static_assert(rcbf_sel(1, 2, 5) == 16 * 3 + 2 + 4 * 1, "piece order");
          const int r = 2 * rho + (v >> 2);
          const double pv = r < KB ? -acc[r < KB ? r : 0][v & 3] : 0.0;   // the error pass adds the products to A
          const __bf16 hi = to_bf16((float)pv);
          const double r1 = pv - (double)(float)hi;
          const __bf16 md = to_bf16((float)r1);
          const __bf16 lo = to_bf16((float)(r1 - (double)(float)md));
          th[v] = hi;
          tm[v] = md;
          tl[v] = lo;
        }
        const int pi = 4 * rho + g4;
        *reinterpret_cast<bf16x8*>(o + 8 * pi) = th;
        *reinterpret_cast<bf16x8*>(o + KP + 8 * pi) = tm;
        *reinterpret_cast<bf16x8*>(o + 2 * KP + 8 * pi) = tl;
      }
    }
  }
}

constexpr int kRcThreads = 256;
constexpr int kRcLdsBytes = 65536;   // coefficient staging budget of one error-pass workgroup

// Compact the non-skeleton columns of a block into `cols` (ascending j);
// returns their number.  All threads of the workgroup call it.
__device__ __forceinline__ int rc_compact_columns(int n, int k, const int32_t* __restrict__ S,
                                                  unsigned char* is_sel, int* cols,
                                                  int* wcount) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int j = tid; j < n; j += kRcThreads) is_sel[j] = 0;
  __syncthreads();
  if (tid < k) is_sel[S[tid]] = 1;
  __syncthreads();
  int ncols = 0;
  for (int base = 0; base < n; base += kRcThreads) {
    const int j = base + tid;
    const bool keep = j < n && !is_sel[j];
    const uint64_t bal = __ballot(keep);
    const int before = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wcount[wave] = __popcll(bal);
    __syncthreads();
    int off = ncols;
    for (int v = 0; v < wave; ++v) off += wcount[v];
    if (keep) cols[off + before] = j;
    int tot = 0;
    for (int v = 0; v < 4; ++v) tot += wcount[v];
    ncols += tot;
    __syncthreads();
  }
  return ncols;
}

// Four consecutive rows i0..i0+3 (i0 a multiple of 4) of one column for the
// residual, rows at or past m read as zero.  VEC (16-byte aligned columns and
// m a multiple of 4): a group is entirely inside or entirely outside the
// block, so one vector load from a clamped address plus a selection covers
// both; otherwise four clamped scalar loads.  Branch-free either way.
template <typename TA, bool VEC>
__device__ __forceinline__ void rc_load4(gptr<TA> __restrict__ colp, int64_t i0, int64_t m,
                                         bool ok, double out[4]) {
  if constexpr (VEC) {
    const bool in = ok && i0 < m;
    gptr<TA> src = colp + (in ? i0 : 0);
    if constexpr (sizeof(TA) == 8) {
      const f64x2 x0 = __builtin_nontemporal_load((gptr<f64x2>)src);
      const f64x2 x1 = __builtin_nontemporal_load((gptr<f64x2>)src + 1);
      out[0] = in ? x0[0] : 0.0;
      out[1] = in ? x0[1] : 0.0;
      out[2] = in ? x1[0] : 0.0;
      out[3] = in ? x1[1] : 0.0;
    } else {
      const f32x4 x = __builtin_nontemporal_load((gptr<f32x4>)src);
#pragma unroll
      for (int v = 0; v < 4; ++v) out[v] = in ? (double)x[v] : 0.0;
    }
  } else {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t i = min(i0 + v, m - 1);
      const double x = (double)colp[i];
      out[v] = (ok && i0 + v < m) ? x : 0.0;
    }
  }
}

// ---------------------------------------------------------------------------
// Reconstruction error on the matrix cores (double precision).
// Ahat(rows, cols) = A(rows, S) P(:, cols) with v_mfma_f64_16x16x4: the
// skeleton A(rows, S) is the A operand (16 rows x 4 selected columns per
// k-step), P the B operand (4 x 16 columns), Ahat accumulates in D.  Rows
// inside a 16-row tile are permuted (tile row rho -> 4 (rho % 4) + rho / 4)
// so that lane (g, c) receives D rows 4g..4g+3 of column c: the residual
// operands are four consecutive entries of one column per lane.
//
// Work item = (block, it.nsub sub-tiles of 4 * 16 * MTR rows starting at
// it.i0).  The non-skeleton columns are compacted once per item and their
// coefficients staged in LDS (pcap columns at a time, normally all of them),
// so the staging is amortised over every sub-tile of the item.  Each wave
// holds its 16 * MTR skeleton rows in registers and streams the staged
// columns 16 at a time.  KS = k-steps (k_max / 4 rounded up).
// Dynamic LDS: pcap * 4 * KS doubles.
// ---------------------------------------------------------------------------
template <typename TA, int KS, int MTR, bool VEC>
__global__ __launch_bounds__(kRcThreads) __attribute__((amdgpu_waves_per_eu(2))) void recon_mfma_kernel(
    const BlkInfo* __restrict__ blks, const RcItem* __restrict__ items, XcdSplit xs, int k_max, int pcap,
    const int32_t* __restrict__ S_ws, const int32_t* __restrict__ k_ws,
    const double* __restrict__ P, TA* __restrict__ skel, double* __restrict__ part) {
  // [pcap][kp + 1]: the odd stride puts the 16 columns one MFMA reads on
  // different banks (a stride of kp, a multiple of 16 doubles, is one bank)
  extern __shared__ __attribute__((aligned(16))) double p_lds[];
  __shared__ double red[8];
  __shared__ int cols[1024];
  __shared__ unsigned char is_sel[1024];
  __shared__ int wcount[4];
  constexpr int kp = 4 * KS;
  constexpr int kSub = 4 * 16 * MTR;
  const int item = xcd_item(xs);
  if (item < 0) return;
  const RcItem it = items[item];
  const BlkInfo bi = blks[it.blk];
  const int n = bi.n;
  const int k = k_ws[it.blk];
  const int32_t* S = S_ws + (int64_t)it.blk * k_max;
  gptr<TA> __restrict__ A = (gptr<TA>)bi.A;
  const double* __restrict__ Pb = P + bi.p_off;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, c16 = lane & 15;
  const int ncols = rc_compact_columns(n, k, S, is_sel, cols, wcount);
  // A operand: lane supplies tile row rho = c16 -> actual row 4 (rho % 4) + rho / 4,
  // k-slot g of step s -> selected column 4 s + g
  const int arow = 4 * (c16 & 3) + (c16 >> 2);
  double a2 = 0.0, e2 = 0.0;

  // one pass per coefficient chunk (a single one unless ncols > pcap)
  for (int c0 = 0; c0 == 0 || c0 < ncols; c0 += pcap) {
    const int cc = max(0, min(pcap, ncols - c0));
    const int ntile = (cc + 15) / 16;
    for (int e = tid; e < ntile * 16 * kp; e += kRcThreads) {
      const int q = e / kp, t = e - q * kp;
      const bool ok = q < cc && t < k_max;
      const double x = cc > 0 ? Pb[(int64_t)cols[c0 + min(q, cc - 1)] * k_max + min(t, k_max - 1)]
                              : 0.0;
      p_lds[q * (kp + 1) + t] = ok ? x : 0.0;   // P rows k..k_max-1 are zero
    }
    __syncthreads();
    for (int rs = 0; rs < it.nsub; ++rs) {
      const int64_t rbase = it.i0 + (int64_t)rs * kSub + (int64_t)wave * 16 * MTR;
      // gather without branches (entries outside the block or past k read the
      // first selected column / row 0, then are zeroed), so the loads overlap
      double as[MTR][KS];
#pragma unroll
      for (int mt = 0; mt < MTR; ++mt) {
        const int64_t i = rbase + 16 * mt + arow;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          as[mt][s] = 0.0;
          if (4 * s >= k) continue;   // uniform: k-steps past the selected columns are never read
          const int t = 4 * s + g;
          as[mt][s] = (double)A[(int64_t)S[t < k ? t : 0] * bi.lda + (i < bi.m ? i : 0)];
        }
      }
#pragma unroll
      for (int mt = 0; mt < MTR; ++mt) {
        const int64_t i = rbase + 16 * mt + arow;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          const int t = 4 * s + g;
          const bool ok = t < k && i < bi.m;
          const double v = ok ? as[mt][s] : 0.0;
          if (ok && skel && c0 == 0) skel[bi.sk_off + (int64_t)t * bi.m + i] = (TA)v;
          as[mt][s] = v;
          if (c0 == 0) a2 += v * v;
        }
      }
      for (int tq = 0; tq < ntile; ++tq) {
        const int q = 16 * tq + c16;
        const bool cok = q < cc;
        gptr<TA> colp = A + (int64_t)cols[c0 + (cok ? q : cc - 1)] * bi.lda;
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

// ---------------------------------------------------------------------------
// Reconstruction error for single-precision data on the bfloat16 matrix
// cores.  A(rows, S) and the negated coefficients -P are split into three
// bfloat16 terms each (hi + mid + lo carries all 24 bits of a float); the
// accumulator of v_mfma_f32_16x16x32_bf16 starts at A(rows, j) and takes the
// six term products of weight at least 2^-16 (hi*hi, hi*mid, mid*hi, hi*lo,
// mid*mid, lo*hi), largest first, so it ends at the residual
// A(rows, j) - A(rows, S) P(:, j) with every rounding at the size of what is
// left.  Squared residuals and squared entries of the non-skeleton columns
// are summed in FP32 over one step (16 per lane, relative error at most
// 16 * 2^-24) and the step sums in FP64 (the skeleton columns' entries in
// FP64).  KS32 = k-steps of 32 selected columns.
//
// A work item is 128 rows (4 waves x 32) of one block; a wave's skeleton
// terms (its 32 rows of A(:, S)) stay in registers.  The non-skeleton columns
// are streamed in steps of 32: the step's A values arrive as whole 128-byte
// lines (two load instructions per 16 columns) loaded one step ahead (two at
// KS32 = 2), and are passed through a wave-private LDS tile into the MFMA
// output layout (lane (g, c16) holds rows 4g..4g+3 of column c16 of each
// 16-row tile).  The P terms (split once by the coefficients kernel, with the
// compact column list) are staged rcbf_cols(KS32) columns at a time (about 26
// KiB of LDS) by plain 16-byte copies behind LDS-only barriers, or at KS32 = 2
// a step at a time from registers loaded a step earlier; the columns' element
// offsets are staged whole at the start, so the prefetch runs across the
// barriers.
// ---------------------------------------------------------------------------
constexpr int kRcBfSubs = 1;
constexpr int kRcMaxCols = 1024;   // widest block (the descriptor limit on n)
__host__ __device__ constexpr int rcbf_cols(int KS32) { return KS32 == 1 ? 96 : (KS32 == 2 ? 64 : 32); }
// resident waves per SIMD the register allocation targets (LDS allows four)
__host__ __device__ constexpr int rcbf_waves(int KS32) { return KS32 == 1 ? 4 : 2; }

template <int KS32, int MTR, bool VEC>
__global__ __launch_bounds__(kRcThreads) __attribute__((amdgpu_waves_per_eu(rcbf_waves(KS32))))
void recon_bf16x3_kernel(
    const BlkInfo* __restrict__ blks, const RcItem* __restrict__ items, XcdSplit xs, int l, int k_max,
    const int32_t* __restrict__ S_ws, const int32_t* __restrict__ k_ws,
    const __bf16* __restrict__ pt_g, const int32_t* __restrict__ cols_g,
    const int32_t* __restrict__ ncols_g, float* __restrict__ skel, double* __restrict__ part) {
  constexpr int KP = 32 * KS32;
  constexpr int kCols = rcbf_cols(KS32);
  // two-step P staging (KS32 = 2): each step's terms copied from registers
  // loaded a step earlier, so the copy never waits for the A prefetch;
  // otherwise chunks of kCols columns copied straight from memory
  constexpr bool kPipeP = KS32 == 2;
  // steps of A loaded ahead: two on the two-step P staging, whose register
  // budget (two waves per SIMD) leaves room for a third line buffer
  constexpr int kPf = kPipeP ? 2 : 1;
  static_assert(!kPipeP || (kCols == 64 && 3 * KP == 8 * 8 * 3), "two 32-column slots");
  // a column's three terms, 3 KP bfloat16 (a multiple of 32 dwords), then 8
  // bfloat16 of padding: the 16 columns one MFMA reads start 4 banks apart
  // instead of on one bank
  constexpr int kPtStride = 3 * KP + 8;
  __shared__ __attribute__((aligned(16))) __bf16 pt[kCols * kPtStride];
  __shared__ __attribute__((aligned(16))) float stage_all[kRcThreads / 64 * 16 * kLineSt];
  __shared__ int64_t coff[kRcMaxCols];   // element offset of each non-skeleton column
  __shared__ double red[8];
  static_assert(MTR == 2, "a wave's rows are one 128-byte line of each column");
  const int item = xcd_item(xs);
  if (item < 0) return;
  const RcItem it = items[item];
  const BlkInfo bi = blks[it.blk];
  const int k = k_ws[it.blk];
  const int32_t* S = S_ws + (int64_t)it.blk * k_max;
  gptr<float> __restrict__ A = (gptr<float>)bi.A;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, c16 = lane & 15, p8 = lane & 7;
  const int wave_u = __builtin_amdgcn_readfirstlane(wave);   // wave-uniform (scalar) copy
  float* __restrict__ st = stage_all + wave * 16 * kLineSt;
  const int64_t col_off = bi.y_off / l;
  const int ncols = ncols_g[it.blk];
  const int ksn = (k + 31) >> 5;   // k-steps holding selected columns (the rest are zero)
  const __bf16* __restrict__ ptb = pt_g + col_off * 3 * KP;
  const int32_t* __restrict__ colb = cols_g + col_off;
  const int64_t rbase = it.i0 + wave_u * 16 * MTR;   // the wave's 32 rows
  // the lane's LDS tile offsets: its two line pieces (columns 8h + lane / 8),
  // and its operand pieces (rows 16 mt + 4g.., column c16)
  int st_w[2], st_r[MTR];
#pragma unroll
  for (int h = 0; h < 2; ++h) st_w[h] = (int)(line_piece(st, 8 * h + (lane >> 3), p8) - st);
#pragma unroll
  for (int mt = 0; mt < MTR; ++mt) st_r[mt] = (int)(line_piece(st, c16, 4 * mt + g) - st);

  // the block's non-skeleton column indices (loads issued first: the item's
  // first loads all overlap)
  static_assert(kRcMaxCols == 4 * kRcThreads, "four column indices per thread");
  int32_t cidx[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int c = tid + u * kRcThreads;
    cidx[u] = colb[c < ncols ? c : 0];
  }
  // A operand: tile row c16, slot v of k-step ks holds selected column
  // rcbf_sel(ks, g, v) (the order of the coefficient terms' pieces), three
  // terms (k-steps past ksn are never read).  The gather is issued without
  // branches (out-of-range entries read row 0 / the first selected column,
  // then are zeroed), behind the column-index loads, so both overlap.
  bf16x8 at[MTR][KS32][3];
  float xsel[MTR][KS32][8];
  double a2 = 0.0, e2 = 0.0;
#pragma unroll
  for (int mt = 0; mt < MTR; ++mt) {
    const int64_t i = rbase + 16 * mt + c16;
    const bool iok = i < bi.m;
#pragma unroll
    for (int ks = 0; ks < KS32; ++ks) {
      if (ks >= ksn) break;
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const int t = rcbf_sel(ks, g, v);
        xsel[mt][ks][v] = A[(int64_t)S[t < k ? t : 0] * bi.lda + (iok ? i : 0)];
      }
    }
  }
#pragma unroll
  for (int mt = 0; mt < MTR; ++mt) {
    const int64_t i = rbase + 16 * mt + c16;
    const bool iok = i < bi.m;
#pragma unroll
    for (int ks = 0; ks < KS32; ++ks) {
      if (ks >= ksn) break;
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const int t = rcbf_sel(ks, g, v);
        const bool ok = t < k && iok;
        const float x = ok ? xsel[mt][ks][v] : 0.0f;
        if (skel && ok) skel[bi.sk_off + (int64_t)t * bi.m + i] = x;
        a2 += (double)x * (double)x;
        const __bf16 h = to_bf16(x);
        const float r1 = x - (float)h;
        const __bf16 md = to_bf16(r1);
        const __bf16 lo = to_bf16(r1 - (float)md);
        at[mt][ks][0][v] = h;
        at[mt][ks][1][v] = md;
        at[mt][ks][2][v] = lo;
      }
    }
  }

  // P terms of columns c0 .. c0 + kCols - 1 into LDS (zero past ncols)
  auto stage_p = [&](int c0) {
    const int cc = min(kCols, ncols - c0);
    lds_barrier();   // every wave is done with the previous chunk
    constexpr int kVec = kCols * 3 * KP / 8;   // 16-byte pieces of the chunk
    for (int e = tid; e < kVec; e += kRcThreads) {
      const int q = e / (3 * KP / 8), r8 = e - q * (3 * KP / 8);
      if (8 * (e % (KP / 8)) >= 32 * ksn) continue;   // terms of k-steps that are skipped
      bf16x8 v = bf16x8{};
      if (q < cc) v = *reinterpret_cast<const bf16x8*>(ptb + (int64_t)c0 * 3 * KP + (int64_t)e * 8);
      *reinterpret_cast<bf16x8*>(pt + q * kPtStride + 8 * r8) = v;
    }
    lds_barrier();
  };

  const int nst = (ncols + 31) >> 5;   // 32-column steps
  // the block's non-skeleton column offsets, once per item (the loads index them)
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int c = tid + u * kRcThreads;
    if (c < ncols) coff[c] = (int64_t)cidx[u] * bi.lda;
  }
  lds_barrier();
  auto body = [&](auto full_c) {
    constexpr bool kFull = decltype(full_c)::value;
    // lines of step s: group gq, instruction h -> column 32 s + 16 gq + 8 h + lane / 8
    // (clamped to the last column; columns past ncols are masked below)
    auto load = [&](int s, float (&x)[2][2][4]) {
#pragma unroll
      for (int gq = 0; gq < 2; ++gq)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int c = min(32 * s + 16 * gq + 8 * h + (lane >> 3), ncols - 1);
          gptr<float> src = A + coff[c];
          if constexpr (kFull) load_line<float, VEC>(src, rbase, p8, x[gq][h]);
          else load_line_tail<float>(src, rbase, bi.m, p8, x[gq][h]);
        }
    };
    // P terms of step s's 32 columns (pipelined form): thread t copies pieces
    // 8 (t % 8) + 64 i .. + 7, i < 3, of column t / 8 (a column's 3 KP terms
    // are contiguous, so 8 threads read its 384 bytes in three 128-byte
    // runs), loaded into registers a step ahead of their copy into LDS slot
    // s & 1; columns past ncols are zero.  The offsets are fixed per thread,
    // the step only moves the (scalar) base.
    constexpr int NPC = 3;
    bf16x8 pv[kPipeP ? NPC : 1];
    const int pq = tid >> 3, pr = 8 * (tid & 7);
    auto load_p = [&](int s) {
      const int c0 = 32 * s, cc = min(32, ncols - c0);
      // the last step reads its last column for the columns past ncols, then zeroes them
      const int qc = cc < 32 ? min(pq, cc - 1) : pq;
      const __bf16* src = ptb + (int64_t)c0 * 3 * KP + (qc * 3 * KP + pr);
#pragma unroll
      for (int i = 0; i < NPC; ++i) pv[i] = *reinterpret_cast<const bf16x8*>(src + 64 * i);
      if (cc < 32) {
#pragma unroll
        for (int i = 0; i < NPC; ++i) pv[i] = pq < cc ? pv[i] : bf16x8{};
      }
    };
    auto store_p = [&](int s) {
      __bf16* dst = pt + (s & 1) * 32 * kPtStride + (pq * kPtStride + pr);
#pragma unroll
      for (int i = 0; i < NPC; ++i) *reinterpret_cast<bf16x8*>(dst + 64 * i) = pv[i];
    };
    auto step = [&](const float (&x)[2][2][4], float (&xn)[2][2][4], int s) {
      if constexpr (kPipeP) {
        // one barrier per step: every wave is done with slot (s + 1) & 1 (step
        // s - 1) and sees slot s & 1.  Each step's P loads are issued before
        // its A prefetch, so the copy never waits for A loads of later steps.
        lds_barrier();
        if (s + 1 < nst) store_p(s + 1);
        if (s + 2 < nst) load_p(s + 2);
        load(min(s + kPf, nst - 1), xn);
      } else {
        if ((32 * s) % kCols == 0) stage_p(32 * s);
        load(min(s + 1, nst - 1), xn);
      }
      float es = 0.0f, as = 0.0f;   // the step's squared residuals and squared entries
      // one 16-column group; MASK: some of its columns lie past ncols (the
      // block's last group only)
      auto group = [&](auto mask_c, const float (&xg)[2][4], int q0) {
        constexpr bool kMask = decltype(mask_c)::value;
        const bool cok = q0 + c16 < ncols;
#pragma unroll
        for (int h = 0; h < 2; ++h)
          *reinterpret_cast<f32x4*>(st + st_w[h]) = f32x4{xg[h][0], xg[h][1], xg[h][2], xg[h][3]};
        f32x4 acc[MTR];   // A(rows, j), then the residual
#pragma unroll
        for (int mt = 0; mt < MTR; ++mt) {
          const f32x4 v = *reinterpret_cast<const f32x4*>(st + st_r[mt]);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const float a = (!kMask || cok) ? v[e] : 0.0f;
            acc[mt][e] = a;
            as = __builtin_fmaf(a, a, as);
          }
        }
        const int qp = q0 % kCols + c16;           // column within the staged chunk
#pragma unroll
        for (int ks = 0; ks < KS32; ++ks) {
          if (ks >= ksn) break;     // uniform: zero terms add nothing
          const __bf16* pq = pt + qp * kPtStride + 32 * ks + 8 * g;
          const bf16x8 p0 = *reinterpret_cast<const bf16x8*>(pq);
          const bf16x8 p1 = *reinterpret_cast<const bf16x8*>(pq + KP);
          const bf16x8 p2 = *reinterpret_cast<const bf16x8*>(pq + 2 * KP);
#pragma unroll
          for (int mt = 0; mt < MTR; ++mt) {
            // largest terms first (p* are the terms of -P)
            acc[mt] = mfma_bf16(at[mt][ks][0], p0, acc[mt]);
            acc[mt] = mfma_bf16(at[mt][ks][0], p1, acc[mt]);
            acc[mt] = mfma_bf16(at[mt][ks][1], p0, acc[mt]);
            acc[mt] = mfma_bf16(at[mt][ks][0], p2, acc[mt]);
            acc[mt] = mfma_bf16(at[mt][ks][1], p1, acc[mt]);
            acc[mt] = mfma_bf16(at[mt][ks][2], p0, acc[mt]);
          }
        }
#pragma unroll
        for (int mt = 0; mt < MTR; ++mt)
#pragma unroll
          for (int v = 0; v < 4; ++v) es = __builtin_fmaf(acc[mt][v], acc[mt][v], es);
      };
#pragma unroll
      for (int gq = 0; gq < 2; ++gq) {
        const int q0 = 32 * s + 16 * gq;           // first column of the group
        if (q0 + 16 <= ncols) group(std::false_type{}, x[gq], q0);
        else group(std::true_type{}, x[gq], q0);
      }
      e2 += (double)es;
      a2 += (double)as;
    };
    int s = 0;
    if constexpr (kPf == 1) {
      float xa[2][2][4], xb[2][2][4];
      if constexpr (kPipeP) {
        load_p(0);
        load(0, xa);
        store_p(0);
        if (nst > 1) load_p(1);
      } else {
        load(0, xa);
      }
      for (; s + 1 < nst; s += 2) {
        step(xa, xb, s);
        step(xb, xa, s + 1);
      }
      if (s < nst) step(xa, xb, s);
    } else {
      // two steps of A in flight: step s reads buffer s % 3 and loads step
      // s + 2 into the buffer step s - 1 has finished with
      float xa[2][2][4], xb[2][2][4], xc[2][2][4];
      // step 0's P and A in flight while the selected columns are split;
      // each step's P issued before its A (the copy waits for no later A)
      load_p(0);
      load(0, xa);
      store_p(0);
      if (nst > 1) load_p(1);
      load(min(1, nst - 1), xb);
      for (; s + 3 <= nst; s += 3) {
        step(xa, xc, s);
        step(xb, xa, s + 1);
        step(xc, xb, s + 2);
      }
      if (s < nst) step(xa, xc, s);
      if (s + 1 < nst) step(xb, xa, s + 1);
    }
  };
  if (ncols > 0) {
    if (rbase + 16 * MTR <= bi.m) body(std::true_type{});
    else body(std::false_type{});
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

// Per-block sums of the row-tile partials, items of block b are the
// contiguous range [first[b], first[b+1]).  One wave per block: lane t sums
// items first + t, first + t + 64, ... in order, then a butterfly over the
// lanes; the order is fixed, so repeated runs give identical bits.
static __global__ __launch_bounds__(kWave) void recon_reduce_kernel(
    int nblocks, const int64_t* __restrict__ first, const double* __restrict__ part,
    double* __restrict__ err2, double* __restrict__ nrm2) {
  const int b = blockIdx.x;
  if (b >= nblocks) return;
  double e = 0.0, a = 0.0;
  for (int64_t x = first[b] + threadIdx.x; x < first[b + 1]; x += kWave) {
    e += part[2 * x];
    a += part[2 * x + 1];
  }
  e = wave_sum(e);
  a = wave_sum(a);
  if (threadIdx.x == 0) {
    err2[b] = e;
    nrm2[b] = a;
  }
}

// Widen the sketch to FP64 (diagnostics).
template <typename TY>
__global__ void copy_sketch_kernel(int64_t total, const TY* __restrict__ Y, double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < total) out[e] = (double)Y[e];
}

}  // namespace spid
