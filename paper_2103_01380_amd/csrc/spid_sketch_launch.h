// spid_sketch_launch.h -- dispatch of the sketch kernels over the launch-shape
// template parameters (16-row tiles MT, column tiles per wave TN, waves NW,
// vector loads VEC).  PR selects the arithmetic (kPrF64, kPrBF16, kPrFP8);
// each sketch source instantiates only its own.
#pragma once

#include "spid_internal.h"

namespace spid_host {

constexpr int kPrF64 = 0, kPrBF16 = 1, kPrFP8 = 2;

// ST: one-snapshot update of snapshot jst over the block groups; TAB: the
// bfloat16 kernel reads Omega from the per-update table (shared Omega only)
// batch: items [i0, i0 + ni) of the batch table (one TN group)
template <int PR, typename TA, int MT, int TN, int NW, bool VEC, bool ST, bool TAB>
void launch_sketch_k(spid_ctx* c, int j0, int j1, int jst, hipStream_t s, int64_t i0 = 0,
                     int64_t ni = 0) {
  const Plan& p = c->plan;
  const size_t nitems = ST ? p.sitems.size() : (size_t)ni;
  const SkItem* items = c->at<SkItem>(ST ? p.off_sitems : p.off_items) + (ST ? 0 : i0);
  const int32_t* perm = c->at<int32_t>(p.off_perm);
  dim3 grid((unsigned)nitems), block(64 * NW);
  // shapes the planner can choose (others are not instantiated): FP64 TN <= 2
  // (2 only for MT <= 4), FP8 TN = 1, BF16 TN = 4 only for MT < 6
  if constexpr (PR == kPrF64) {
    if constexpr (TN == 1 || (TN == 2 && MT <= 4))
      hipLaunchKernelGGL((sketch_f64_kernel<TA, MT, TN, NW, VEC, ST>), grid, block, 0, s,
                         c->at<BlkInfo>(p.off_blk), items, c->desc.l, c->desc.seed,
                         c->desc.omega_per_block, j0, j1, perm, jst,
                         p.omtab_cols > 0 ? c->at<double>(p.off_omtab) : nullptr,
                         c->at<double>(p.off_Y), c->at<double>(p.off_part));
  } else if constexpr (PR == kPrFP8) {
    if constexpr (TN == 1)
      hipLaunchKernelGGL((sketch_fp8_kernel<TA, MT, TN, NW, VEC, ST>), grid, block, 0, s,
                         c->at<BlkInfo>(p.off_blk), items, c->desc.l, c->desc.seed,
                         c->desc.omega_per_block, j0, j1, perm, jst, c->desc.lp_terms,
                         c->at<float>(p.off_Y), c->at<float>(p.off_part));
  } else {
    if constexpr (TN <= 2 || MT < 6)
      hipLaunchKernelGGL((sketch_bf16_kernel<TA, MT, TN, NW, VEC, ST, TAB>), grid, block, 0, s,
                         c->at<BlkInfo>(p.off_blk), items, c->desc.l, c->desc.seed,
                         c->desc.omega_per_block, j0, j1, perm, jst, c->desc.lp_terms,
                         TAB ? c->at<bf16x8>(p.off_omtab) : nullptr, c->at<float>(p.off_Y),
                         c->at<float>(p.off_part));
  }
}

// instantiated (TN, NW) pairs: 8 waves x 1-4 tiles or 4 waves x 1 tile
template <int PR, bool TAB, typename TA, int MT, int TN>
void launch_sketch_t(spid_ctx* c, int j0, int j1, hipStream_t s, int64_t i0, int64_t ni) {
  const bool vec = c->all_vec;
  if (c->plan.sh.NW == 8) {
    if (vec) launch_sketch_k<PR, TA, MT, TN, 8, true, false, TAB>(c, j0, j1, 0, s, i0, ni);
    else launch_sketch_k<PR, TA, MT, TN, 8, false, false, TAB>(c, j0, j1, 0, s, i0, ni);
  } else {
    if constexpr (TN == 1) {
      if (vec) launch_sketch_k<PR, TA, MT, 1, 4, true, false, TAB>(c, j0, j1, 0, s, i0, ni);
      else launch_sketch_k<PR, TA, MT, 1, 4, false, false, TAB>(c, j0, j1, 0, s, i0, ni);
    }
  }
}

// one launch per non-empty TN group of the batch items (widest tiles first)
template <int PR, bool TAB, typename TA, int MT>
void launch_sketch_mt(spid_ctx* c, int j0, int j1, hipStream_t s) {
  const int64_t* ts = c->plan.tn_start;
  if (ts[3] > ts[2]) launch_sketch_t<PR, TAB, TA, MT, 4>(c, j0, j1, s, ts[2], ts[3] - ts[2]);
  if (ts[2] > ts[1]) launch_sketch_t<PR, TAB, TA, MT, 2>(c, j0, j1, s, ts[1], ts[2] - ts[1]);
  if (ts[1] > ts[0]) launch_sketch_t<PR, TAB, TA, MT, 1>(c, j0, j1, s, ts[0], ts[1] - ts[0]);
}

template <int PR, bool TAB, typename TA>
void launch_sketch_a(spid_ctx* c, int j0, int j1, hipStream_t s) {
  switch (c->plan.sh.MT) {
    case 1: launch_sketch_mt<PR, TAB, TA, 1>(c, j0, j1, s); break;
    case 2: launch_sketch_mt<PR, TAB, TA, 2>(c, j0, j1, s); break;
    case 3: launch_sketch_mt<PR, TAB, TA, 3>(c, j0, j1, s); break;
    case 4: launch_sketch_mt<PR, TAB, TA, 4>(c, j0, j1, s); break;
    case 6: launch_sketch_mt<PR, TAB, TA, 6>(c, j0, j1, s); break;
    default: launch_sketch_mt<PR, TAB, TA, 8>(c, j0, j1, s); break;
  }
}

template <int PR, bool TAB = false>
void sketch_batch(spid_ctx* c, int j0, int j1, hipStream_t s) {
  if (c->desc.a_dtype == SPID_A_F64) launch_sketch_a<PR, TAB, double>(c, j0, j1, s);
  else launch_sketch_a<PR, TAB, float>(c, j0, j1, s);
}

// one-snapshot form: one 16-column tile per wave (the blocks of a group), or
// for FP8 the resident-Omega kernel (launcher supplied by the FP8 source)
template <int PR, typename TA, int MT>
bool launch_sketch_stream_mt(spid_ctx* c, int j, hipStream_t s);

template <int PR, typename TA, int MT>
bool launch_sketch_stream_plain(spid_ctx* c, int j, hipStream_t s) {
  constexpr bool kTab = PR == kPrBF16;   // one-snapshot updates need a shared Omega
  if (c->all_vec) launch_sketch_k<PR, TA, MT, 1, kStreamNW, true, true, kTab>(c, 0, 0, j, s);
  else launch_sketch_k<PR, TA, MT, 1, kStreamNW, false, true, kTab>(c, 0, 0, j, s);
  return true;
}

template <int PR, typename TA>
bool launch_sketch_stream_a(spid_ctx* c, int j, hipStream_t s) {
  switch (c->plan.sh.MT) {
    case 1: return launch_sketch_stream_mt<PR, TA, 1>(c, j, s);
    case 2: return launch_sketch_stream_mt<PR, TA, 2>(c, j, s);
    case 3: return launch_sketch_stream_mt<PR, TA, 3>(c, j, s);
    case 4: return launch_sketch_stream_mt<PR, TA, 4>(c, j, s);
    case 6: return launch_sketch_stream_mt<PR, TA, 6>(c, j, s);
    default: return launch_sketch_stream_mt<PR, TA, 8>(c, j, s);
  }
}

template <int PR>
bool sketch_stream(spid_ctx* c, int j, hipStream_t s) {
  if (c->desc.a_dtype == SPID_A_F64) return launch_sketch_stream_a<PR, double>(c, j, s);
  return launch_sketch_stream_a<PR, float>(c, j, s);
}

}  // namespace spid_host
