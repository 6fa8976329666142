// spid_sketch_fp8.hip -- e4m3 sketch launches (split-term A with per-32-row
// scales, FP32 accumulation), including the whole-K one-snapshot kernel.
#include "spid_sketch_launch.h"

namespace spid_host {

template <int MT, bool VEC>
bool launch_fp8_stream(spid_ctx* c, int j, hipStream_t s) {
  const Plan& p = c->plan;
  hipLaunchKernelGGL((sketch_fp8_stream_kernel<MT, kStreamNW, VEC>),
                     dim3((unsigned)(p.ritems.size() / 3)), dim3(64 * kStreamNW), 0, s,
                     c->at<BlkInfo>(p.off_blk), c->at<SkItem>(p.off_sitems),
                     c->at<int32_t>(p.off_ritems), c->desc.l, c->at<i32x4>(p.off_omtab),
                     c->at<int32_t>(p.off_perm), j, c->desc.lp_terms, c->at<float>(p.off_Y));
  return true;
}

// FP32 data: the whole-K streaming kernel; FP64 data: the plain one-snapshot shape
template <int PR, typename TA, int MT>
bool launch_sketch_stream_mt(spid_ctx* c, int j, hipStream_t s) {
  if constexpr (std::is_same<TA, float>::value) {
    if (!c->plan.ritems.empty())
      return c->all_vec ? launch_fp8_stream<MT, true>(c, j, s) : launch_fp8_stream<MT, false>(c, j, s);
  }
  return launch_sketch_stream_plain<PR, TA, MT>(c, j, s);
}

void sketch_batch_fp8(spid_ctx* c, int j0, int j1, hipStream_t s) {
  sketch_batch<kPrFP8>(c, j0, j1, s);
}

bool sketch_stream_fp8(spid_ctx* c, int j, hipStream_t s) { return sketch_stream<kPrFP8>(c, j, s); }

}  // namespace spid_host
