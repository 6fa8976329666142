// spid_sketch_fp8.hip -- e4m3 sketch launches (split-term A with per-32-row
// scales, FP32 accumulation), including the resident-Omega one-snapshot kernel.
#include "spid_sketch_launch.h"

namespace spid_host {

template <typename TA, int MT, bool VEC>
bool launch_fp8_resident(spid_ctx* c, int j, hipStream_t s) {
  const Plan& p = c->plan;
  const size_t lds = (size_t)kResChunks * MT * 16 * kOm8Stride;
  auto kern = sketch_fp8_resident_kernel<TA, MT, kStreamNW, VEC>;
  if (!allow_lds((const void*)kern, lds)) return false;
  hipLaunchKernelGGL(kern, dim3((unsigned)(p.ritems.size() / 3)), dim3(64 * kStreamNW), lds, s,
                     c->at<BlkInfo>(p.off_blk), c->at<SkItem>(p.off_sitems),
                     c->at<int32_t>(p.off_ritems), c->desc.l, c->at<uint8_t>(p.off_omtab),
                     c->at<int32_t>(p.off_perm), j, c->desc.lp_terms, c->at<float>(p.off_Y),
                     c->at<float>(p.off_part));
  return true;
}

template <int PR, typename TA, int MT>
bool launch_sketch_stream_mt(spid_ctx* c, int j, hipStream_t s) {
  if (!c->plan.ritems.empty())
    return c->all_vec ? launch_fp8_resident<TA, MT, true>(c, j, s)
                      : launch_fp8_resident<TA, MT, false>(c, j, s);
  return launch_sketch_stream_plain<PR, TA, MT>(c, j, s);
}

void sketch_batch_fp8(spid_ctx* c, int j0, int j1, hipStream_t s) {
  sketch_batch<kPrFP8>(c, j0, j1, s);
}

bool sketch_stream_fp8(spid_ctx* c, int j, hipStream_t s) { return sketch_stream<kPrFP8>(c, j, s); }

}  // namespace spid_host
