// spid_sketch_bf16.hip -- bfloat16 sketch launches (split-term A, FP32
// accumulation) with Omega keyed per block, regenerated in the kernels; the
// shared-Omega launches read the per-update table (spid_sketch_bf16_tab.hip).
#include "spid_sketch_launch.h"

namespace spid_host {

void sketch_batch_bf16(spid_ctx* c, int j0, int j1, hipStream_t s) {
  if (c->plan.omtab_cols > 0) sketch_batch_bf16_tab(c, j0, j1, s);
  else sketch_batch<kPrBF16, false>(c, j0, j1, s);
}

}  // namespace spid_host
