// spid_sketch_bf16.hip -- bfloat16 sketch launches (split-term A, FP32 accumulation).
#include "spid_sketch_launch.h"

namespace spid_host {

template <int PR, typename TA, int MT>
bool launch_sketch_stream_mt(spid_ctx* c, int j, hipStream_t s) {
  return launch_sketch_stream_plain<PR, TA, MT>(c, j, s);
}

void sketch_batch_bf16(spid_ctx* c, int j0, int j1, hipStream_t s) {
  sketch_batch<kPrBF16>(c, j0, j1, s);
}

bool sketch_stream_bf16(spid_ctx* c, int j, hipStream_t s) {
  return sketch_stream<kPrBF16>(c, j, s);
}

}  // namespace spid_host
