// spid_sketch_f64.hip -- double-precision sketch launches (FP64 matrix cores).
#include "spid_sketch_launch.h"

namespace spid_host {

template <int PR, typename TA, int MT>
bool launch_sketch_stream_mt(spid_ctx* c, int j, hipStream_t s) {
  return launch_sketch_stream_plain<PR, TA, MT>(c, j, s);
}

void sketch_batch_f64(spid_ctx* c, int j0, int j1, hipStream_t s) {
  sketch_batch<kPrF64>(c, j0, j1, s);
}

bool sketch_stream_f64(spid_ctx* c, int j, hipStream_t s) { return sketch_stream<kPrF64>(c, j, s); }

}  // namespace spid_host
