// spid_sketch_bf16_tab.hip -- bfloat16 sketch launches with Omega shared by
// all blocks (Section 2): the sketch matrix is regenerated once per update as a
// table in MFMA operand order and read by the batch and one-snapshot kernels;
// the launch of every Omega table (double, bfloat16, and e4m3 for the FP8
// one-snapshot kernel).
#include "spid_sketch_launch.h"

namespace spid_host {

bool launch_omega_table(spid_ctx* c, hipStream_t s) {
  const Plan& p = c->plan;
  const int64_t n = (int64_t)p.sh.MT * 8 * p.omtab_cols;   // pairs of rows x columns
  const dim3 grid((unsigned)((n + 255) / 256));
  if (c->desc.prec == SPID_SK_BF16)
    hipLaunchKernelGGL((omega_table_kernel<0>), grid, dim3(256), 0, s, c->desc.l, p.sh.MT,
                       p.omtab_cols, c->desc.seed, c->at<__bf16>(p.off_omtab));
  else if (c->desc.prec == SPID_SK_F64)
    hipLaunchKernelGGL((omega_table_f64_kernel<double>), grid, dim3(256), 0, s, c->desc.l, p.sh.MT,
                       p.omtab_cols, c->desc.seed, c->at<double>(p.off_omtab));
  else
    hipLaunchKernelGGL((omega_table_e4m3_kernel<uint8_t>), grid, dim3(256), 0, s, c->desc.l,
                       p.sh.MT, p.omtab_cols, c->desc.seed, c->at<uint8_t>(p.off_omtab));
  return hipGetLastError() == hipSuccess;
}

void sketch_batch_bf16_tab(spid_ctx* c, int j0, int j1, hipStream_t s) {
  sketch_batch<kPrBF16, true>(c, j0, j1, s);
}

template <int PR, typename TA, int MT>
bool launch_sketch_stream_mt(spid_ctx* c, int j, hipStream_t s) {
  return launch_sketch_stream_plain<PR, TA, MT>(c, j, s);
}

bool sketch_stream_bf16(spid_ctx* c, int j, hipStream_t s) {
  return sketch_stream<kPrBF16>(c, j, s);
}

}  // namespace spid_host
