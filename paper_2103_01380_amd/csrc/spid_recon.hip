// spid_recon.hip -- launches of the coefficient kernels (back-substitution,
// Algorithm 1 of arXiv 2103.01380) and of the error passes (Section 5.1; the
// single-pass form of Algorithm 3 for the coarse-grid sketch).
#include "spid_internal.h"

namespace spid_host {

// one attribute call per kernel instantiation for dynamic LDS above 64 KiB
template <typename TA, int KS, int MTR>
bool launch_recon_t(spid_ctx* c, const double* P, void* skel, hipStream_t s) {
  const Plan& p = c->plan;
  const size_t lds = sizeof(double) * p.sh.PCAP * (4 * KS + 1);
  auto launch = [&](auto kern) {
    if (!allow_lds((const void*)kern, lds)) return false;
    hipLaunchKernelGGL(kern, dim3(p.rc_xcd_grid), dim3(kRcThreads), lds, s,
                       c->at<BlkInfo>(p.off_blk), c->at<RcItem>(p.off_rc), p.rc_xcd, c->desc.k_max,
                       p.sh.PCAP, c->at<int32_t>(p.off_S), c->at<int32_t>(p.off_k), P,
                       static_cast<TA*>(skel), c->at<double>(p.off_rcpart));
    return true;
  };
  if (c->all_vec4) return launch(recon_mfma_kernel<TA, KS, MTR, true>);
  return launch(recon_mfma_kernel<TA, KS, MTR, false>);
}

// single-precision data on the mixed path: split-bfloat16 error pass
template <int KS32, int MTR>
bool launch_recon_bf16_t(spid_ctx* c, const double* P, void* skel, hipStream_t s) {
  (void)P;   // the split coefficients written by spid_coeffs are used
  const Plan& p = c->plan;
  auto launch = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(p.rc_xcd_grid), dim3(kRcThreads), 0, s,
                       c->at<BlkInfo>(p.off_blk), c->at<RcItem>(p.off_rc), p.rc_xcd, c->desc.l,
                       c->desc.k_max, c->at<int32_t>(p.off_S), c->at<int32_t>(p.off_k),
                       c->at<__bf16>(p.off_pt), c->at<int32_t>(p.off_cols),
                       c->at<int32_t>(p.off_ncols), static_cast<float*>(skel),
                       c->at<double>(p.off_rcpart));
  };
  if (c->all_vec4) launch(recon_bf16x3_kernel<KS32, MTR, true>);
  else launch(recon_bf16x3_kernel<KS32, MTR, false>);
  return true;
}

template <typename TA>
bool launch_recon_a(spid_ctx* c, const double* P, void* skel, hipStream_t s) {
  const Shape& sh = c->plan.sh;
  if constexpr (sizeof(TA) == 4) {
    if (sh.rc_bf16) {
      switch (sh.KS32) {
        case 1: return launch_recon_bf16_t<1, 2>(c, P, skel, s);
        case 2: return launch_recon_bf16_t<2, 2>(c, P, skel, s);
        default: return launch_recon_bf16_t<3, 2>(c, P, skel, s);
      }
    }
  }
  switch (sh.KS) {
    case 1: return launch_recon_t<TA, 1, 4>(c, P, skel, s);
    case 2: return launch_recon_t<TA, 2, 4>(c, P, skel, s);
    case 4: return launch_recon_t<TA, 4, 4>(c, P, skel, s);
    case 8: return launch_recon_t<TA, 8, 4>(c, P, skel, s);
    case 12: return launch_recon_t<TA, 12, 2>(c, P, skel, s);
    case 16: return launch_recon_t<TA, 16, 2>(c, P, skel, s);
    default: return launch_recon_t<TA, 24, 2>(c, P, skel, s);
  }
}

template <int KB>
bool launch_coeffs_t(spid_ctx* c, double* P, hipStream_t s) {
  const Plan& p = c->plan;
  const size_t lds = coeffs_lds_bytes(KB);
  if (!allow_lds((const void*)coeffs_kernel<KB>, lds)) return false;
  const bool bf = p.sh.rc_bf16 != 0;
  if (bf && p.sh.KS32 != (KB + 1) / 2) return false;   // the terms' pieces cover 32 KS32 rows
  hipLaunchKernelGGL((coeffs_kernel<KB>), dim3(c->desc.nblocks), dim3(kCoThreads), lds, s,
                     c->at<BlkInfo>(p.off_blk), c->desc.l, c->desc.k_max, c->at<double>(p.off_R),
                     c->at<int32_t>(p.off_S), c->at<int32_t>(p.off_k), P,
                     bf ? c->at<__bf16>(p.off_pt) : nullptr, 32 * p.sh.KS32,
                     bf ? c->at<int32_t>(p.off_cols) : nullptr,
                     bf ? c->at<int32_t>(p.off_ncols) : nullptr);
  return true;
}

template <typename TA, int KS, int MTR>
bool launch_interp_t(spid_ctx* c, const double* P, hipStream_t s) {
  const Plan& p = c->plan;
  const size_t lds = sizeof(double) * p.sh.PCAP * (4 * KS + 1);
  auto launch = [&](auto kern) {
    if (!allow_lds((const void*)kern, lds)) return false;
    hipLaunchKernelGGL(kern, dim3(p.rc_xcd_grid), dim3(kRcThreads), lds, s,
                       c->at<BlkInfo>(p.off_blk), c->at<GridInfo>(p.off_grid),
                       c->at<RcItem>(p.off_rc), p.rc_xcd, c->desc.l, c->desc.k_max,
                       p.sh.PCAP,
                       c->at<int32_t>(p.off_S), c->at<int32_t>(p.off_k),
                       c->at<double>(p.off_Y), P, c->at<double>(p.off_rcpart));
    return true;
  };
  if (c->all_vec4) return launch(interp_mfma_kernel<TA, KS, MTR, true>);
  return launch(interp_mfma_kernel<TA, KS, MTR, false>);
}

template <typename TA>
bool launch_interp_a(spid_ctx* c, const double* P, void* cskel, hipStream_t s) {
  bool ok;
  switch (c->plan.sh.KS) {
    case 1: ok = launch_interp_t<TA, 1, 4>(c, P, s); break;
    case 2: ok = launch_interp_t<TA, 2, 4>(c, P, s); break;
    case 4: ok = launch_interp_t<TA, 4, 4>(c, P, s); break;
    case 8: ok = launch_interp_t<TA, 8, 4>(c, P, s); break;
    case 12: ok = launch_interp_t<TA, 12, 2>(c, P, s); break;
    case 16: ok = launch_interp_t<TA, 16, 2>(c, P, s); break;
    default: ok = launch_interp_t<TA, 24, 2>(c, P, s); break;
  }
  if (!ok) return false;
  if (cskel) {
    const Plan& p = c->plan;
    int mcmax = 1;
    for (const GridInfo& g : p.grid) mcmax = std::max(mcmax, g.mc);
    const int64_t per_blk = (int64_t)mcmax * c->desc.k_max;
    dim3 grid((unsigned)std::min<int64_t>((per_blk + 255) / 256, 1 << 20),
              (unsigned)std::min(c->desc.nblocks, 65535));
    hipLaunchKernelGGL((coarse_skeleton_kernel<TA>), grid, dim3(256), 0, s,
                       c->at<BlkInfo>(p.off_blk), c->at<GridInfo>(p.off_grid), c->desc.nblocks,
                       c->desc.l, c->desc.k_max, c->at<int32_t>(p.off_S),
                       c->at<int32_t>(p.off_k), c->at<double>(p.off_Y), static_cast<TA*>(cskel));
  }
  return true;
}

template <int KB>
bool launch_coeffs_job(const BlkInfo* blks, int nblocks, int l, int k_max, const double* R,
                       const int32_t* S, const int32_t* k, double* P, hipStream_t s) {
  const size_t lds = coeffs_lds_bytes(KB);
  if (!allow_lds((const void*)coeffs_kernel<KB>, lds)) return false;
  hipLaunchKernelGGL((coeffs_kernel<KB>), dim3(nblocks), dim3(kCoThreads), lds, s, blks, l,
                     k_max, R, S, k, P, (__bf16*)nullptr, 32, (int32_t*)nullptr,
                     (int32_t*)nullptr);
  return true;
}

bool launch_coeffs_any(int kmax_t, const BlkInfo* blks, int nblocks, int l, int k_max,
                       const double* R, const int32_t* S, const int32_t* k, double* P,
                       hipStream_t s) {
  switch (kmax_t) {
    case 8:
    case 16: return launch_coeffs_job<1>(blks, nblocks, l, k_max, R, S, k, P, s);
    case 32: return launch_coeffs_job<2>(blks, nblocks, l, k_max, R, S, k, P, s);
    case 48: return launch_coeffs_job<3>(blks, nblocks, l, k_max, R, S, k, P, s);
    case 64: return launch_coeffs_job<4>(blks, nblocks, l, k_max, R, S, k, P, s);
    default: return launch_coeffs_job<6>(blks, nblocks, l, k_max, R, S, k, P, s);
  }
}

bool launch_coeffs_ctx(spid_ctx* c, double* P, hipStream_t s) {
  switch (c->plan.sh.KMAX) {
    case 8:
    case 16: return launch_coeffs_t<1>(c, P, s);
    case 32: return launch_coeffs_t<2>(c, P, s);
    case 48: return launch_coeffs_t<3>(c, P, s);
    case 64: return launch_coeffs_t<4>(c, P, s);
    default: return launch_coeffs_t<6>(c, P, s);
  }
}

bool launch_recon_ctx(spid_ctx* c, const double* P, void* skel, hipStream_t s) {
  return c->desc.a_dtype == SPID_A_F64 ? launch_recon_a<double>(c, P, skel, s)
                                       : launch_recon_a<float>(c, P, skel, s);
}

bool launch_interp_ctx(spid_ctx* c, const double* P, void* cskel, hipStream_t s) {
  return c->desc.a_dtype == SPID_A_F64 ? launch_interp_a<double>(c, P, cskel, s)
                                       : launch_interp_a<float>(c, P, cskel, s);
}

}  // namespace spid_host
