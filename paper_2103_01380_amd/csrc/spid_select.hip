// spid_select.hip -- launches of the column-selection kernels (pivoted
// modified Gram-Schmidt on the sketch, Algorithm 1 of arXiv 2103.01380).
#include "spid_internal.h"

namespace spid_host {


// register kernel: groups of LPC lanes holding 4 columns, RPT rows per lane,
// one barrier per step
template <typename TY, int RPT, int LPC, int MAXTHR>
void launch_select_step(const SelJob<TY>& j, hipStream_t s) {
  hipLaunchKernelGGL((select_step_kernel<TY, RPT, LPC, 4, MAXTHR>), dim3(j.nblocks),
                     dim3(j.sh.sel_thr), 0, s, j.blks, j.l, j.k_max, j.tol, j.rank_floor, j.Y,
                     j.R, j.S, j.k, j.st);
}

template <typename TY, int LPC, int MAXTHR>
void launch_select_rpt(const SelJob<TY>& j, hipStream_t s) {
  // rows per lane: ceil(l / LPC) in fours, so LPC = 4, 8 (l > 32) take 12 or 16
  if constexpr (LPC == 2) {
    if (j.sh.sel_rpt == 4) return launch_select_step<TY, 4, LPC, MAXTHR>(j, s);
    if (j.sh.sel_rpt == 8) return launch_select_step<TY, 8, LPC, MAXTHR>(j, s);
  }
  if (j.sh.sel_rpt == 12) launch_select_step<TY, 12, LPC, MAXTHR>(j, s);
  else launch_select_step<TY, 16, LPC, MAXTHR>(j, s);
}

template <typename TY, int RR, int MAXTHR>
bool launch_select_hybrid_t(const SelJob<TY>& j, hipStream_t s) {
  auto kern = select_hybrid_kernel<TY, RR, MAXTHR>;
  if (!allow_lds((const void*)kern, j.sh.sel_lds)) return false;
  hipLaunchKernelGGL(kern, dim3(j.nblocks), dim3(j.sh.sel_thr), j.sh.sel_lds, s, j.blks, j.l,
                     j.k_max, j.tol, j.rank_floor, j.Y, j.R, j.S, j.k, j.st);
  return true;
}

template <typename TY>
bool select_job_t(const SelJob<TY>& j, hipStream_t s) {
  const SelShape& sh = j.sh;
  if (sh.sel_tall) {
    if constexpr (std::is_same<TY, double>::value) {
      auto launch = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(j.nblocks), dim3(kTallThreads), 0, s, j.blks, j.l,
                           j.k_max, j.tol, j.rank_floor, j.Y, j.W, j.R, j.S, j.k, j.st);
      };
      if (j.l <= 4 * kWave) launch(select_tall_kernel<4>);
      else if (j.l <= 8 * kWave) launch(select_tall_kernel<8>);
      else if (j.l <= 16 * kWave) launch(select_tall_kernel<16>);
      else launch(select_tall_kernel<0>);
      return true;
    }
    return false;   // tall sketches are double precision
  }
  if (sh.sel_lpc) {
    if (sh.sel_lpc == 2) launch_select_rpt<TY, 2, 256>(j, s);
    else if (sh.sel_lpc == 4) launch_select_rpt<TY, 4, 512>(j, s);
    else launch_select_rpt<TY, 8, 768>(j, s);
    return true;
  }
  if (sh.sel_rr) {
    if (sh.sel_thr > 512) {
      if (sh.sel_rr == 32) return launch_select_hybrid_t<TY, 32, 1024>(j, s);
      return launch_select_hybrid_t<TY, 16, 1024>(j, s);
    }
    if (sh.sel_rr == 48) return launch_select_hybrid_t<TY, 48, 512>(j, s);
    if (sh.sel_rr == 32) return launch_select_hybrid_t<TY, 32, 512>(j, s);
    return launch_select_hybrid_t<TY, 16, 512>(j, s);
  }
  return false;   // pick_sel leaves no other case
}

// Row-split selection of a few very tall coarse sketches: init, then three launches per
// step and a final pivot launch (blocks that stopped return at once).
bool launch_select_split(spid_ctx* c, hipStream_t s) {
  const Plan& p = c->plan;
  const spid_desc& d = c->desc;
  const int nb = d.nblocks;
  const BlkInfo* blks = c->at<BlkInfo>(p.off_blk);
  const int64_t* poff = c->at<int64_t>(p.off_spoff);
  double* pnorm = c->at<double>(p.off_spnorm);
  double* pdot = c->at<double>(p.off_spdot);
  unsigned char* used = c->at<unsigned char>(p.off_spused);
  SplitState* st = c->at<SplitState>(p.off_spstate);
  int32_t* bad = c->at<int32_t>(p.off_spbad);
  double* W = c->at<double>(p.off_W);
  double* R = c->at<double>(p.off_R);
  int32_t* S = c->at<int32_t>(p.off_S);
  int32_t* k = c->at<int32_t>(p.off_k);
  int32_t* sts = c->at<int32_t>(p.off_st);
  const dim3 g2((unsigned)p.split_nch, (unsigned)nb);
  hipLaunchKernelGGL(split_clear_kernel, dim3((nb + 255) / 256), dim3(256), 0, s, nb, bad);
  hipLaunchKernelGGL(split_init_kernel, g2, dim3(kSplitThreads), 0, s, blks, d.l,
                     c->at<double>(p.off_Y), W, poff, pnorm, bad);
  const int kcap = std::min(d.k_max, std::min(d.l, p.max_n));
  for (int step = 0; step <= kcap; ++step) {
    hipLaunchKernelGGL(split_pivot_kernel, dim3(nb), dim3(kSplitThreads), 0, s, blks, d.l,
                       d.k_max, d.tol, d.rank_floor, step, poff, pnorm, used, st, bad, R, S, k,
                       sts);
    if (step == kcap) break;
    hipLaunchKernelGGL(split_dot_kernel, g2, dim3(kSplitThreads), 0, s, blks, d.l, poff, st,
                       used, W, pdot);
    hipLaunchKernelGGL(split_update_kernel, g2, dim3(kSplitThreads), 0, s, blks, d.l, step, poff,
                       st, used, pdot, W, pnorm, R);
  }
  return true;
}

bool launch_select_job_f64(const SelJob<double>& j, hipStream_t s) { return select_job_t(j, s); }
bool launch_select_job_f32(const SelJob<float>& j, hipStream_t s) { return select_job_t(j, s); }

bool launch_select_ctx(spid_ctx* c, hipStream_t s) {
  const Plan& p = c->plan;
  if (p.ydt == 0) {
    if (p.split) return launch_select_split(c, s);
    SelJob<double> j{c->at<BlkInfo>(p.off_blk), c->desc.nblocks, c->desc.l, c->desc.k_max,
                     c->desc.tol, c->desc.rank_floor, c->at<double>(p.off_Y),
                     c->at<double>(p.off_W), c->at<double>(p.off_R), c->at<int32_t>(p.off_S),
                     c->at<int32_t>(p.off_k), c->at<int32_t>(p.off_st), p.sh.sel};
    return select_job_t<double>(j, s);
  }
  SelJob<float> j{c->at<BlkInfo>(p.off_blk), c->desc.nblocks, c->desc.l, c->desc.k_max,
                  c->desc.tol, c->desc.rank_floor, c->at<float>(p.off_Y), c->at<double>(p.off_W),
                  c->at<double>(p.off_R), c->at<int32_t>(p.off_S), c->at<int32_t>(p.off_k),
                  c->at<int32_t>(p.off_st), p.sh.sel};
  return select_job_t<float>(j, s);
}

}  // namespace spid_host
