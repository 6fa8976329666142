// spid.hip -- host side of the C ABI declared in include/spid.h: descriptor
// validation, workspace planning, work-item tables and kernel dispatch for
// gfx950.  Every compute entry point only enqueues kernels on the caller's
// stream.
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "spid_internal.h"

using namespace spid;

namespace spid_host {

namespace {
thread_local std::string g_err;
}

spid_status fail(spid_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

spid_status hip_check(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(SPID_EHIP, "%s: %s", what, hipGetErrorString(e));
  return SPID_OK;
}

bool allow_lds(const void* kernel, size_t bytes) {
  if (bytes <= 65536) return true;
  return hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) ==
         hipSuccess;
}

namespace {

spid_status validate(const spid_desc* d) {
  if (!d) return fail(SPID_EINVAL, "descriptor is NULL");
  if (d->nblocks < 1) return fail(SPID_EINVAL, "nblocks must be >= 1 (got %d)", d->nblocks);
  if (!d->h_m || !d->h_n) return fail(SPID_EINVAL, "h_m and h_n must be host arrays");
  const bool coarse = d->prec == SPID_SK_SUBSAMPLE;
  if (!coarse && (d->l < 1 || d->l > kMaxL))
    return fail(SPID_EINVAL, "l must be in [1, %d] (got %d)", kMaxL, d->l);
  if (coarse && (d->l < 1 || d->l > kMaxLCoarse))
    return fail(SPID_EINVAL, "coarse-grid sketch: l must be in [1, %d] (got %d)", kMaxLCoarse,
                d->l);
  if (d->k_max < 1 || d->k_max > kMaxK)
    return fail(SPID_EINVAL, "k_max must be in [1, %d] (got %d)", kMaxK, d->k_max);
  if (!(d->tol >= 0.0)) return fail(SPID_EINVAL, "tol must be >= 0");
  if (!(d->rank_floor >= 0.0)) return fail(SPID_EINVAL, "rank_floor must be >= 0");
  if (d->a_dtype != SPID_A_F64 && d->a_dtype != SPID_A_F32)
    return fail(SPID_EINVAL, "a_dtype must be SPID_A_F64 or SPID_A_F32");
  if (d->prec != SPID_SK_F64 && d->prec != SPID_SK_BF16 && d->prec != SPID_SK_FP8E4M3 && !coarse)
    return fail(SPID_EINVAL,
                "sketch must be SPID_SK_F64, _BF16, _FP8E4M3 or _SUBSAMPLE (got %d)", d->prec);
  if (coarse && !d->h_grid)
    return fail(SPID_EINVAL, "coarse-grid sketch: h_grid must be a host array of block grids");
  if (d->ts_windows < 0) return fail(SPID_EINVAL, "ts_windows must be >= 0");
  if (d->ts_windows > 0) {
    if (d->ts_k1 < 1 || d->ts_k1 > kMaxK)
      return fail(SPID_EINVAL, "two-stage: ts_k1 must be in [1, %d] (got %d)", kMaxK, d->ts_k1);
    if ((int64_t)d->ts_windows * d->ts_k1 > kMaxN)
      return fail(SPID_EINVAL, "two-stage: ts_windows * ts_k1 must be <= %d", kMaxN);
    if (d->a_dtype == SPID_A_F32 && (d->prec == SPID_SK_BF16 || d->prec == SPID_SK_FP8E4M3))
      return fail(SPID_EINVAL,
                  "two-stage: not available with FP32 data and a BF16/FP8 sketch (the "
                  "split-bfloat16 error pass needs spid_coeffs)");
  }
  if ((d->prec == SPID_SK_BF16 || d->prec == SPID_SK_FP8E4M3) &&
      (d->lp_terms < 1 || d->lp_terms > 3))
    return fail(SPID_EINVAL, "lp_terms must be 1..3 (got %d)", d->lp_terms);
  for (int b = 0; b < d->nblocks; ++b) {
    const int64_t m = d->h_m[b];
    const int32_t n = d->h_n[b];
    if (m < 1 || m >= (int64_t(1) << 31))
      return fail(SPID_EINVAL, "block %d: m must be in [1, 2^31) (got %lld)", b, (long long)m);
    if (n < 1 || n > kMaxN)
      return fail(SPID_EINVAL, "block %d: n must be in [1, %d] (got %d)", b, kMaxN, n);
    if (d->tol == 0.0 && (d->k_max > d->l || d->k_max > n))
      return fail(SPID_EINVAL,
                  "block %d: fixed rank k_max=%d exceeds min(l=%d, n=%d)", b, d->k_max, d->l, n);
    if (d->ts_windows > n)
      return fail(SPID_EINVAL, "block %d: %d windows exceed n = %d", b, d->ts_windows, n);
    if (coarse) {
      const spid_grid& g = d->h_grid[b];
      if (g.nx < 1 || g.ny < 1 || g.nz < 1 || g.nfields < 1 || g.sx < 1 || g.sy < 1 || g.sz < 1)
        return fail(SPID_EINVAL, "block %d: grid sizes and intervals must be >= 1", b);
      const int64_t pts = (int64_t)g.nx * g.ny * g.nz * g.nfields;
      if (pts != m)
        return fail(SPID_EINVAL, "block %d: grid has %lld rows, m = %lld", b, (long long)pts,
                    (long long)m);
      const int64_t mc = (int64_t)g.nfields * ((g.nx + g.sx - 1) / g.sx) *
                         ((g.ny + g.sy - 1) / g.sy) * ((g.nz + g.sz - 1) / g.sz);
      if (mc > d->l)
        return fail(SPID_EINVAL, "block %d: %lld coarse rows exceed l = %d", b, (long long)mc,
                    d->l);
    }
  }
  return SPID_OK;
}

spid_status validate_tuning(const spid_desc* d, const spid_tuning* t, int mt) {
  if (!t) return SPID_OK;
  if (t->sk_tn != 0 && t->sk_tn != 1 && t->sk_tn != 2 && t->sk_tn != 4)
    return fail(SPID_EINVAL, "tuning: sk_tn must be 0, 1, 2 or 4 (got %d)", t->sk_tn);
  if (t->sk_tn != 0) {
    const bool f64 = d->prec == SPID_SK_F64;
    if (f64 && (t->sk_tn == 4 || (t->sk_tn == 2 && mt > 4)))
      return fail(SPID_EINVAL, "tuning: sk_tn=%d not available for the FP64 sketch with l=%d",
                  t->sk_tn, d->l);
    if (d->prec == SPID_SK_BF16 && t->sk_tn == 4 && mt >= 6)
      return fail(SPID_EINVAL, "tuning: sk_tn=4 not available for the BF16 sketch with l=%d", d->l);
    if (d->prec == SPID_SK_FP8E4M3 && t->sk_tn != 1)
      return fail(SPID_EINVAL, "tuning: the FP8 sketch takes sk_tn=1 (got %d)", t->sk_tn);
  }
  if (t->sk_nw != 0 && t->sk_nw != 4 && t->sk_nw != 8)
    return fail(SPID_EINVAL, "tuning: sk_nw must be 0, 4 or 8 (got %d)", t->sk_nw);
  if (t->sk_items != 0 && (t->sk_items < 64 || t->sk_items > 65536))
    return fail(SPID_EINVAL, "tuning: sk_items must be 0 or 64..65536 (got %d)", t->sk_items);
  if (t->rc_rpi < 0 || t->rc_rpi > 16)
    return fail(SPID_EINVAL, "tuning: rc_rpi must be 0..16 (got %d)", t->rc_rpi);
  if (t->st_groups < 0 || t->st_groups > 16)
    return fail(SPID_EINVAL, "tuning: st_groups must be 0..16 (got %d)", t->st_groups);
  return SPID_OK;
}

spid_status make_plan(const spid_desc* d, const spid_tuning* tune, Plan& p) {
  spid_status st = validate(d);
  if (st != SPID_OK) return st;
  st = validate_tuning(d, tune, pick_mt(d->l));
  if (st != SPID_OK) return st;
  const int nb = d->nblocks;
  p.coarse = d->prec == SPID_SK_SUBSAMPLE;
  p.ydt = (d->prec == SPID_SK_F64 || p.coarse) ? 0 : 1;
  for (int b = 0; b < nb; ++b) {
    p.sum_n += d->h_n[b];
    p.sum_m += d->h_m[b];
    p.max_n = std::max(p.max_n, (int)d->h_n[b]);
  }
  Shape& sh = p.sh;
  sh.MT = pick_mt(d->l);
  // columns per workgroup tile: 64*TN
  if (p.ydt == 0) {
    // FP64 MFMA needs two waves per SIMD: 8 waves of 1-2 column tiles
    sh.TN = (p.max_n >= 256 && sh.MT <= 4) ? 2 : 1;
    sh.NW = p.max_n >= 128 ? 8 : 4;
  } else {
    // 8 waves (two per SIMD) of up to 4 column tiles: 512 columns per workgroup
    sh.TN = p.max_n >= 512 ? 4 : (p.max_n >= 256 ? 2 : 1);
    if (sh.MT >= 6 && sh.TN > 2) sh.TN = 2;
    if (d->prec == SPID_SK_FP8E4M3) sh.TN = 1;
    sh.NW = p.max_n >= 128 ? 8 : 4;
  }
  if (tune && tune->sk_tn) sh.TN = tune->sk_tn;
  if (tune && tune->sk_nw) sh.NW = tune->sk_nw;
  if (sh.NW == 4 && sh.TN != 1) {
    if (tune && tune->sk_nw == 4) return fail(SPID_EINVAL, "tuning: sk_nw=4 requires sk_tn=1");
    sh.NW = 8;
  }
  if (!pick_sel(d->l, p.max_n, p.coarse, sh.sel))
    return fail(SPID_EINVAL, "l=%d with n up to %d exceeds the selection register/LDS budget",
                d->l, p.max_n);
  sh.KMAX = pick_kmax(d->k_max);
  {
    const int ks = (d->k_max + 3) / 4;
    const int opts[] = {1, 2, 4, 8, 12, 16, 24};
    sh.KS = 24;
    for (int o : opts)
      if (ks <= o) {
        sh.KS = o;
        break;
      }
    sh.rc_bf16 = (d->a_dtype == SPID_A_F32 &&
                  (d->prec == SPID_SK_BF16 || d->prec == SPID_SK_FP8E4M3)) ? 1 : 0;
    sh.KS32 = (d->k_max + 31) / 32;
    sh.MTR = sh.rc_bf16 ? 2 : (sh.KS <= 8 ? 4 : 2);
    sh.RC_SUB = 4 * 16 * sh.MTR;
    if (sh.rc_bf16) {
      // one sub-tile per item, split coefficients staged rcbf_cols(KS32) columns at a time
      sh.PCAP = rcbf_cols(sh.KS32);
      sh.RPI = kRcBfSubs;
    } else {
      // coefficient staging: as many columns as the LDS budget holds (multiple of 16)
      const size_t per_col = 8 * (4 * (size_t)sh.KS + 1);   // padded LDS stride
      const int cap = (int)(kRcLdsBytes / per_col) / 16 * 16;
      const int need = (p.max_n + 15) / 16 * 16;
      sh.PCAP = std::max(16, std::min(cap, need));
      // sub-tiles per item: enough items to keep every CU busy (~8 per CU), at most 16
      int64_t subs = 0;
      for (int b = 0; b < nb; ++b) subs += (d->h_m[b] + sh.RC_SUB - 1) / sh.RC_SUB;
      sh.RPI = (int)std::max<int64_t>(1, std::min<int64_t>(16, subs / 2048));
      if (tune && tune->rc_rpi) sh.RPI = tune->rc_rpi;
    }
  }

  // sketch work items: column tiles x K splits.  BF16 with the default shape:
  // each block's tile is as narrow as its width allows (TN = 1, 2 or 4 tiles of
  // 16 columns per wave), so narrow blocks of an uneven batch do not run
  // mostly-empty tiles; otherwise every block uses sh.TN.
  const bool tn_by_block = p.ydt == 1 && d->prec == SPID_SK_BF16 && !(tune && tune->sk_tn) &&
                           sh.NW == 8;
  sh.tn_by_block = tn_by_block ? 1 : 0;
  auto tn_of = [&](int32_t nb_cols) {
    if (!tn_by_block) return sh.TN;
    int t = nb_cols <= 16 * sh.NW ? 1 : (nb_cols <= 32 * sh.NW ? 2 : 4);
    if (t == 4 && sh.MT >= 6) t = 2;
    return t;
  };
  const int tile_cols = 16 * sh.NW * sh.TN;
  // Cost-balanced K splits: an item's cost ~ rows x columns it streams.  A
  // block is split along K when its column tiles exceed the target item cost
  // (total / kTargetItems), keeping at least min_rows rows per split.
  double total_cost = 0.0;
  for (int b = 0; b < nb; ++b) total_cost += (double)d->h_m[b] * d->h_n[b];
  const int64_t kTargetItems = (tune && tune->sk_items) ? tune->sk_items : 2048;
  sh.sk_items = (int)kTargetItems;
  const int64_t min_rows = 256;
  const double target_cost = std::max(total_cost / kTargetItems, (double)min_rows * tile_cols);
  p.blk.resize(nb);
  int64_t y_off = 0, r_off = 0, p_off = 0, sk_off = 0, part_off = 0;
  for (int b = 0; b < nb; ++b) {
    const int64_t m = d->h_m[b];
    const int32_t n = d->h_n[b];
    const int tcols = 16 * sh.NW * tn_of(n);
    const double tile_cost = (double)m * std::min(n, tcols);
    int nsplit = (int)std::ceil(tile_cost / target_cost);
    nsplit = (int)std::max<int64_t>(1, std::min<int64_t>(nsplit, m / min_rows));
    if (p.coarse) nsplit = 1;
    // rows per split, multiple of the chunk
    int64_t rows = (m + nsplit - 1) / nsplit;
    rows = (rows + kKC - 1) / kKC * kKC;
    nsplit = (int)((m + rows - 1) / rows);
    BlkInfo bi{};
    bi.A = nullptr;
    bi.lda = m;
    bi.m = m;
    bi.n = n;
    bi.y_off = y_off;
    bi.r_off = r_off;
    bi.p_off = p_off;
    bi.sk_off = sk_off;
    bi.nsplit = nsplit;
    bi.part_off = nsplit > 1 ? part_off : 0;
    bi.vec_ok = 0;
    p.blk[b] = bi;
    y_off += (int64_t)d->l * n;
    r_off += (int64_t)d->k_max * n;
    p_off += (int64_t)d->k_max * n;
    sk_off += (int64_t)d->k_max * m;
    if (nsplit > 1) {
      part_off += (int64_t)nsplit * d->l * n;
      p.split_blocks.push_back(b);
      p.max_split_n = std::max(p.max_split_n, (int)n);
    }
    for (int c0 = 0; c0 < n && !p.coarse; c0 += tcols)
      for (int s = 0; s < nsplit; ++s) {
        SkItem it{};
        it.blk = b;
        it.c0 = c0;
        it.split = s;
        it.r0 = (int64_t)s * rows;
        it.r1 = std::min(m, (int64_t)(s + 1) * rows);
        p.items.push_back(it);
      }
    p.rc_first.push_back((int64_t)p.rc.size());
    const int64_t item_rows = (int64_t)sh.RC_SUB * sh.RPI;
    for (int64_t i0 = 0; i0 < m; i0 += item_rows) {
      RcItem r{};
      r.blk = b;
      r.i0 = i0;
      r.nsub = (int32_t)std::min<int64_t>(sh.RPI, (m - i0 + sh.RC_SUB - 1) / sh.RC_SUB);
      p.rc.push_back(r);
    }
  }
  p.rc_first.push_back((int64_t)p.rc.size());
  p.part_elems = part_off;
  {
    // error-pass items cut into 8 contiguous ranges of about equal cost (rows x
    // columns streamed), one per XCD
    std::vector<double> pre(p.rc.size() + 1, 0.0);
    for (size_t i = 0; i < p.rc.size(); ++i) {
      const RcItem& r = p.rc[i];
      const double rows = std::min<double>((double)r.nsub * sh.RC_SUB, (double)(d->h_m[r.blk] - r.i0));
      pre[i + 1] = pre[i] + rows * d->h_n[r.blk];
    }
    size_t cut = 0, longest = 0;
    p.rc_xcd.start[0] = 0;
    for (int x = 1; x <= 8; ++x) {
      const double goal = pre.back() * x / 8.0;
      while (cut < p.rc.size() && pre[cut] < goal) ++cut;
      if (x == 8) cut = p.rc.size();
      p.rc_xcd.start[x] = (int32_t)cut;
      longest = std::max<size_t>(longest, cut - (size_t)p.rc_xcd.start[x - 1]);
    }
    p.rc_xcd_grid = (unsigned)(8 * std::max<size_t>(1, longest));
  }

  if (p.coarse) {
    p.grid.resize(nb);
    int64_t cs_off = 0;
    for (int b = 0; b < nb; ++b) {
      const spid_grid& g = d->h_grid[b];
      GridInfo gi{};
      gi.nx = g.nx;
      gi.ny = g.ny;
      gi.nz = g.nz;
      gi.nf = g.nfields;
      gi.sx = g.sx;
      gi.sy = g.sy;
      gi.sz = g.sz;
      gi.cx = (g.nx + g.sx - 1) / g.sx;
      gi.cy = (g.ny + g.sy - 1) / g.sy;
      gi.cz = (g.nz + g.sz - 1) / g.sz;
      gi.mc = g.nfields * gi.cx * gi.cy * gi.cz;
      gi.cs_off = cs_off;
      cs_off += (int64_t)gi.mc * d->k_max;
      p.sum_mc += gi.mc;
      p.grid[b] = gi;
    }
  }

  // too few blocks to fill the chip with one workgroup each: split their rows
  if (p.coarse && sh.sel.sel_tall && nb < 128 && d->l > 4 * kSplitRows) {
    p.split = true;
    p.split_nch = (d->l + kSplitRows - 1) / kSplitRows;
    p.split_off.resize(nb);
    int64_t o = 0;
    for (int b = 0; b < nb; ++b) {
      p.split_off[b] = o;
      o += (int64_t)p.split_nch * d->h_n[b];
    }
    p.split_elems = o;
  }

  if (d->ts_windows > 0) {
    const int nw = d->ts_windows, k1 = d->ts_k1;
    p.ts_nwin = nw;
    p.ts_k1 = k1;
    p.ts_kmax1 = pick_kmax(k1);
    p.ts_win.resize((size_t)nb * nw);
    p.ts_blk2.resize(nb);
    int max_w = 0;
    int64_t r1 = 0, y2 = 0, r2 = 0;
    for (int b = 0; b < nb; ++b) {
      const int32_t n = d->h_n[b];
      for (int w = 0; w < nw; ++w) {
        const int c0 = (int)((int64_t)w * n / nw), c1 = (int)((int64_t)(w + 1) * n / nw);
        BlkInfo wi = p.blk[b];
        wi.y_off = p.blk[b].y_off + (int64_t)c0 * d->l;
        wi.n = c1 - c0;
        wi.r_off = r1;
        wi.p_off = r1;
        wi.nsplit = 1;
        r1 += (int64_t)k1 * wi.n;
        max_w = std::max(max_w, wi.n);
        p.ts_win[(size_t)b * nw + w] = wi;
      }
      BlkInfo b2 = p.blk[b];
      b2.n = nw * k1;
      b2.y_off = y2;
      b2.r_off = r2;
      b2.p_off = r2;
      b2.nsplit = 1;
      y2 += (int64_t)d->l * b2.n;
      r2 += (int64_t)d->k_max * b2.n;
      p.ts_blk2[b] = b2;
    }
    p.ts_n2sum = (int64_t)nb * nw * k1;
    if (!pick_sel(d->l, max_w, p.coarse, p.ts_sel1) ||
        !pick_sel(d->l, nw * k1, p.coarse, p.ts_sel2))
      return fail(SPID_EINVAL, "two-stage: l=%d exceeds the selection register/LDS budget",
                  d->l);
  }

  // one-snapshot (stream) plan: needs Omega shared by all blocks
  p.st_ok = d->omega_per_block == 0 && !p.coarse;
  if (p.st_ok) {
    p.perm.resize(nb);
    for (int b = 0; b < nb; ++b) p.perm[b] = b;
    std::stable_sort(p.perm.begin(), p.perm.end(),
                     [&](int32_t a, int32_t b2) { return d->h_m[a] > d->h_m[b2]; });
    double st_total = 0.0;
    for (int b = 0; b < nb; ++b) st_total += (double)d->h_m[b];
    const double st_target = std::max(st_total / kTargetItems, (double)min_rows * kStreamGroup);
    int64_t st_off = 0;
    for (int first = 0; first < nb;) {
      const int64_t m = d->h_m[p.perm[first]];
      int last = first;
      while (last < nb && last - first < kStreamGroup && d->h_m[p.perm[last]] == m) ++last;
      const int gsize = last - first;
      int nsplit = (int)std::ceil((double)m * gsize / st_target);
      nsplit = (int)std::max<int64_t>(1, std::min<int64_t>(nsplit, m / min_rows));
      int64_t rows = (m + nsplit - 1) / nsplit;
      rows = (rows + kKC - 1) / kKC * kKC;
      if (d->prec == SPID_SK_FP8E4M3) {
        // one work item streams a group over all of K (Omega from the update's table)
        nsplit = 1;
        rows = m;
      }
      nsplit = (int)((m + rows - 1) / rows);
      const int64_t gpart = nsplit > 1 ? st_off : 0;
      if (nsplit > 1) {
        p.sheads.push_back((int32_t)p.sitems.size());
        st_off += (int64_t)nsplit * kStreamGroup * d->l;
      }
      for (int sp = 0; sp < nsplit; ++sp) {
        SkItem it{};
        it.blk = p.perm[first];
        it.c0 = first;
        it.split = sp;
        it.gsize = gsize;
        it.r0 = (int64_t)sp * rows;
        it.r1 = std::min(m, (int64_t)(sp + 1) * rows);
        it.gnsplit = nsplit;
        it.gpart = gpart;
        p.sitems.push_back(it);
      }
      first = last;
    }
    p.st_part_elems = st_off;
    if (d->prec == SPID_SK_FP8E4M3) {
      // groups in runs of equal m; gw of them per work item (one by default: the
      // items need no shared set-up, so more of them only lengthen each)
      int64_t gw = 1;
      if (tune && tune->st_groups) gw = tune->st_groups;
      sh.st_groups = (int)gw;
      size_t i = 0;
      while (i < p.sitems.size()) {
        // run of consecutive groups with the same m and K split
        const SkItem& h = p.sitems[i];
        const int ns = h.gnsplit;
        size_t j = i;
        while (j < p.sitems.size() && p.sitems[j].gnsplit == ns &&
               d->h_m[p.sitems[j].blk] == d->h_m[h.blk])
          j += ns;
        const int64_t ngroups = (int64_t)(j - i) / ns;
        for (int sp = 0; sp < ns; ++sp)
          for (int64_t g0 = 0; g0 < ngroups; g0 += gw) {
            p.ritems.push_back((int32_t)(i + g0 * ns + sp));
            p.ritems.push_back((int32_t)std::min<int64_t>(gw, ngroups - g0));
            p.ritems.push_back(ns);
          }
        i = j;
      }
    }
  }
  // longest items first (the hardware dispatches workgroups in grid order)
  // grouped by TN (1, 2, 4), within a group longest items first (the hardware
  // dispatches workgroups in grid order)
  {
    auto tn_index = [&](const SkItem& it) {
      const int t = tn_of(d->h_n[it.blk]);
      return t == 1 ? 0 : (t == 2 ? 1 : 2);
    };
    auto cost = [&](const SkItem& it) {
      return (it.r1 - it.r0) *
             std::min<int64_t>(16 * sh.NW * tn_of(d->h_n[it.blk]), d->h_n[it.blk] - it.c0);
    };
    std::stable_sort(p.items.begin(), p.items.end(), [&](const SkItem& a, const SkItem& b2) {
      const int ta = tn_index(a), tb = tn_index(b2);
      if (ta != tb) return ta < tb;
      return cost(a) > cost(b2);
    });
    int64_t cnt[3] = {0, 0, 0};
    for (const SkItem& it : p.items) ++cnt[tn_index(it)];
    p.tn_start[0] = 0;
    for (int i = 0; i < 3; ++i) p.tn_start[i + 1] = p.tn_start[i] + cnt[i];
  }
  const size_t ysz = p.ydt == 0 ? 8 : 4;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  p.off_blk = take(sizeof(BlkInfo) * nb);
  p.off_items = take(sizeof(SkItem) * p.items.size());
  p.off_split = take(sizeof(int32_t) * std::max<size_t>(1, p.split_blocks.size()));
  p.off_rc = take(sizeof(RcItem) * p.rc.size());
  p.off_rcfirst = take(sizeof(int64_t) * p.rc_first.size());
  p.off_Y = take(ysz * (size_t)d->l * p.sum_n);
  p.off_part = take(ysz * (size_t)std::max<int64_t>({(int64_t)1, p.part_elems, p.st_part_elems}));
  p.off_R = take(sizeof(double) * (size_t)d->k_max * p.sum_n);
  p.off_S = take(sizeof(int32_t) * (size_t)nb * d->k_max);
  p.off_k = take(sizeof(int32_t) * nb);
  p.off_st = take(sizeof(int32_t) * nb);
  p.off_rcpart = take(sizeof(double) * 2 * p.rc.size());
  p.off_perm = take(sizeof(int32_t) * std::max<size_t>(1, p.perm.size()));
  p.off_sitems = take(sizeof(SkItem) * std::max<size_t>(1, p.sitems.size()));
  p.off_sheads = take(sizeof(int32_t) * std::max<size_t>(1, p.sheads.size()));
  p.off_ritems = take(sizeof(int32_t) * std::max<size_t>(1, p.ritems.size()));
  if (d->omega_per_block == 0 && !p.coarse &&
      (d->prec == SPID_SK_BF16 || d->prec == SPID_SK_F64 ||
       (d->prec == SPID_SK_FP8E4M3 && d->a_dtype == SPID_A_F32 && !p.ritems.empty()))) {
    int64_t max_m = 0;
    for (int b = 0; b < nb; ++b) max_m = std::max<int64_t>(max_m, d->h_m[b]);
    const int64_t ch = d->prec == SPID_SK_FP8E4M3 ? kKC8 : kKC;
    p.omtab_cols = (max_m + ch - 1) / ch * ch;
  }
  const size_t om_es = d->prec == SPID_SK_F64 ? 8 : (d->prec == SPID_SK_BF16 ? 2 : 1);
  p.off_omtab = take(om_es * (size_t)sh.MT * 16 * (size_t)std::max<int64_t>(1, p.omtab_cols));
  // mixed error pass: split-bfloat16 coefficients and compact column lists
  const size_t kp_bf = 32 * (size_t)sh.KS32;
  p.off_pt = take(sh.rc_bf16 ? sizeof(uint16_t) * 3 * kp_bf * (size_t)p.sum_n : 256);
  p.off_cols = take(sh.rc_bf16 ? sizeof(int32_t) * (size_t)p.sum_n : 256);
  p.off_ncols = take(sizeof(int32_t) * nb);
  p.off_grid = take(sizeof(GridInfo) * std::max<size_t>(1, p.grid.size()));
  p.off_W = take((sh.sel.sel_tall || p.ts_sel1.sel_tall) ? sizeof(double) * (size_t)d->l * p.sum_n
                                                         : 256);
  p.off_spoff = take(sizeof(int64_t) * std::max<size_t>(1, p.split_off.size()));
  p.off_spnorm = take(sizeof(double) * (size_t)std::max<int64_t>(1, p.split_elems));
  p.off_spdot = take(sizeof(double) * (size_t)std::max<int64_t>(1, p.split_elems));
  p.off_spused = take(p.split ? (size_t)nb * kTallMaxN : 256);
  p.off_spstate = take(sizeof(SplitState) * (p.split ? (size_t)nb : 1));
  p.off_spbad = take(sizeof(int32_t) * (p.split ? (size_t)nb : 1));
  {
    const bool ts = p.ts_nwin > 0;
    const size_t nwt = ts ? p.ts_win.size() : 1;
    const size_t k1 = ts ? p.ts_k1 : 1;
    p.off_tswin = take(sizeof(BlkInfo) * nwt);
    p.off_tsblk2 = take(sizeof(BlkInfo) * std::max<size_t>(1, p.ts_blk2.size()));
    p.off_tsR1 = take(ts ? sizeof(double) * k1 * (size_t)p.sum_n : 256);
    p.off_tsP1 = take(ts ? sizeof(double) * k1 * (size_t)p.sum_n : 256);
    p.off_tsS1 = take(sizeof(int32_t) * nwt * k1);
    p.off_tsk1 = take(sizeof(int32_t) * nwt);
    p.off_tsst1 = take(sizeof(int32_t) * nwt);
    p.off_tsY2 = take(ts ? ysz * (size_t)d->l * p.ts_n2sum : 256);
    p.off_tsW2 = take(ts && p.ts_sel2.sel_tall ? sizeof(double) * (size_t)d->l * p.ts_n2sum : 256);
    p.off_tsR2 = take(ts ? sizeof(double) * (size_t)d->k_max * p.ts_n2sum : 256);
    p.off_tsP2 = take(ts ? sizeof(double) * (size_t)d->k_max * p.ts_n2sum : 256);
    p.off_tsS2 = take(sizeof(int32_t) * (size_t)nb * d->k_max);
    p.off_tsk2 = take(sizeof(int32_t) * nb);
    p.off_tsst2 = take(sizeof(int32_t) * nb);
  }
  p.total = off;
  return SPID_OK;
}

}  // namespace
}  // namespace spid_host

using namespace spid_host;

namespace {

void sketch_batch_prec(spid_ctx* c, int j0, int j1, hipStream_t s) {
  if (c->plan.ydt == 0) sketch_batch_f64(c, j0, j1, s);
  else if (c->desc.prec == SPID_SK_FP8E4M3) sketch_batch_fp8(c, j0, j1, s);
  else sketch_batch_bf16(c, j0, j1, s);
}

bool sketch_stream_prec(spid_ctx* c, int j, hipStream_t s) {
  if (c->plan.ydt == 0) return sketch_stream_f64(c, j, s);
  if (c->desc.prec == SPID_SK_FP8E4M3) return sketch_stream_fp8(c, j, s);
  return sketch_stream_bf16(c, j, s);
}

}  // namespace

// ---- allocation-free contexts (spid_create_static)
// The workspace of callers that cannot allocate device memory: one array per
// device, allocated with the code object when the library is loaded on it and
// held until the process ends.  Host code never passes the array's name to a
// kernel or a copy (on the host it only stands in for the symbol): it takes the
// device address from hipGetSymbolAddress, once per device, and uses that.
namespace {
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
constexpr int kMaxStaticDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
std::mutex g_static_mu;
void* g_static_ptr[kMaxStaticDevices];                 // per device, under g_static_mu
std::atomic<uint64_t> g_static_gen[kMaxStaticDevices];  // last static context per device

// A context made by spid_create_static that a later one on the same device has
// replaced: its tables in the scratch array are gone.
spid_status check_live(const spid_ctx* c) {
  if (c->static_dev >= 0 && g_static_gen[c->static_dev].load() != c->static_gen)
    return fail(SPID_ESTATE,
                "context created by spid_create_static was replaced by a later "
                "spid_create_static on device %d (they share the static scratch array)",
                c->static_dev);
  return SPID_OK;
}
}  // namespace

// ============================================================================ C ABI

extern "C" size_t spid_workspace_bytes(const spid_desc* desc) {
  return spid_workspace_bytes_tuned(desc, nullptr);
}

extern "C" size_t spid_workspace_bytes_tuned(const spid_desc* desc, const spid_tuning* tuning) {
  Plan p;
  if (make_plan(desc, tuning, p) != SPID_OK) return 0;
  return p.total;
}

extern "C" spid_status spid_create(const spid_desc* desc, void* d_workspace, size_t ws_bytes,
                                   spid_ctx** out) {
  return spid_create_tuned(desc, nullptr, d_workspace, ws_bytes, out);
}

extern "C" spid_status spid_get_tuning(const spid_ctx* c, spid_tuning* out) {
  if (!c || !out) return fail(SPID_EINVAL, "NULL argument to spid_get_tuning");
  const Shape& sh = c->plan.sh;
  out->sk_tn = sh.tn_by_block ? 0 : sh.TN;
  out->sk_nw = sh.NW;
  out->sk_items = sh.sk_items;
  out->rc_rpi = sh.rc_bf16 ? 1 : sh.RPI;
  out->st_groups = sh.st_groups;
  return SPID_OK;
}

extern "C" spid_status spid_create_tuned(const spid_desc* desc, const spid_tuning* tuning,
                                         void* d_workspace, size_t ws_bytes, spid_ctx** out) {
  if (!out) return fail(SPID_EINVAL, "out is NULL");
  *out = nullptr;
  spid_ctx* c = new (std::nothrow) spid_ctx();
  if (!c) return fail(SPID_EINVAL, "host allocation failed");
  spid_status st = make_plan(desc, tuning, c->plan);
  if (st != SPID_OK) {
    delete c;
    return st;
  }
  const Plan& p = c->plan;
  if (!d_workspace || ((uintptr_t)d_workspace % kAlign) != 0) {
    delete c;
    return fail(SPID_EWORKSPACE, "workspace must be a 256-byte aligned device pointer");
  }
  if (ws_bytes < p.total) {
    delete c;
    return fail(SPID_EWORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, p.total);
  }
  c->desc = *desc;
  c->desc.h_grid = nullptr;   // the grids live in the plan
  c->m.assign(desc->h_m, desc->h_m + desc->nblocks);
  c->n.assign(desc->h_n, desc->h_n + desc->nblocks);
  c->desc.h_m = c->m.data();
  c->desc.h_n = c->n.data();
  c->ws = static_cast<char*>(d_workspace);
  c->covered.assign(p.max_n, 0);
  hipError_t e = hipMemcpy(c->ws + p.off_blk, p.blk.data(), sizeof(BlkInfo) * p.blk.size(),
                           hipMemcpyHostToDevice);
  if (e == hipSuccess && !p.items.empty())
    e = hipMemcpy(c->ws + p.off_items, p.items.data(), sizeof(SkItem) * p.items.size(),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess && !p.split_blocks.empty())
    e = hipMemcpy(c->ws + p.off_split, p.split_blocks.data(),
                  sizeof(int32_t) * p.split_blocks.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(c->ws + p.off_rc, p.rc.data(), sizeof(RcItem) * p.rc.size(),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(c->ws + p.off_rcfirst, p.rc_first.data(), sizeof(int64_t) * p.rc_first.size(),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess && !p.perm.empty())
    e = hipMemcpy(c->ws + p.off_perm, p.perm.data(), sizeof(int32_t) * p.perm.size(),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess && !p.sitems.empty())
    e = hipMemcpy(c->ws + p.off_sitems, p.sitems.data(), sizeof(SkItem) * p.sitems.size(),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess && !p.sheads.empty())
    e = hipMemcpy(c->ws + p.off_sheads, p.sheads.data(), sizeof(int32_t) * p.sheads.size(),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess && !p.ritems.empty())
    e = hipMemcpy(c->ws + p.off_ritems, p.ritems.data(), sizeof(int32_t) * p.ritems.size(),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess && p.coarse)
    e = hipMemcpy(c->ws + p.off_grid, p.grid.data(), sizeof(GridInfo) * p.grid.size(),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess && p.split)
    e = hipMemcpy(c->ws + p.off_spoff, p.split_off.data(), sizeof(int64_t) * p.split_off.size(),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess && p.ts_nwin > 0)
    e = hipMemcpy(c->ws + p.off_tswin, p.ts_win.data(), sizeof(BlkInfo) * p.ts_win.size(),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess && p.ts_nwin > 0)
    e = hipMemcpy(c->ws + p.off_tsblk2, p.ts_blk2.data(), sizeof(BlkInfo) * p.ts_blk2.size(),
                  hipMemcpyHostToDevice);

  if (e != hipSuccess) {
    delete c;
    return fail(SPID_EHIP, "spid_create: %s", hipGetErrorString(e));
  }
  *out = c;
  return SPID_OK;
}

extern "C" spid_status spid_create_static(const spid_desc* desc, const spid_tuning* tuning,
                                          spid_ctx** out) {
  if (!out) return fail(SPID_EINVAL, "out is NULL");
  *out = nullptr;
  Plan p;
  spid_status st = make_plan(desc, tuning, p);
  if (st != SPID_OK) return st;
  if (p.total > kStaticScratchBytes)
    return fail(SPID_EWORKSPACE,
                "spid_create_static: the descriptor needs %zu bytes of workspace, the static "
                "scratch array holds %zu (spid_create takes a caller workspace of any size)",
                p.total, kStaticScratchBytes);
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(SPID_EHIP, "spid_create_static: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxStaticDevices)
    return fail(SPID_EINVAL, "spid_create_static: device %d beyond %d", dev, kMaxStaticDevices);
  void* ptr = nullptr;
  uint64_t gen = 0;
  {
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_ptr[dev]) {
      e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr)
        return fail(SPID_EHIP, "spid_create_static: address of the scratch array: %s",
                    hipGetErrorString(e));
      g_static_ptr[dev] = ptr;
    }
    ptr = g_static_ptr[dev];
    // the previous static context on this device loses the array now; work it
    // enqueued must end before its tables are overwritten
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return fail(SPID_EHIP, "spid_create_static: %s", hipGetErrorString(e));
    gen = ++g_static_gen[dev];
  }
  st = spid_create_tuned(desc, tuning, ptr, kStaticScratchBytes, out);
  if (st != SPID_OK) return st;
  (*out)->static_dev = dev;
  (*out)->static_gen = gen;
  return SPID_OK;
}

extern "C" spid_status spid_bind_A(spid_ctx* c, const void* const* h_block_ptrs,
                                   const int64_t* h_lda) {
  if (!c || !h_block_ptrs || !h_lda) return fail(SPID_EINVAL, "NULL argument to spid_bind_A");
  if (check_live(c) != SPID_OK) return SPID_ESTATE;
  Plan& p = c->plan;
  const size_t es = c->desc.a_dtype == SPID_A_F64 ? 8 : 4;
  for (int b = 0; b < c->desc.nblocks; ++b) {
    if (!h_block_ptrs[b]) return fail(SPID_EINVAL, "block %d: NULL data pointer", b);
    if (h_lda[b] < c->m[b])
      return fail(SPID_EINVAL, "block %d: lda=%lld < m=%lld", b, (long long)h_lda[b],
                  (long long)c->m[b]);
    if (((uintptr_t)h_block_ptrs[b]) % es != 0)
      return fail(SPID_EINVAL, "block %d: pointer not aligned to the element size", b);
  }
  for (int b = 0; b < c->desc.nblocks; ++b) {
    BlkInfo& bi = p.blk[b];
    bi.A = h_block_ptrs[b];
    bi.lda = h_lda[b];
    bi.vec_ok = (((uintptr_t)bi.A % 16) == 0 && ((bi.lda * (int64_t)es) % 16) == 0) ? 1 : 0;
  }
  c->all_vec = true;
  for (const BlkInfo& bi : p.blk) c->all_vec = c->all_vec && bi.vec_ok;
  c->all_vec4 = c->all_vec;
  for (const BlkInfo& bi : p.blk) c->all_vec4 = c->all_vec4 && (bi.m % 4 == 0);
  hipError_t e = hipMemcpy(c->ws + p.off_blk, p.blk.data(), sizeof(BlkInfo) * p.blk.size(),
                           hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(SPID_EHIP, "spid_bind_A: %s", hipGetErrorString(e));
  c->bound = true;
  c->selected = false;
  c->coeffs_done = false;
  std::fill(c->covered.begin(), c->covered.end(), 0);
  return SPID_OK;
}

extern "C" spid_status spid_sketch_update(spid_ctx* c, int32_t j0, int32_t w, void* stream) {
  if (!c) return fail(SPID_EINVAL, "NULL context");
  if (check_live(c) != SPID_OK) return SPID_ESTATE;
  if (!c->bound) return fail(SPID_ESTATE, "spid_sketch_update before spid_bind_A");
  if (j0 < 0 || w < 1) return fail(SPID_EINVAL, "need j0 >= 0 and w >= 1 (got %d, %d)", j0, w);
  const Plan& p = c->plan;
  const int j1 = (int)std::min<int64_t>((int64_t)j0 + w, p.max_n);
  if (j0 >= p.max_n) return fail(SPID_EINVAL, "j0=%d is past every block's last column", j0);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (p.coarse) {
    const int64_t per_blk = (int64_t)c->desc.l * (j1 - j0);
    dim3 grid((unsigned)std::min<int64_t>((per_blk + 255) / 256, 1 << 20),
              (unsigned)std::min(c->desc.nblocks, 65535));
    if (c->desc.a_dtype == SPID_A_F64)
      hipLaunchKernelGGL((subsample_kernel<double>), grid, dim3(256), 0, s,
                         c->at<BlkInfo>(p.off_blk), c->at<GridInfo>(p.off_grid),
                         c->desc.nblocks, c->desc.l, j0, j1, c->at<double>(p.off_Y));
    else
      hipLaunchKernelGGL((subsample_kernel<float>), grid, dim3(256), 0, s,
                         c->at<BlkInfo>(p.off_blk), c->at<GridInfo>(p.off_grid),
                         c->desc.nblocks, c->desc.l, j0, j1, c->at<double>(p.off_Y));
    spid_status st = hip_check("subsample kernel launch");
    if (st != SPID_OK) return st;
    for (int j = j0; j < j1; ++j) c->covered[j] = 1;
    c->selected = false;
    c->coeffs_done = false;
    return SPID_OK;
  }
  // shared Omega: regenerated from the generator for this update into the
  // small table the sketch kernels read (l x max m_b, L2-resident): the
  // double-precision and bfloat16 kernels, and the FP8 one-snapshot kernel
  const bool one_snapshot = p.st_ok && j1 - j0 <= kStreamMaxW;
  if (p.omtab_cols > 0 && (c->desc.prec != SPID_SK_FP8E4M3 || one_snapshot)) {
    if (!launch_omega_table(c, s)) return fail(SPID_EHIP, "Omega table launch failed");
  }
  if (one_snapshot) {
    // a few snapshots: one launch per snapshot with the blocks as MFMA columns
    for (int j = j0; j < j1; ++j) {
      const bool ok = sketch_stream_prec(c, j, s);
      if (!ok) return fail(SPID_EHIP, "stream sketch: cannot reserve the Omega LDS");
      spid_status st = hip_check("stream sketch kernel launch");
      if (st != SPID_OK) return st;
      if (!p.sheads.empty()) {
        dim3 grid((unsigned)(((int64_t)c->desc.l * kStreamGroup + 255) / 256),
                  (unsigned)p.sheads.size());
        if (p.ydt == 0)
          hipLaunchKernelGGL((sketch_stream_reduce_kernel<double>), grid, dim3(256), 0, s,
                             c->at<BlkInfo>(p.off_blk), c->at<int32_t>(p.off_perm),
                             c->at<SkItem>(p.off_sitems), c->at<int32_t>(p.off_sheads),
                             c->desc.l, kStreamGroup, j, c->at<double>(p.off_Y),
                             c->at<double>(p.off_part));
        else
          hipLaunchKernelGGL((sketch_stream_reduce_kernel<float>), grid, dim3(256), 0, s,
                             c->at<BlkInfo>(p.off_blk), c->at<int32_t>(p.off_perm),
                             c->at<SkItem>(p.off_sitems), c->at<int32_t>(p.off_sheads),
                             c->desc.l, kStreamGroup, j, c->at<float>(p.off_Y),
                             c->at<float>(p.off_part));
        st = hip_check("stream sketch reduce launch");
        if (st != SPID_OK) return st;
      }
    }
    for (int j = j0; j < j1; ++j) c->covered[j] = 1;
    c->selected = false;
    c->coeffs_done = false;
    return SPID_OK;
  }
  sketch_batch_prec(c, j0, j1, s);
  spid_status st = hip_check("sketch kernel launch");
  if (st != SPID_OK) return st;
  if (!p.split_blocks.empty()) {
    dim3 grid((unsigned)(((int64_t)c->desc.l * p.max_split_n + 255) / 256),
              (unsigned)p.split_blocks.size());
    if (p.ydt == 0)
      hipLaunchKernelGGL((sketch_reduce_kernel<double>), grid, dim3(256), 0, s,
                         c->at<BlkInfo>(p.off_blk), c->at<int32_t>(p.off_split), c->desc.l, j0,
                         j1, c->at<double>(p.off_Y), c->at<double>(p.off_part));
    else
      hipLaunchKernelGGL((sketch_reduce_kernel<float>), grid, dim3(256), 0, s,
                         c->at<BlkInfo>(p.off_blk), c->at<int32_t>(p.off_split), c->desc.l, j0,
                         j1, c->at<float>(p.off_Y), c->at<float>(p.off_part));
    st = hip_check("sketch reduce launch");
    if (st != SPID_OK) return st;
  }
  for (int j = j0; j < j1; ++j) c->covered[j] = 1;
  c->selected = false;
  c->coeffs_done = false;
  return SPID_OK;
}

extern "C" spid_status spid_select(spid_ctx* c, int32_t* d_k, int32_t* d_S, int32_t* d_status,
                                   void* stream) {
  if (!c) return fail(SPID_EINVAL, "NULL context");
  if (check_live(c) != SPID_OK) return SPID_ESTATE;
  for (int j = 0; j < c->plan.max_n; ++j)
    if (!c->covered[j])
      return fail(SPID_ESTATE, "spid_select: sketch column %d has not been computed", j);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool ok = launch_select_ctx(c, s);
  if (!ok) return fail(SPID_EHIP, "select: cannot reserve the selection LDS");
  spid_status st = hip_check("select kernel launch");
  if (st != SPID_OK) return st;
  if (d_k || d_S || d_status) {
    const int64_t tot = std::max<int64_t>((int64_t)c->desc.nblocks * c->desc.k_max,
                                          c->desc.nblocks);
    hipLaunchKernelGGL(select_export_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                       c->desc.nblocks, c->desc.k_max, c->at<int32_t>(c->plan.off_S),
                       c->at<int32_t>(c->plan.off_k), c->at<int32_t>(c->plan.off_st), d_k, d_S,
                       d_status);
    st = hip_check("select export launch");
    if (st != SPID_OK) return st;
  }
  c->selected = true;
  c->coeffs_done = false;
  c->two_stage = false;
  return SPID_OK;
}

extern "C" spid_status spid_coeffs(spid_ctx* c, double* d_P, void* stream) {
  if (!c || !d_P) return fail(SPID_EINVAL, "NULL argument to spid_coeffs");
  if (check_live(c) != SPID_OK) return SPID_ESTATE;
  if (!c->selected) return fail(SPID_ESTATE, "spid_coeffs before spid_select");
  if (c->two_stage)
    return fail(SPID_ESTATE,
                "spid_coeffs after spid_select_two_stage (which writes the coefficients)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool ok = launch_coeffs_ctx(c, d_P, s);
  if (!ok) return fail(SPID_EHIP, "coeffs: cannot reserve the R11 LDS");
  c->coeffs_done = true;
  return hip_check("coeffs kernel launch");
}

extern "C" spid_status spid_reconstruct(spid_ctx* c, const double* d_P, double* d_err2,
                                        double* d_nrm2, void* d_skeleton, void* stream) {
  if (!c || !d_P || !d_err2 || !d_nrm2) return fail(SPID_EINVAL, "NULL argument to spid_reconstruct");
  if (check_live(c) != SPID_OK) return SPID_ESTATE;
  if (!c->selected) return fail(SPID_ESTATE, "spid_reconstruct before spid_select");
  if (!c->coeffs_done) return fail(SPID_ESTATE, "spid_reconstruct before spid_coeffs");
  const Plan& p = c->plan;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool ok = launch_recon_ctx(c, d_P, d_skeleton, s);
  if (!ok) return fail(SPID_EHIP, "reconstruct: cannot reserve the coefficient LDS");
  spid_status st = hip_check("reconstruct kernel launch");
  if (st != SPID_OK) return st;
  hipLaunchKernelGGL(recon_reduce_kernel, dim3(c->desc.nblocks), dim3(kWave), 0, s,
                     c->desc.nblocks, c->at<int64_t>(p.off_rcfirst), c->at<double>(p.off_rcpart),
                     d_err2, d_nrm2);
  return hip_check("reconstruct reduce launch");
}

namespace {

template <typename TY>
spid_status two_stage_t(spid_ctx* c, double* d_P, hipStream_t s) {
  const Plan& p = c->plan;
  const spid_desc& d = c->desc;
  const int nb = d.nblocks, nw = p.ts_nwin, k1 = p.ts_k1;
  const BlkInfo* win = c->at<BlkInfo>(p.off_tswin);
  const BlkInfo* blk2 = c->at<BlkInfo>(p.off_tsblk2);
  // stage 1: rank-k1 ID of every window
  SelJob<TY> j1{win, nb * nw, d.l, k1, 0.0, d.rank_floor, c->at<TY>(p.off_Y),
                c->at<double>(p.off_W), c->at<double>(p.off_tsR1), c->at<int32_t>(p.off_tsS1),
                c->at<int32_t>(p.off_tsk1), c->at<int32_t>(p.off_tsst1), p.ts_sel1};
  if (!launch_select_job<TY>(j1, s)) return fail(SPID_EHIP, "two-stage: stage-1 selection");
  spid_status st = hip_check("two-stage stage-1 selection launch");
  if (st != SPID_OK) return st;
  if (!launch_coeffs_any(p.ts_kmax1, win, nb * nw, d.l, k1, c->at<double>(p.off_tsR1),
                         c->at<int32_t>(p.off_tsS1), c->at<int32_t>(p.off_tsk1),
                         c->at<double>(p.off_tsP1), s))
    return fail(SPID_EHIP, "two-stage: stage-1 coefficients");
  st = hip_check("two-stage stage-1 coefficients launch");
  if (st != SPID_OK) return st;
  // stage 2: the sketch of the concatenated skeletons, gathered from the resident sketch
  const int64_t per_blk = (int64_t)nw * k1 * d.l;
  dim3 grid((unsigned)std::min<int64_t>((per_blk + 255) / 256, 1 << 20),
            (unsigned)std::min(nb, 65535));
  hipLaunchKernelGGL((ts_gather_kernel<TY>), grid, dim3(256), 0, s, win, blk2, nb, nw, k1, d.l,
                     c->at<int32_t>(p.off_tsS1), c->at<int32_t>(p.off_tsk1), c->at<TY>(p.off_Y),
                     c->at<TY>(p.off_tsY2));
  st = hip_check("two-stage gather launch");
  if (st != SPID_OK) return st;
  SelJob<TY> j2{blk2, nb, d.l, d.k_max, d.tol, d.rank_floor, c->at<TY>(p.off_tsY2),
                c->at<double>(p.off_tsW2), c->at<double>(p.off_tsR2), c->at<int32_t>(p.off_tsS2),
                c->at<int32_t>(p.off_tsk2), c->at<int32_t>(p.off_tsst2), p.ts_sel2};
  if (!launch_select_job<TY>(j2, s)) return fail(SPID_EHIP, "two-stage: stage-2 selection");
  st = hip_check("two-stage stage-2 selection launch");
  if (st != SPID_OK) return st;
  if (!launch_coeffs_any(p.sh.KMAX, blk2, nb, d.l, d.k_max, c->at<double>(p.off_tsR2),
                         c->at<int32_t>(p.off_tsS2), c->at<int32_t>(p.off_tsk2),
                         c->at<double>(p.off_tsP2), s))
    return fail(SPID_EHIP, "two-stage: stage-2 coefficients");
  st = hip_check("two-stage stage-2 coefficients launch");
  if (st != SPID_OK) return st;
  hipLaunchKernelGGL(ts_combine_kernel, dim3(nb), dim3(256), 0, s, c->at<BlkInfo>(p.off_blk), win,
                     blk2, nw, k1, d.k_max, c->at<int32_t>(p.off_tsS1),
                     c->at<int32_t>(p.off_tsk1), c->at<int32_t>(p.off_tsst1),
                     c->at<double>(p.off_tsP1), c->at<int32_t>(p.off_tsS2),
                     c->at<int32_t>(p.off_tsk2), c->at<int32_t>(p.off_tsst2),
                     c->at<double>(p.off_tsP2), d_P, c->at<int32_t>(p.off_S),
                     c->at<int32_t>(p.off_k), c->at<int32_t>(p.off_st));
  return hip_check("two-stage combine launch");
}

}  // namespace

extern "C" spid_status spid_select_two_stage(spid_ctx* c, int32_t* d_k, int32_t* d_S,
                                             int32_t* d_status, double* d_P, void* stream) {
  if (!c || !d_P) return fail(SPID_EINVAL, "NULL argument to spid_select_two_stage");
  if (check_live(c) != SPID_OK) return SPID_ESTATE;
  if (c->plan.ts_nwin < 1)
    return fail(SPID_EINVAL, "spid_select_two_stage: the descriptor has no ts_windows");
  for (int j = 0; j < c->plan.max_n; ++j)
    if (!c->covered[j])
      return fail(SPID_ESTATE, "spid_select_two_stage: sketch column %d has not been computed", j);
  hipStream_t s = static_cast<hipStream_t>(stream);
  spid_status st = c->plan.ydt == 0 ? two_stage_t<double>(c, d_P, s) : two_stage_t<float>(c, d_P, s);
  if (st != SPID_OK) return st;
  if (d_k || d_S || d_status) {
    const int64_t tot = std::max<int64_t>((int64_t)c->desc.nblocks * c->desc.k_max,
                                          c->desc.nblocks);
    hipLaunchKernelGGL(select_export_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                       c->desc.nblocks, c->desc.k_max, c->at<int32_t>(c->plan.off_S),
                       c->at<int32_t>(c->plan.off_k), c->at<int32_t>(c->plan.off_st), d_k, d_S,
                       d_status);
    st = hip_check("select export launch");
    if (st != SPID_OK) return st;
  }
  // the final selection and coefficients are in place: the error pass may follow
  c->selected = true;
  c->coeffs_done = true;
  c->two_stage = true;
  return SPID_OK;
}

extern "C" spid_status spid_reconstruct_interp(spid_ctx* c, const double* d_P, double* d_err2,
                                               double* d_nrm2, void* d_coarse_skeleton,
                                               void* stream) {
  if (!c || !d_P || !d_err2 || !d_nrm2)
    return fail(SPID_EINVAL, "NULL argument to spid_reconstruct_interp");
  if (check_live(c) != SPID_OK) return SPID_ESTATE;
  if (!c->plan.coarse)
    return fail(SPID_EINVAL, "spid_reconstruct_interp needs the coarse-grid sketch");
  if (!c->selected) return fail(SPID_ESTATE, "spid_reconstruct_interp before spid_select");
  if (!c->coeffs_done) return fail(SPID_ESTATE, "spid_reconstruct_interp before spid_coeffs");
  const Plan& p = c->plan;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool ok = launch_interp_ctx(c, d_P, d_coarse_skeleton, s);
  if (!ok) return fail(SPID_EHIP, "reconstruct_interp: cannot reserve the coefficient LDS");
  spid_status st = hip_check("interpolated error kernel launch");
  if (st != SPID_OK) return st;
  hipLaunchKernelGGL(recon_reduce_kernel, dim3(c->desc.nblocks), dim3(kWave), 0, s,
                     c->desc.nblocks, c->at<int64_t>(p.off_rcfirst), c->at<double>(p.off_rcpart),
                     d_err2, d_nrm2);
  return hip_check("interpolated error reduce launch");
}

extern "C" spid_status spid_copy_sketch(spid_ctx* c, double* d_Y, void* stream) {
  if (!c || !d_Y) return fail(SPID_EINVAL, "NULL argument to spid_copy_sketch");
  if (check_live(c) != SPID_OK) return SPID_ESTATE;
  const Plan& p = c->plan;
  const int64_t total = (int64_t)c->desc.l * p.sum_n;
  hipStream_t s = static_cast<hipStream_t>(stream);
  dim3 grid((unsigned)((total + 255) / 256));
  if (p.ydt == 0)
    hipLaunchKernelGGL((copy_sketch_kernel<double>), grid, dim3(256), 0, s, total,
                       c->at<double>(p.off_Y), d_Y);
  else
    hipLaunchKernelGGL((copy_sketch_kernel<float>), grid, dim3(256), 0, s, total,
                       c->at<float>(p.off_Y), d_Y);
  return hip_check("copy sketch launch");
}

extern "C" spid_status spid_destroy(spid_ctx* c) {
  delete c;
  return SPID_OK;
}

extern "C" const char* spid_last_error(void) { return g_err.c_str(); }
