// spid_internal.h -- host-side internals shared by the translation units of
// libspid.so: limits, the launch-shape and workspace plan, the context, and the
// per-stage launchers (each stage's kernels are instantiated in its own source
// file so that the library builds in parallel).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/spid.h"
#include "spid_kernels.h"
#include "spid_subsample.h"
#include "spid_two_stage.h"

namespace spid_host {

using namespace spid;

// Records the message for spid_last_error() and returns st.
spid_status fail(spid_status st, const char* fmt, ...);

constexpr int kMaxL = 128;
constexpr int kMaxLCoarse = 1 << 22;               // coarse-grid sketch rows
constexpr int kMaxK = 96;
constexpr int kMaxN = 1024;
static_assert(kRcMaxCols >= kMaxN, "the mixed error pass stages a whole column list");
constexpr int kStreamNW = 8;                       // waves of a one-snapshot sketch workgroup
constexpr int kStreamGroup = 16 * kStreamNW;       // blocks per group (one 16-column tile per wave)
constexpr int kStreamMaxW = 4;                     // updates of up to this many snapshots use it

constexpr size_t kAlign = 256;

inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Selection kernel choice for a sketch height l and widest block max_n.
//   register kernel (sel_lpc > 0): groups of sel_lpc lanes hold 4 columns,
//     each lane sel_rpt rows (l <= 128, n <= 512; n <= 384 for l > 64);
//   hybrid (sel_rr > 0): one column per thread, sel_rr rows in registers, the
//     rest in LDS (wider blocks);
//   tall (sel_tall): coarse sketches taller than 128 rows, in global memory.
struct SelShape {
  int LMAX = 16, sel_thr = 64, sel_rr = 0, sel_lpc = 0, sel_rpt = 0, sel_tall = 0;
  size_t sel_lds = 0;
};

// tile/template choices for a descriptor
struct Shape {
  int MT;        // 16-row MFMA tiles covering l
  int TN;        // 16-column tiles per wave in the sketch
  int NW;        // waves per sketch workgroup (columns per workgroup = 16 * NW * TN)
  SelShape sel;  // selection kernel
  int KMAX;      // register skeleton width in the error pass
  int KS;        // k-steps of 4 selected columns in the matrix-core error pass
  int MTR;       // 16-row MFMA tiles per wave in the error pass
  int RC_SUB;    // rows of an error-pass sub-tile (4 waves x 16 * MTR)
  int RPI;       // sub-tiles per error-pass work item
  int PCAP;      // non-skeleton columns whose coefficients are staged in LDS at once
  int rc_bf16;   // 1: split-bfloat16 error pass (FP32 data, low-precision sketch)
  int KS32;      // k-steps of 32 selected columns in the split-bfloat16 error pass
  int sk_items;  // target number of sketch work items
  int st_groups = 0;  // one-snapshot FP8 updates: block groups per work item
  int tn_by_block = 0;  // 1: BF16 batch sketch tiles sized per block (TN 1, 2, 4)
};

inline int pick_mt(int l) {
  const int t = (l + 15) / 16;
  if (t <= 4) return t;
  if (t <= 6) return 6;
  return 8;
}

inline int pick_lmax(int l) {
  const int opts[] = {16, 32, 48, 56, 64, 96, 128};
  for (int o : opts)
    if (l <= o) return o;
  return 128;
}

inline int pick_kmax(int k) {
  const int opts[] = {8, 16, 32, 48, 64, 96};
  for (int o : opts)
    if (k <= o) return o;
  return 96;
}

// false: no register/LDS kernel fits and the global-memory kernel is not allowed
inline bool pick_sel(int l, int max_n, bool allow_tall, SelShape& sh) {
  sh = SelShape{};
  sh.LMAX = pick_lmax(l);
  sh.sel_tall = (allow_tall && l > kMaxL) ? 1 : 0;
  if (sh.sel_tall) return true;   // coarse sketch taller than the register/LDS kernels take
  {
    const int lpc = l <= 32 ? 2 : (l <= 64 ? 4 : 8);
    if (l <= kMaxL && max_n <= (lpc == 8 ? 384 : 512)) {
      sh.sel_lpc = lpc;
      sh.sel_rpt = std::max(4, ((l + lpc - 1) / lpc + 3) / 4 * 4);
      const int groups = (max_n + 3) / 4;
      sh.sel_thr = std::max(64, (groups * lpc + 63) / 64 * 64);
      return true;
    }
  }
  // hybrid: one column per thread, RR rows in registers, the rest in LDS
  sh.sel_thr = std::max(64, (max_n + 63) / 64 * 64);
  const int rr_opts[] = {48, 32, 16};
  for (int rr : rr_opts) {
    if (sh.sel_thr > 512 && rr > 32) continue;   // 1024 threads: 128 registers per lane
    const size_t lds = sizeof(double) * (size_t)std::max(0, l - rr) * sh.sel_thr;
    if (lds <= 150 * 1024) {
      sh.sel_rr = rr;
      sh.sel_lds = lds;
      return true;
    }
  }
  if (!allow_tall) return false;
  sh.sel_tall = 1;
  return true;
}

// Workspace plan (sizes in bytes, offsets from the workspace base)
struct Plan {
  Shape sh;
  int ydt;                       // 0: Y in FP64, 1: Y in FP32
  std::vector<BlkInfo> blk;
  std::vector<SkItem> items;
  // batch sketch items grouped by column tiles per wave: items
  // [tn_start[i], tn_start[i+1]) run with TN = 1, 2, 4 (i = 0, 1, 2); one launch
  // per non-empty group.  BF16 sketches by default size TN to each block's
  // width; otherwise every item is in the group of sh.TN.
  int64_t tn_start[4] = {0, 0, 0, 0};
  std::vector<int32_t> split_blocks;
  std::vector<RcItem> rc;
  std::vector<int64_t> rc_first;
  XcdSplit rc_xcd{};          // error-pass items per XCD (ranges of about equal cost)
  unsigned rc_xcd_grid = 0;   // 8 * the longest range
  // one-snapshot updates: blocks ordered by m (perm), groups of kStreamGroup
  // equal-m blocks x K ranges (sitems), heads of groups with several K ranges
  bool st_ok = false;
  std::vector<int32_t> perm;
  std::vector<SkItem> sitems;
  std::vector<int32_t> sheads;
  std::vector<int32_t> ritems;   // FP8 one-snapshot items: (first stream item, count, stride)
  int64_t st_part_elems = 0;
  // coarse-grid sketch: block grids (the single-pass error uses the error-pass items)
  bool coarse = false;
  std::vector<GridInfo> grid;
  int64_t sum_mc = 0;
  // a few very tall coarse sketches: selection with the rows split over workgroups
  bool split = false;
  int split_nch = 0;
  std::vector<int64_t> split_off;   // per block: offset of its chunk partials (nch * n_b)
  int64_t split_elems = 0;
  // modified two-stage ID: window table (nblocks * nwin), stage-2 table (nblocks)
  int ts_nwin = 0, ts_k1 = 0, ts_kmax1 = 8;
  SelShape ts_sel1, ts_sel2;
  std::vector<BlkInfo> ts_win, ts_blk2;
  int64_t ts_n2sum = 0;
  int64_t sum_n = 0, sum_m = 0, part_elems = 0;
  int max_n = 0, max_split_n = 0;
  // Omega shared by all blocks, regenerated at the start of every sketch update
  // into a table of MT*16 rows x omtab_cols columns (max m rounded up to the
  // chunk; 0: no table): double chunk rows for the double-precision kernel,
  // bfloat16 in MFMA operand order for the bfloat16 kernels, e4m3 in f8f6f4
  // operand order for the FP8 one-snapshot kernel
  int64_t omtab_cols = 0;
  size_t off_omtab = 0;
  size_t off_blk, off_items, off_split, off_rc, off_rcfirst, off_Y, off_part, off_R, off_S, off_k,
      off_st, off_rcpart, off_perm, off_sitems, off_sheads, off_ritems, off_pt, off_cols, off_ncols,
      off_grid, off_W, off_spoff, off_spnorm, off_spdot, off_spused, off_spstate, off_spbad,
      off_tswin, off_tsblk2, off_tsR1, off_tsP1, off_tsS1, off_tsk1, off_tsst1,
      off_tsY2, off_tsW2, off_tsR2, off_tsP2, off_tsS2, off_tsk2, off_tsst2, total;
};

}  // namespace spid_host

struct spid_ctx {
  spid_desc desc;
  std::vector<int64_t> m;
  std::vector<int32_t> n;
  spid_host::Plan plan;
  char* ws = nullptr;
  bool bound = false;
  bool selected = false;
  bool coeffs_done = false;        // spid_coeffs ran after the last selection
  bool two_stage = false;          // the last selection was spid_select_two_stage
  bool all_vec = false;            // every block's column starts are 16-byte aligned
  bool all_vec4 = false;           // ... and every m is a multiple of 4
  std::vector<uint8_t> covered;   // per column index: sketched since bind
  int static_dev = -1;             // spid_create_static: device whose scratch array it uses
  uint64_t static_gen = 0;         // ... and the generation of that array it owns
  template <typename T>
  T* at(size_t off) const {
    return reinterpret_cast<T*>(ws + off);
  }
};


namespace spid_host {

// Status of the last HIP launch (EHIP with the runtime's message).
spid_status hip_check(const char* what);

// Kernels whose dynamic LDS exceeds 64 KiB must opt in before every launch
// (cheap host call, no stream work, safe under graph capture).
bool allow_lds(const void* kernel, size_t bytes);

template <typename TY>
struct SelJob {
  const BlkInfo* blks;
  int nblocks, l, k_max;
  double tol, rank_floor;
  const TY* Y;
  double* W;           // working copy of the global-memory kernel (same offsets as Y)
  double* R;
  int32_t *S, *k, *st;
  SelShape sh;
};

// ---- per-stage launchers (defined in the stage sources)
// sketch of columns [j0, j1) of every block, one launch over the batch items
void sketch_batch_f64(spid_ctx* c, int j0, int j1, hipStream_t s);    // spid_sketch_f64.hip
void sketch_batch_bf16(spid_ctx* c, int j0, int j1, hipStream_t s);   // spid_sketch_bf16.hip
void sketch_batch_bf16_tab(spid_ctx* c, int j0, int j1, hipStream_t s); // spid_sketch_bf16_tab.hip
// the Omega table of the update (spid_sketch_bf16_tab.hip); false if the launch failed
bool launch_omega_table(spid_ctx* c, hipStream_t s);
void sketch_batch_fp8(spid_ctx* c, int j0, int j1, hipStream_t s);    // spid_sketch_fp8.hip
// one-snapshot sketch of column j (blocks as the MFMA columns); false if the
// LDS opt-in failed
bool sketch_stream_f64(spid_ctx* c, int j, hipStream_t s);
bool sketch_stream_bf16(spid_ctx* c, int j, hipStream_t s);
bool sketch_stream_fp8(spid_ctx* c, int j, hipStream_t s);
// selection (spid_select.hip)
bool launch_select_job_f64(const SelJob<double>& j, hipStream_t s);
bool launch_select_job_f32(const SelJob<float>& j, hipStream_t s);
bool launch_select_ctx(spid_ctx* c, hipStream_t s);
// coefficients, error passes (spid_recon.hip)
bool launch_coeffs_any(int kmax_t, const BlkInfo* blks, int nblocks, int l, int k_max,
                       const double* R, const int32_t* S, const int32_t* k, double* P,
                       hipStream_t s);
bool launch_coeffs_ctx(spid_ctx* c, double* P, hipStream_t s);
bool launch_recon_ctx(spid_ctx* c, const double* P, void* skel, hipStream_t s);
bool launch_interp_ctx(spid_ctx* c, const double* P, void* cskel, hipStream_t s);

template <typename TY>
inline bool launch_select_job(const SelJob<TY>& j, hipStream_t s) {
  if constexpr (std::is_same<TY, double>::value) return launch_select_job_f64(j, s);
  else return launch_select_job_f32(j, s);
}

}  // namespace spid_host
