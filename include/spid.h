/*
 * spid.h -- C ABI of the MI355X (gfx950) sketched column interpolative
 * decomposition of per-subdomain snapshot matrices.
 *
 * Method (arXiv 2103.01380, "Task-parallel in-situ temporal compression of
 * large-scale CFD data"):
 *   A_b (m_b spatial values x n_b snapshots, Section 2) is compressed per
 *   spatial block independently (Section 3.2) into k_b selected time columns
 *   S_b and a coefficient matrix P_b with A_b ~ A_b(:,S_b) P_b:
 *     1. sketch      Y_b = Omega A_b, Omega l x m_b i.i.d. standard normal
 *                    (Section 2, random projection; indices and coefficients
 *                    of the sketch transfer to A);
 *     2. select      rank-k column-pivoted QR of Y_b by modified Gram-Schmidt
 *                    (Section 2, Algorithm 1 "mgsqr"), or stopped at a
 *                    tolerance (Remark 2.1);
 *     3. coeffs      P_b = [I_k | R11^+ R12] Z^T (Section 2, Algorithm 1);
 *     4. reconstruct ||A_b - A_b(:,S_b) P_b||_F^2 and ||A_b||_F^2, the parts of
 *                    the relative Frobenius error of Section 5.1.
 *   With the coarse-grid sketch (SPID_SK_SUBSAMPLE) step 1 is the row
 *   subsample B = A(J,:) (Algorithm 2, SubID) and step 4 also has the
 *   single-pass form M B(:,S) P (Algorithm 3, spid_reconstruct_interp).
 *
 * Conventions for every entry point:
 *   - Pointers marked d_ are device (HBM) pointers, h_ are host pointers.  The
 *     caller owns every buffer.  The library never allocates device memory:
 *     all of its state lives in the caller's workspace.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     The compute calls only enqueue kernels (no host synchronisation, no
 *     allocation), so the sequence sketch -> select -> coeffs -> reconstruct
 *     can be captured into a HIP graph.
 *   - Host-side validation is synchronous: on error nothing is enqueued, a
 *     negative spid_status is returned and spid_last_error() describes it.
 *     Numerical conditions of a block never fail the batch; they are
 *     reported per block in d_status (SPID_BLOCK_*).
 *   - Matrices are column-major.  Block b of A is m_b x n_b with leading
 *     dimension lda_b >= m_b, in the context's A dtype.
 */
#ifndef SPID_H
#define SPID_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct spid_ctx spid_ctx;

typedef enum {
  SPID_OK = 0,
  SPID_EINVAL = -1,     /* invalid argument or descriptor */
  SPID_EWORKSPACE = -2, /* workspace too small or misaligned (256 B) */
  SPID_EHIP = -3,       /* a HIP call or kernel launch failed */
  SPID_ESTATE = -4      /* call out of order (e.g. select before the sketch
                           covers every column, coeffs before select) */
} spid_status;

/* per-block numerical status written by spid_select */
enum {
  SPID_BLOCK_OK = 0,
  SPID_BLOCK_RANK_DEFICIENT = 1, /* a zero pivot (or one under rank_floor):
                                    fewer than k_max columns were taken */
  SPID_BLOCK_NONFINITE = 2,      /* NaN/Inf in the sketch: k_b = 0 */
  SPID_BLOCK_TOL_NOT_MET = 3     /* tolerance mode reached k_max first */
};

typedef enum { SPID_A_F64 = 0, SPID_A_F32 = 1 } spid_adtype;

/* Arithmetic of the sketch product.  F64: double-precision Omega and A on the
 * FP64 matrix cores.  BF16 / FP8E4M3: Omega is the double-precision normal
 * rounded to nearest-even bfloat16 / OCP e4m3, A is split into lp_terms
 * low-precision terms (hi + lo [+ lo2]) with FP32 accumulation; for FP8 every
 * 32 consecutive rows of a column carry their own power-of-two scale (the
 * per-block scaling).  Selection and coefficients are always FP64. */
typedef enum {
  SPID_SK_F64 = 0,
  SPID_SK_BF16 = 1,
  SPID_SK_FP8E4M3 = 2,
  /* Deterministic coarse-grid sketch (Section 2; Algorithm 2, SubID): the
   * sketch is the row subsample Y_b = A_b(J_b, :), J_b every s-th point per
   * direction of block b's grid (h_grid[b]), copied exactly (widened to
   * FP64).  Rows m_c,b .. l-1 of Y_b are zero.  No Omega: seed,
   * omega_per_block and lp_terms are ignored. */
  SPID_SK_SUBSAMPLE = 3
} spid_skprec;

/* Structured grid of one block for the coarse-grid sketch (Section 2,
 * coarse-grid representation; Section 5.2 subsamples every s-th point per
 * spatial direction).  The block stacks nfields fields, each an
 * nx x ny x nz grid: row f*nx*ny*nz + x + nx*(y + ny*z), so
 * m_b = nfields*nx*ny*nz.  Coarse coordinates per direction are
 * 0, s, 2s, ... < N (ceil(N/s) points); the coarse rows J_b keep the same
 * ordering, m_c,b = nfields * prod ceil(N/s). */
typedef struct {
  int32_t nx, ny, nz;  /* fine points per direction (>= 1) */
  int32_t nfields;     /* fields stacked along the rows (>= 1) */
  int32_t sx, sy, sz;  /* subsampling interval per direction (>= 1) */
} spid_grid;

typedef struct {
  int32_t nblocks;          /* number of spatial blocks (>= 1) */
  const int64_t* h_m;       /* host [nblocks]: rows m_b (>= 1) */
  const int32_t* h_n;       /* host [nblocks]: snapshots n_b, 1..1024 */
  int32_t l;                /* sketch rows: 1 <= l <= 128 (Gaussian); coarse
                               grid: max_b m_c,b <= l <= 2^22 */
  int32_t k_max;            /* rank (tol == 0) or rank cap (tol > 0), <= 96;
                               fixed rank requires k_max <= min(l, n_b) */
  double tol;               /* 0: fixed rank.  > 0: stop after the first step
                               with ||Y - Y(:,S)P||_F <= tol ||Y||_F (Remark
                               2.1), k_b <= min(k_max, l, n_b) */
  double rank_floor;        /* > 0: stop before a pivot whose squared residual
                               norm is <= rank_floor^2 * max_j ||Y(:,j)||^2 */
  uint64_t seed;            /* Omega seed (Philox4x32-10 key) */
  int32_t omega_per_block;  /* 0: Omega(r,i) shared by all blocks (block b
                               uses the prefix of m_b columns); 1: block b
                               keys its own Omega with b+1 */
  int32_t a_dtype;          /* spid_adtype */
  int32_t prec;             /* spid_skprec */
  int32_t lp_terms;         /* 1..3 split terms of A for BF16/FP8 (ignored
                               for F64) */
  const spid_grid* h_grid;  /* host [nblocks]: block grids, required for
                               SPID_SK_SUBSAMPLE (NULL otherwise) */
  int32_t ts_windows;       /* > 0: reserve the modified two-stage ID of
                               spid_select_two_stage with this many temporal
                               windows per block (<= every n_b); 0: off */
  int32_t ts_k1;            /* two-stage: stage-1 rank of every window,
                               1..96, ts_windows * ts_k1 <= 1024 */
} spid_desc;

/* Launch-shape choices (the batching schedule of Section 3.2's independent
 * blocks on one GPU).  Any field 0 = the library's default for the
 * descriptor; an autotuner times candidates and passes the fastest.  Shapes
 * never change results beyond the order of floating-point sums inside a
 * sketch column (K splits), so every choice meets the same parity rules.
 *   sk_tn    16-column MFMA tiles per wave in the sketch: 1, 2 or 4
 *            (FP64: 1 or 2, and 2 only for l <= 64; BF16: 4 only for
 *            l <= 80; FP8: 1).  BF16 default (0, 8 waves): each block's
 *            tiles sized to its width (1 per wave up to 128 columns, 2 up to
 *            256, else 4), one launch per size; spid_get_tuning reports 0
 *   sk_nw    waves per sketch workgroup: 8, or 4 with sk_tn = 1
 *   sk_items target number of sketch work items (64..65536): blocks are
 *            split along their rows (K) until about this many items exist
 *   rc_rpi   error-pass row sub-tiles per work item, 1..16 (double-precision
 *            error pass only; the split-bfloat16 pass uses one)
 *   st_groups one-snapshot FP8 updates of FP32 data: groups of 128 equal-m
 *            blocks one work item streams in turn, 1..16 (default 1) */
typedef struct {
  int32_t sk_tn;
  int32_t sk_nw;
  int32_t sk_items;
  int32_t rc_rpi;
  int32_t st_groups;
} spid_tuning;

/* Bytes of device workspace a descriptor needs (0 if the descriptor is
 * invalid; spid_last_error() says why).  Host-only, no HIP call. */
size_t spid_workspace_bytes(const spid_desc* desc);

/* The same for explicit launch shapes (tuning may be NULL = defaults). */
size_t spid_workspace_bytes_tuned(const spid_desc* desc, const spid_tuning* tuning);

/* Create a context on the current HIP device.  `d_workspace` (256-byte
 * aligned, >= spid_workspace_bytes) is owned by the caller and must outlive
 * the context.  Copies the block table into the workspace with a synchronous
 * copy (a set-up call: not for graph capture).  *out receives a host object
 * freed by spid_destroy. */
spid_status spid_create(const spid_desc* desc, void* d_workspace, size_t ws_bytes,
                        spid_ctx** out);

/* spid_create with explicit launch shapes (NULL = defaults).  EINVAL for a
 * value outside the ranges listed at spid_tuning. */
spid_status spid_create_tuned(const spid_desc* desc, const spid_tuning* tuning,
                              void* d_workspace, size_t ws_bytes, spid_ctx** out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, hosts that forbid hipMalloc): spid_create_tuned
 * without a caller workspace.  The context uses a file-scope device array of
 * the library, 64 MiB per device (held from the library's first use on the
 * device until the process ends), as its workspace; nothing is allocated.
 * EWORKSPACE (with the size needed) when spid_workspace_bytes_tuned exceeds
 * 64 MiB.  Every static context on a device shares that device's array: the
 * call waits for the device to finish its queued work (hipDeviceSynchronize),
 * then takes the array over, and any earlier static context on the device gets
 * ESTATE from every later call.  Calls on static contexts must not overlap in
 * time with another spid_create_static on the same device.  The kernels need no
 * zeroed workspace (every value they read was written by an earlier stage of
 * the same context).  tuning may be NULL.  A set-up call: not for graph
 * capture; the compute calls on the context are capturable as usual. */
spid_status spid_create_static(const spid_desc* desc, const spid_tuning* tuning, spid_ctx** out);

/* The launch shapes a context uses (defaults resolved), for the record. */
spid_status spid_get_tuning(const spid_ctx* ctx, spid_tuning* out);

/* Bind the snapshot data: h_block_ptrs[b] is the device address of block b
 * (column-major, m_b x n_b, A dtype), h_lda[b] >= m_b its leading dimension
 * (elements).  Host arrays of length nblocks; synchronous set-up copy.  May
 * be called again to rebind; it resets the sketch coverage. */
spid_status spid_bind_A(spid_ctx* ctx, const void* const* h_block_ptrs, const int64_t* h_lda);

/* Sketch update (Section 2, B = Omega A; Algorithm 5's per-step storage of a
 * snapshot becomes a sketch update): for every block,
 *   Y_b(:, j) = Omega_b A_b(:, j)   for j0 <= j < min(j0 + w, n_b).
 * Overwrites those sketch columns, so repeating a call is idempotent.  Called
 * once with (0, max n) for a resident batch, or once per arriving snapshot
 * with w = 1. */
spid_status spid_sketch_update(spid_ctx* ctx, int32_t j0, int32_t w, void* stream);

/* Column selection (Section 2, Algorithm 1 mgsqr on the sketch; Remark 2.1):
 * pivot = largest remaining column norm (ties: lowest column index), one
 * modified Gram-Schmidt sweep per step, norms recomputed each step.
 * Outputs (device): d_k[nblocks] = k_b, d_S[nblocks*k_max] = pivot columns of
 * block b at d_S[b*k_max + t] in pivot order (-1 past k_b),
 * d_status[nblocks].  Any output pointer may be NULL.  R is kept in the
 * workspace for spid_coeffs.  ESTATE unless every column was sketched. */
spid_status spid_select(spid_ctx* ctx, int32_t* d_k, int32_t* d_S, int32_t* d_status,
                        void* stream);

/* Modified (two-stage) ID (Section 3.4.2), in place of spid_select +
 * spid_coeffs; needs desc.ts_windows > 0.  Block b's columns form ts_windows
 * consecutive windows, window w = columns [floor(w n_b / W), floor((w+1) n_b / W)).
 *   Stage 1: rank-ts_k1 ID of every window's sketch (rank_floor applies):
 *            pivots I_w and coefficients C_w.
 *   Stage 2: ID of the concatenated window skeletons A_b(:, I_U) (I_U the
 *            stage-1 pivots shifted to columns of A_b, window order) with the
 *            descriptor's tol (0: fixed rank k_max), at most k_max columns.
 *            Its sketch is Y_b(:, I_U), gathered from the resident sketch: no
 *            pass over A.
 * Outputs as spid_select (d_S = columns of A_b in stage-2 pivot order) plus
 * d_P = C^1 C^{0'} (k_max x n_b per block, the layout of spid_coeffs, rows
 * >= k_b zero, P_b(:, S[t]) = e_t).  Afterwards spid_reconstruct measures
 * ||A_b - A_b(:,S_b) P_b||.  A window whose sketch is non-finite makes the
 * block NONFINITE (k_b = 0).  ESTATE unless every column was sketched;
 * EINVAL without ts_windows.  Any of d_k, d_S, d_status may be NULL. */
spid_status spid_select_two_stage(spid_ctx* ctx, int32_t* d_k, int32_t* d_S, int32_t* d_status,
                                  double* d_P, void* stream);

/* Coefficients (Section 2, Algorithm 1): P_b = [I | R11^+ R12] Z^T, FP64.
 * d_P holds every block's k_max x n_b column-major matrix (leading dimension
 * k_max) at element offset k_max * sum_{c<b} n_c; P_b(:, S[t]) = e_t exactly,
 * other columns solve R11 x = R12(:, j) by back-substitution, rows >= k_b are
 * zero.  ESTATE before spid_select, and after spid_select_two_stage (which
 * writes the coefficients itself). */
spid_status spid_coeffs(spid_ctx* ctx, double* d_P, void* stream);

/* Reconstruction error (Section 5.1) against the stored A:
 *   d_err2[b] = ||A_b - A_b(:,S_b) P_b||_F^2 (FP64 sum of squares),
 *   d_nrm2[b] = ||A_b||_F^2.
 * d_P as written by spid_coeffs (ESTATE unless spid_coeffs ran after the last
 * spid_select).  With FP32 data and a BF16/FP8 sketch the error pass reads
 * the split-bfloat16 copy of the same P that spid_coeffs keeps in the
 * workspace, and sums the squares of 16 entries per lane in FP32 before the
 * FP64 sums (relative error of those partial sums at most 16 * 2^-24).  d_skeleton (nullable) receives A_b(:,S_b),
 * m_b x k_max column-major in the A dtype at element offset
 * k_max * sum_{c<b} m_c (columns >= k_b untouched).  Sums are deterministic
 * (fixed reduction order).  ESTATE before spid_coeffs. */
spid_status spid_reconstruct(spid_ctx* ctx, const double* d_P, double* d_err2, double* d_nrm2,
                             void* d_skeleton, void* stream);

/* Single-pass ID error (Section 2, equation (single_ID); Algorithm 3),
 * coarse-grid sketch only:
 *   d_err2[b] = ||A_b - M_b B_b(:,S_b) P_b||_F^2 (FP64 sum of squares),
 *   d_nrm2[b] = ||A_b||_F^2,
 * B_b = Y_b the coarse sketch and M_b the trilinear interpolation from the
 * coarse grid to the fine grid, field by field (fine points at or past the
 * last coarse coordinate of a direction take that coordinate's value).
 * d_coarse_skeleton (nullable) receives B_b(:,S_b), m_c,b x k_max
 * column-major in the A dtype at element offset k_max * sum_{c<b} m_c,c
 * (columns >= k_b untouched): with P_b and the grid, what Algorithm 3
 * stores.  Reads A once; the skeleton-gather pass of spid_reconstruct (the
 * SubID error) is independent of it.  EINVAL for a Gaussian sketch, ESTATE
 * before spid_coeffs. */
spid_status spid_reconstruct_interp(spid_ctx* ctx, const double* d_P, double* d_err2,
                                    double* d_nrm2, void* d_coarse_skeleton, void* stream);

/* Test/diagnostic access: copy the sketch Y, widened to FP64, into d_Y
 * (block b: l x n_b column-major at element offset l * sum_{c<b} n_c). */
spid_status spid_copy_sketch(spid_ctx* ctx, double* d_Y, void* stream);

/* Release the host object (the workspace stays the caller's). */
spid_status spid_destroy(spid_ctx* ctx);

/* Message for the last non-OK status returned on this thread. */
const char* spid_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SPID_H */
