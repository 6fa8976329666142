/*
 * spid_oracle.c -- plain, slow, double-precision CPU reference of the sketched
 * column interpolative decomposition (ID) of per-subdomain snapshot matrices.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no source, header, table or
 * constant with the GPU library and includes none of its files.
 *
 * What it follows (arXiv 2103.01380, "Task-parallel in-situ temporal
 * compression of large-scale CFD data"):
 *   - Section 2, the column ID: every column of A is the least-squares
 *     combination of k selected columns, A ~ A(:,I) C, with C(:,I) = I_k.
 *   - Section 2, derivation from a column-pivoted QR A Z = Q R, partition of R
 *     into R11 (k x k) and R12 (k x (n-k)), and C = [I_k | R11^+ R12] Z^T;
 *     Algorithm 1 (Column ID), whose QR is a rank-k pivoted modified
 *     Gram-Schmidt ("mgsqr").
 *   - Section 2, sketching: the indices and coefficients are computed on a
 *     sketch B (l x n, k < l << m) and transferred to A as A ~ A(:,I_B) C_B;
 *     the sketch used here is the Gaussian random projection B = Omega A with
 *     i.i.d. standard normal Omega (l x m).
 *   - Section 2, the deterministic coarse-grid sketch B = A(J,:) (Algorithm
 *     2, SubID: A ~ A(:,I_B) C_B) and the single-pass form A ~ M B(:,I_B) C_B
 *     with an interpolation operator M (equation (single_ID), Algorithm 3);
 *     Section 5.2 subsamples every s-th point per direction and interpolates
 *     trilinearly.
 *   - Remark 2.1: the pivoted QR may stop at a tolerance instead of a fixed
 *     rank.
 *   - Section 3.2: every spatial block is compressed independently.
 *   - Equation (cf): compression factor CF = m n / (k (m + n)).
 *   - Section 5.1: relative Frobenius error ||A - A_approx||_F / ||A||_F.
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - Omega entries come from Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
 *     "Parallel random numbers: as easy as 1, 2, 3", SC'11) and the
 *     Box-Muller transform (Box & Muller 1958).  The counter is
 *     (spatial row i, row pair r/2, block key, stream id), the key is the
 *     64-bit seed.  Two 53-bit uniforms per Philox output.
 *   - Pivot rule: largest remaining column norm, ties to the lowest column
 *     index; norms are recomputed after every step (no downdating); a single
 *     Gram-Schmidt sweep, no re-orthogonalisation.
 *   - R11^+ R12 is formed by back-substitution (R11 is upper triangular with a
 *     nonzero diagonal whenever the pivots are nonzero, so the pseudo-inverse
 *     is the inverse).
 *   - Tolerance stop: after a step, stop when the Frobenius norm of the
 *     sketch residual is at most tol times the Frobenius norm of the sketch.
 *   - Coarse grid: coordinates 0, s, 2s, ... below the point count of each
 *     direction (ceil(N/s) points, which ends on the last point when s divides
 *     N - 1, as for the paper's 64-point intervals 3, 7 and 9); a fine point
 *     past the last coarse coordinate takes that coordinate's value.  Fields
 *     are interpolated separately.
 *   - Optional low-precision sketch matrix: Omega entries rounded to nearest
 *     even bfloat16 or OCP fp8-e4m3 from the double-precision normal (this
 *     defines a different Gaussian-like sketch matrix; the arithmetic stays in
 *     double precision).
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared -pthread (no -ffast-math, no
 * BLAS).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define REF_OK 0
#define REF_EINVAL (-1)

/* per-block numerical status, same meaning as the GPU library's */
#define REF_ST_OK 0
#define REF_ST_RANK_DEFICIENT 1
#define REF_ST_NONFINITE 2
#define REF_ST_TOL_NOT_MET 3

#define REF_A_F64 0
#define REF_A_F32 1

#define REF_OMEGA_F64 0
#define REF_OMEGA_BF16 1
#define REF_OMEGA_FP8E4M3 2

/* ------------------------------------------------------------------------- */
/* Philox4x32-10, written from the SC'11 description.                        */
/* ------------------------------------------------------------------------- */

/* one 32x32 -> 64 bit product, split into its high and low words */
static void mul_hi_lo(uint32_t a, uint32_t b, uint32_t* hi, uint32_t* lo) {
  uint64_t p = (uint64_t)a * (uint64_t)b;
  *hi = (uint32_t)(p >> 32);
  *lo = (uint32_t)p;
}

void spid_ref_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                            uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u; /* round multipliers */
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u; /* Weyl key increments */
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; round++) {
    if (round > 0) {
      k0 += W0;
      k1 += W1;
    }
    uint32_t hi0, lo0, hi1, lo1;
    mul_hi_lo(M0, c0, &hi0, &lo0);
    mul_hi_lo(M1, c2, &hi1, &lo1);
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

/* Round a double to the nearest bfloat16 (ties to even), returned as double.
 * bfloat16 keeps the float32 exponent range and 8 significant bits. */
static double round_to_bf16(double x) {
  if (x == 0.0 || !isfinite(x)) return x;
  int e;
  frexp(x, &e); /* |x| = f * 2^e, f in [0.5, 1) */
  /* normal bf16: 8 significant bits -> quantum 2^(e-8); below the smallest
   * normal (2^-126) the quantum stays 2^-133 */
  int q = e - 8;
  if (q < -133) q = -133;
  double scaled = ldexp(x, -q);       /* exact: only the exponent changes */
  double r = nearbyint(scaled);       /* default rounding mode: ties-to-even */
  return ldexp(r, q);
}

/* Round a double to the nearest OCP fp8 e4m3 ("fn") value, ties to even,
 * saturating at +-448 (the format's largest finite magnitude). */
static double round_to_e4m3(double x) {
  if (x == 0.0 || !isfinite(x)) return x;
  int e;
  frexp(x, &e);
  /* 4 significant bits -> quantum 2^(e-4); smallest normal 2^-6, subnormal
   * quantum 2^-9 */
  int q = e - 4;
  if (q < -9) q = -9;
  double r = nearbyint(ldexp(x, -q));
  double v = ldexp(r, q);
  if (v > 448.0) v = 448.0;
  if (v < -448.0) v = -448.0;
  return v;
}

/* Omega(r, i) of the sketch: standard normal from Philox + Box-Muller.
 * Counter = (i, r/2, block_key, stream 0); key = (seed low, seed high).
 * Row 2q is rho*cos(theta), row 2q+1 is rho*sin(theta). */
double spid_ref_omega(uint64_t seed, uint32_t block_key, int64_t r, int64_t i,
                      int32_t omega_prec) {
  uint32_t ctr[4] = {(uint32_t)i, (uint32_t)(r / 2), block_key, 0u};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t x[4];
  spid_ref_philox4x32_10(ctr, key, x);
  /* two 53-bit integers: 27 high bits of one word, 26 of the next */
  uint64_t n1 = ((uint64_t)(x[0] >> 5) << 26) | (uint64_t)(x[1] >> 6);
  uint64_t n2 = ((uint64_t)(x[2] >> 5) << 26) | (uint64_t)(x[3] >> 6);
  double u1 = (double)(n1 + 1) * 0x1p-53; /* (0, 1] : log is finite */
  double u2 = (double)n2 * 0x1p-53;       /* [0, 1) */
  double rho = sqrt(-2.0 * log(u1));
  double theta = 6.283185307179586 * u2; /* 2*pi rounded to double */
  double z = (r % 2 == 0) ? rho * cos(theta) : rho * sin(theta);
  if (omega_prec == REF_OMEGA_BF16) return round_to_bf16(z);
  if (omega_prec == REF_OMEGA_FP8E4M3) return round_to_e4m3(z);
  return z;
}

double spid_ref_round_bf16(double x) { return round_to_bf16(x); }
double spid_ref_round_e4m3(double x) { return round_to_e4m3(x); }

/* fill Omega (l x m, column-major, leading dimension l) */
void spid_ref_omega_matrix(uint64_t seed, uint32_t block_key, int32_t l,
                           int64_t m, int32_t omega_prec, double* omega) {
  for (int64_t i = 0; i < m; i++)
    for (int32_t r = 0; r < l; r++)
      omega[i * l + r] = spid_ref_omega(seed, block_key, r, i, omega_prec);
}

static double a_entry(const void* A, int32_t a_dtype, int64_t lda, int64_t i,
                      int64_t j) {
  if (a_dtype == REF_A_F32) return (double)((const float*)A)[j * lda + i];
  return ((const double*)A)[j * lda + i];
}

/* ------------------------------------------------------------------------- */
/* Sketch B = Omega A (Section 2, random projection).                        */
/* A: m x n column-major (leading dimension lda), float or double.          */
/* Y: l x n column-major (leading dimension l), double.                     */
/* Only columns j0 .. j0+w-1 are (over)written.                              */
/* Sum over the spatial index i in ascending order.                          */
/* ------------------------------------------------------------------------- */
int spid_ref_sketch(int64_t m, int32_t n, const void* A, int64_t lda,
                    int32_t a_dtype, int32_t l, uint64_t seed,
                    uint32_t block_key, int32_t omega_prec, int32_t j0,
                    int32_t w, double* Y) {
  if (m < 0 || n < 0 || l <= 0 || lda < m || j0 < 0 || w < 0 || j0 + w > n)
    return REF_EINVAL;
  for (int32_t j = j0; j < j0 + w; j++)
    for (int32_t r = 0; r < l; r++) Y[(int64_t)j * l + r] = 0.0;
  double* om = (double*)malloc(sizeof(double) * (size_t)l);
  if (!om) return REF_EINVAL;
  for (int64_t i = 0; i < m; i++) {
    for (int32_t r = 0; r < l; r++)
      om[r] = spid_ref_omega(seed, block_key, r, i, omega_prec);
    for (int32_t j = j0; j < j0 + w; j++) {
      double a = a_entry(A, a_dtype, lda, i, j);
      for (int32_t r = 0; r < l; r++) Y[(int64_t)j * l + r] += om[r] * a;
    }
  }
  free(om);
  return REF_OK;
}

/* ------------------------------------------------------------------------- */
/* Coarse grid of the deterministic sketch (Section 2: B = A(J,:) keeps the   */
/* rows of a coarse-grid representation; Section 5.2 subsamples every s-th  */
/* point in each spatial direction).                                          */
/*                                                                           */
/* grid[7] = {nx, ny, nz, nf, sx, sy, sz}: the block stacks nf fields, each   */
/* on an nx x ny x nz structured grid; fine row = f*nx*ny*nz + x + nx*(y +   */
/* ny*z).  Coarse coordinates per direction are 0, s, 2s, ... below the      */
/* point count (ceil(N/s) of them); the coarse rows J are ordered the same   */
/* way (field, then z, y, x with x fastest).                                 */
/* ------------------------------------------------------------------------- */
static int32_t coarse_points(int32_t npts, int32_t s) { return (npts + s - 1) / s; }

/* Number of coarse rows m_c of a grid, or -1 when the grid is invalid. */
int32_t spid_ref_coarse_count(const int32_t* grid) {
  for (int d = 0; d < 7; d++)
    if (grid[d] < 1) return -1;
  int64_t c = (int64_t)grid[3] * coarse_points(grid[0], grid[4]) *
              coarse_points(grid[1], grid[5]) * coarse_points(grid[2], grid[6]);
  return c > INT32_MAX ? -1 : (int32_t)c;
}

/* The coarse rows J (ascending), m_c of them; returns m_c or -1. */
int32_t spid_ref_coarse_rows(const int32_t* grid, int32_t* J) {
  int32_t mc = spid_ref_coarse_count(grid);
  if (mc < 0) return -1;
  int32_t nx = grid[0], ny = grid[1], nz = grid[2], nf = grid[3];
  int32_t cx = coarse_points(nx, grid[4]), cy = coarse_points(ny, grid[5]);
  int32_t cz = coarse_points(nz, grid[6]);
  int64_t pts = (int64_t)nx * ny * nz;
  int32_t r = 0;
  for (int32_t f = 0; f < nf; f++)
    for (int32_t tz = 0; tz < cz; tz++)
      for (int32_t ty = 0; ty < cy; ty++)
        for (int32_t tx = 0; tx < cx; tx++)
          J[r++] = (int32_t)(f * pts + (int64_t)tx * grid[4] +
                             (int64_t)nx * ((int64_t)ty * grid[5] + (int64_t)ny * tz * grid[6]));
  return mc;
}

/* Linear interpolation weights along one direction: fine coordinate x from   */
/* coarse points t*s, t < nc.  Between two coarse points the usual two        */
/* weights; at or beyond the last coarse point (a direction whose point count */
/* is not 1 + a multiple of s) the value of the last coarse point.            */
static void lin_weights(int32_t x, int32_t s, int32_t nc, int32_t t[2], double w[2]) {
  int32_t t0 = x / s;
  if (t0 >= nc - 1) {
    t[0] = t[1] = nc - 1;
    w[0] = 1.0;
    w[1] = 0.0;
    return;
  }
  double frac = (double)(x - t0 * s) / (double)s;
  t[0] = t0;
  t[1] = t0 + 1;
  w[0] = 1.0 - frac;
  w[1] = frac;
}

/* Row i of the trilinear interpolation operator M (fine grid <- coarse grid, */
/* field by field): 8 coarse-row indices and weights (the tensor product of   */
/* the three directions' linear weights).  Returns 0, or -1 for a bad row.    */
int spid_ref_interp_row(const int32_t* grid, int64_t i, int32_t idx[8], double w[8]) {
  if (spid_ref_coarse_count(grid) < 0) return -1;
  int32_t nx = grid[0], ny = grid[1], nz = grid[2], nf = grid[3];
  int64_t pts = (int64_t)nx * ny * nz;
  if (i < 0 || i >= pts * nf) return -1;
  int32_t f = (int32_t)(i / pts);
  int64_t p = i - f * pts;
  int32_t x = (int32_t)(p % nx), y = (int32_t)((p / nx) % ny), z = (int32_t)(p / ((int64_t)nx * ny));
  int32_t cx = coarse_points(nx, grid[4]), cy = coarse_points(ny, grid[5]);
  int32_t cz = coarse_points(nz, grid[6]);
  int32_t tx[2], ty[2], tz[2];
  double wx[2], wy[2], wz[2];
  lin_weights(x, grid[4], cx, tx, wx);
  lin_weights(y, grid[5], cy, ty, wy);
  lin_weights(z, grid[6], cz, tz, wz);
  int c = 0;
  for (int a = 0; a < 2; a++)
    for (int b = 0; b < 2; b++)
      for (int d = 0; d < 2; d++) {
        idx[c] = f * cx * cy * cz + tx[d] + cx * (ty[b] + cy * tz[a]);
        w[c] = wz[a] * wy[b] * wx[d];
        c++;
      }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Subsampled sketch B = A(J, :) (Section 2; Algorithm 2, step 3): row r of  */
/* B is row J[r] of A, widened exactly to double.  Y: mc x n column-major,   */
/* leading dimension ldy >= mc.  Only columns j0 .. j0+w-1 are written.      */
/* ------------------------------------------------------------------------- */
int spid_ref_subsample(int64_t m, int32_t n, const void* A, int64_t lda,
                       int32_t a_dtype, const int32_t* J, int32_t mc, int32_t ldy,
                       int32_t j0, int32_t w, double* Y) {
  if (m < 0 || n < 0 || mc <= 0 || ldy < mc || lda < m || j0 < 0 || w < 0 || j0 + w > n || !J)
    return REF_EINVAL;
  for (int32_t r = 0; r < mc; r++)
    if (J[r] < 0 || J[r] >= m) return REF_EINVAL;
  for (int32_t j = j0; j < j0 + w; j++)
    for (int32_t r = 0; r < mc; r++)
      Y[(int64_t)j * ldy + r] = a_entry(A, a_dtype, lda, J[r], j);
  return REF_OK;
}

/* ------------------------------------------------------------------------- */
/* mgsqr: rank-k column-pivoted QR by modified Gram-Schmidt (Section 2,     */
/* Algorithm 1), optionally stopped at a tolerance (Remark 2.1).             */
/*                                                                           */
/* In : Y, l x n column-major (not modified).                               */
/* Out: S[0..k_eff-1] pivot columns in pivot order (rest -1), *k_eff,       */
/*      R (k_max x n, row-major: R[s*n + j] = R(s, j) in ORIGINAL column    */
/*      numbering, so R11[s][t] = R[s*n + S[t]] and R12 are the columns not */
/*      in S), nu (final squared residual column norms, selected -> 0),     */
/*      gaps[s] = (sqrt(nu_(1)) - sqrt(nu_(2))) / sqrt(nu0max) at step s     */
/*      (top two remaining norms; 1 when one column remains), *status.      */
/* rank_floor > 0 stops before a pivot whose squared norm is at most        */
/* rank_floor^2 * nu0max.                                                     */
/* ------------------------------------------------------------------------- */
int spid_ref_select(int32_t l, int32_t n, const double* Y, int32_t k_max,
                    double tol, double rank_floor, int32_t* S, int32_t* k_eff,
                    double* R, double* nu_out, double* gaps, int32_t* status,
                    double* res2_out) {
  if (l <= 0 || n <= 0 || k_max <= 0 || tol < 0.0 || rank_floor < 0.0)
    return REF_EINVAL;
  int32_t kcap = k_max;
  if (kcap > l) kcap = l;
  if (kcap > n) kcap = n;
  double* W = (double*)malloc(sizeof(double) * (size_t)l * (size_t)n);
  double* nu = (double*)malloc(sizeof(double) * (size_t)n);
  double* q = (double*)malloc(sizeof(double) * (size_t)l);
  unsigned char* sel = (unsigned char*)calloc((size_t)n, 1);
  if (!W || !nu || !q || !sel) {
    free(W); free(nu); free(q); free(sel);
    return REF_EINVAL;
  }
  memcpy(W, Y, sizeof(double) * (size_t)l * (size_t)n);
  for (int32_t s = 0; s < k_max; s++) {
    S[s] = -1;
    gaps[s] = 0.0;
    for (int32_t j = 0; j < n; j++) R[(int64_t)s * n + j] = 0.0;
  }
  int32_t st = REF_ST_OK;
  /* non-finite sketch entries: nothing can be selected */
  for (int64_t t = 0; t < (int64_t)l * n; t++)
    if (!isfinite(W[t])) st = REF_ST_NONFINITE;
  double F2 = 0.0, nu0max = 0.0;
  for (int32_t j = 0; j < n; j++) {
    double acc = 0.0;
    for (int32_t r = 0; r < l; r++) acc += W[(int64_t)j * l + r] * W[(int64_t)j * l + r];
    nu[j] = acc;
    F2 += acc;
    if (acc > nu0max) nu0max = acc;
  }
  int32_t taken = 0;
  if (st == REF_ST_OK) {
    for (int32_t s = 0; s < kcap; s++) {
      /* pivot: largest remaining norm, lowest index on ties */
      int32_t p = -1;
      double best = -1.0, second = -1.0;
      for (int32_t j = 0; j < n; j++) {
        if (sel[j]) continue;
        if (nu[j] > best) {
          second = best;
          best = nu[j];
          p = j;
        } else if (nu[j] > second) {
          second = nu[j];
        }
      }
      if (p < 0 || best <= 0.0) {
        st = REF_ST_RANK_DEFICIENT;
        break;
      }
      if (rank_floor > 0.0 && best <= rank_floor * rank_floor * nu0max) {
        st = REF_ST_RANK_DEFICIENT;
        break;
      }
      gaps[s] = (second < 0.0) ? 1.0
                               : (sqrt(best) - sqrt(second > 0.0 ? second : 0.0)) / sqrt(nu0max);
      /* r_ss = ||W(:,p)||, q = W(:,p) / r_ss */
      double pn = 0.0;
      for (int32_t r = 0; r < l; r++) pn += W[(int64_t)p * l + r] * W[(int64_t)p * l + r];
      double rss = sqrt(pn);
      for (int32_t r = 0; r < l; r++) q[r] = W[(int64_t)p * l + r] / rss;
      S[s] = p;
      sel[p] = 1;
      R[(int64_t)s * n + p] = rss;
      taken = s + 1;
      /* orthogonalise every remaining column against q (one MGS sweep) */
      double rest = 0.0;
      for (int32_t j = 0; j < n; j++) {
        if (sel[j]) continue;
        double* wj = W + (int64_t)j * l;
        double d = 0.0;
        for (int32_t r = 0; r < l; r++) d += q[r] * wj[r];
        R[(int64_t)s * n + j] = d;
        for (int32_t r = 0; r < l; r++) wj[r] -= d * q[r];
        double acc = 0.0;
        for (int32_t r = 0; r < l; r++) acc += wj[r] * wj[r];
        nu[j] = acc;
        rest += acc;
      }
      if (tol > 0.0 && sqrt(rest) <= tol * sqrt(F2)) break;
      if (tol > 0.0 && s == kcap - 1) st = REF_ST_TOL_NOT_MET;
    }
  }
  double res2 = 0.0;
  for (int32_t j = 0; j < n; j++) {
    if (sel[j]) nu[j] = 0.0;
    if (nu_out) nu_out[j] = nu[j];
    res2 += nu[j];
  }
  if (res2_out) *res2_out = res2;
  *k_eff = taken;
  *status = st;
  free(W);
  free(nu);
  free(q);
  free(sel);
  return REF_OK;
}

/* ------------------------------------------------------------------------- */
/* Coefficients C = [I_k | R11^+ R12] Z^T (Section 2, Algorithm 1).          */
/* P: k_max x n column-major (leading dimension k_max); rows >= k_eff are 0. */
/* P(:, S[t]) = e_t; every other column solves R11 x = R12(:, j) by          */
/* back-substitution.                                                        */
/* ------------------------------------------------------------------------- */
int spid_ref_coeffs(int32_t k_eff, int32_t k_max, int32_t n, const double* R,
                    const int32_t* S, double* P) {
  if (k_eff < 0 || k_eff > k_max || n <= 0) return REF_EINVAL;
  for (int64_t t = 0; t < (int64_t)k_max * n; t++) P[t] = 0.0;
  unsigned char* sel = (unsigned char*)calloc((size_t)n, 1);
  double* x = (double*)malloc(sizeof(double) * (size_t)(k_eff > 0 ? k_eff : 1));
  if (!sel || !x) {
    free(sel); free(x);
    return REF_EINVAL;
  }
  for (int32_t t = 0; t < k_eff; t++) {
    sel[S[t]] = 1;
    P[(int64_t)S[t] * k_max + t] = 1.0; /* identity block */
  }
  for (int32_t j = 0; j < n; j++) {
    if (sel[j]) continue;
    for (int32_t s = k_eff - 1; s >= 0; s--) {
      double acc = R[(int64_t)s * n + j];                 /* R12(s, j) */
      for (int32_t t = s + 1; t < k_eff; t++)
        acc -= R[(int64_t)s * n + S[t]] * x[t];           /* R11(s, t) x_t */
      x[s] = acc / R[(int64_t)s * n + S[s]];              /* / R11(s, s) */
    }
    for (int32_t s = 0; s < k_eff; s++) P[(int64_t)j * k_max + s] = x[s];
  }
  free(sel);
  free(x);
  return REF_OK;
}

/* ------------------------------------------------------------------------- */
/* Modified (two-stage) ID (Section 3.4.2) on the sketch Y (l x n) of one     */
/* block.  Windows w = 0..nwin-1 hold columns [c_w, c_{w+1}), c_w =          */
/* floor(w n / nwin) (n/N time steps each when nwin divides n).              */
/*   Stage 1: rank-k1 ID of each window: I_w (window positions), C_w.        */
/*   Stage 2: the concatenated skeleton A^{0'} = A(:, I_U), I_U the union of  */
/*     the I_w shifted by c_w in window order, has the sketch Y(:, I_U) (one  */
/*     sketch matrix serves every column); its ID with tolerance tol2 and at  */
/*     most k_max columns gives I_1 (positions in I_U) and C^1.              */
/*   Result: S = I_U(I_1) in stage-2 pivot order, P = C^1 C^{0'} (k_max x n, */
/*     column-major, rows >= k zero), C^{0'} block-diagonal of the C_w.      */
/* status: the stage-2 status, or NONFINITE (k = 0) when a window's sketch   */
/* holds a non-finite entry.  gaps: the stage-2 relative top-two gaps.       */
/* ------------------------------------------------------------------------- */
int spid_ref_two_stage(int32_t l, int32_t n, const double* Y, int32_t nwin, int32_t k1,
                       double rank_floor, int32_t k_max, double tol2, int32_t* S,
                       int32_t* k_eff, int32_t* status, double* P, double* gaps) {
  if (l <= 0 || n <= 0 || nwin < 1 || nwin > n || k1 < 1 || k_max < 1 || tol2 < 0.0)
    return REF_EINVAL;
  int rc = REF_OK;
  int32_t* I1 = (int32_t*)malloc(sizeof(int32_t) * (size_t)nwin * k1);
  int32_t* kw = (int32_t*)calloc((size_t)nwin, sizeof(int32_t));
  int32_t* IU = (int32_t*)malloc(sizeof(int32_t) * (size_t)nwin * k1);
  int32_t* owner = (int32_t*)malloc(sizeof(int32_t) * (size_t)nwin * k1);
  double* Cw = (double*)calloc((size_t)k1 * n, sizeof(double));       /* C_w, window by window */
  double* R1 = (double*)malloc(sizeof(double) * (size_t)k1 * n);
  double* g1 = (double*)malloc(sizeof(double) * (size_t)k1);
  double* Y2 = (double*)malloc(sizeof(double) * (size_t)l * nwin * k1);
  double* R2 = (double*)malloc(sizeof(double) * (size_t)k_max * nwin * k1);
  double* C1 = (double*)malloc(sizeof(double) * (size_t)k_max * nwin * k1);
  if (!I1 || !kw || !IU || !owner || !Cw || !R1 || !g1 || !Y2 || !R2 || !C1) {
    rc = REF_EINVAL;
    goto done;
  }
  for (int64_t t = 0; t < (int64_t)k_max * n; t++) P[t] = 0.0;
  for (int32_t s = 0; s < k_max; s++) {
    S[s] = -1;
    gaps[s] = 0.0;
  }
  *k_eff = 0;
  /* Stage 1 */
  int32_t nu_cols = 0, nonfinite = 0;
  for (int32_t w = 0; w < nwin; w++) {
    int32_t c0 = (int32_t)((int64_t)w * n / nwin), c1 = (int32_t)((int64_t)(w + 1) * n / nwin);
    int32_t nw = c1 - c0, st1;
    rc = spid_ref_select(l, nw, Y + (int64_t)c0 * l, k1, 0.0, rank_floor, I1 + (int64_t)w * k1,
                         kw + w, R1, NULL, g1, &st1, NULL);
    if (rc != REF_OK) goto done;
    if (st1 == REF_ST_NONFINITE) nonfinite = 1;
    rc = spid_ref_coeffs(kw[w], k1, nw, R1, I1 + (int64_t)w * k1, Cw + (int64_t)c0 * k1);
    if (rc != REF_OK) goto done;
    for (int32_t t = 0; t < kw[w]; t++) {
      IU[nu_cols] = c0 + I1[(int64_t)w * k1 + t];
      owner[nu_cols] = w;
      nu_cols++;
    }
  }
  if (nonfinite || nu_cols == 0) {
    *status = nonfinite ? REF_ST_NONFINITE : REF_ST_RANK_DEFICIENT;
    goto done;
  }
  /* Stage 2: the sketch of A(:, I_U) is Y(:, I_U) */
  for (int32_t c = 0; c < nu_cols; c++)
    memcpy(Y2 + (int64_t)c * l, Y + (int64_t)IU[c] * l, sizeof(double) * (size_t)l);
  int32_t S2[1024], k2 = 0;
  if (k_max > 1024) {
    rc = REF_EINVAL;
    goto done;
  }
  rc = spid_ref_select(l, nu_cols, Y2, k_max, tol2, rank_floor, S2, &k2, R2, NULL, gaps, status,
                       NULL);
  if (rc != REF_OK) goto done;
  rc = spid_ref_coeffs(k2, k_max, nu_cols, R2, S2, C1);
  if (rc != REF_OK) goto done;
  /* C^{1'} = C^1 C^{0'}: column j of window w combines the stage-2 columns of   */
  /* that window's skeleton with the stage-1 coefficients of j                   */
  for (int32_t w = 0; w < nwin; w++) {
    int32_t c0 = (int32_t)((int64_t)w * n / nwin), c1 = (int32_t)((int64_t)(w + 1) * n / nwin);
    for (int32_t j = c0; j < c1; j++)
      for (int32_t s = 0; s < k2; s++) {
        double acc = 0.0;
        int32_t t = 0;
        for (int32_t c = 0; c < nu_cols; c++) {
          if (owner[c] != w) continue;
          acc += C1[(int64_t)c * k_max + s] * Cw[(int64_t)j * k1 + t];
          t++;
        }
        P[(int64_t)j * k_max + s] = acc;
      }
  }
  for (int32_t s = 0; s < k2; s++) S[s] = IU[S2[s]];
  *k_eff = k2;
done:
  free(I1); free(kw); free(IU); free(owner); free(Cw); free(R1); free(g1); free(Y2); free(R2);
  free(C1);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* Reconstruction error against the stored A (Section 5.1):                  */
/* err2 = sum_j ||A(:,j) - sum_t A(:,S[t]) P(t,j)||^2 over every column,     */
/* nrm2 = ||A||_F^2.  Sums in ascending i, then ascending j.                 */
/* ------------------------------------------------------------------------- */
int spid_ref_reconstruct(int64_t m, int32_t n, const void* A, int64_t lda,
                         int32_t a_dtype, int32_t k_eff, int32_t k_max,
                         const int32_t* S, const double* P, double* err2,
                         double* nrm2) {
  if (m < 0 || n <= 0 || lda < m || k_eff < 0 || k_eff > k_max) return REF_EINVAL;
  double e2 = 0.0, a2 = 0.0;
  for (int32_t j = 0; j < n; j++) {
    double ej = 0.0, aj = 0.0;
    for (int64_t i = 0; i < m; i++) {
      double approx = 0.0;
      for (int32_t t = 0; t < k_eff; t++)
        approx += a_entry(A, a_dtype, lda, i, S[t]) * P[(int64_t)j * k_max + t];
      double a = a_entry(A, a_dtype, lda, i, j);
      double r = a - approx;
      ej += r * r;
      aj += a * a;
    }
    e2 += ej;
    a2 += aj;
  }
  *err2 = e2;
  *nrm2 = a2;
  return REF_OK;
}

/* Single-pass error (Section 2, equation (single_ID); Algorithm 3): the     */
/* approximation is M B(:,S) P, with M the trilinear interpolation of         */
/* spid_ref_interp_row and B the coarse sketch (mc x n, leading dimension     */
/* ldb).  err2 = sum_j ||A(:,j) - (M B(:,S) P)(:,j)||^2, nrm2 = ||A||_F^2.    */
/* The interpolated skeleton K = M B(:,S) (m x k) is formed first, then K P;  */
/* sums in ascending i, then ascending j.                                     */
int spid_ref_interp_error(const int32_t* grid, int64_t m, int32_t n, const void* A,
                          int64_t lda, int32_t a_dtype, const double* B, int32_t ldb,
                          int32_t k_eff, int32_t k_max, const int32_t* S,
                          const double* P, double* err2, double* nrm2) {
  int32_t mc = spid_ref_coarse_count(grid);
  if (mc < 0 || (int64_t)grid[0] * grid[1] * grid[2] * grid[3] != m || ldb < mc ||
      n <= 0 || lda < m || k_eff < 0 || k_eff > k_max)
    return REF_EINVAL;
  double* K = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1) *
                              (size_t)(k_eff > 0 ? k_eff : 1));
  if (!K) return REF_EINVAL;
  for (int64_t i = 0; i < m; i++) {
    int32_t idx[8];
    double w[8];
    spid_ref_interp_row(grid, i, idx, w);
    for (int32_t t = 0; t < k_eff; t++) {
      double v = 0.0;
      for (int c = 0; c < 8; c++) v += w[c] * B[(int64_t)S[t] * ldb + idx[c]];
      K[(int64_t)t * m + i] = v;
    }
  }
  double e2 = 0.0, a2 = 0.0;
  for (int32_t j = 0; j < n; j++) {
    double ej = 0.0, aj = 0.0;
    for (int64_t i = 0; i < m; i++) {
      double approx = 0.0;
      for (int32_t t = 0; t < k_eff; t++)
        approx += K[(int64_t)t * m + i] * P[(int64_t)j * k_max + t];
      double a = a_entry(A, a_dtype, lda, i, j);
      double r = a - approx;
      ej += r * r;
      aj += a * a;
    }
    e2 += ej;
    a2 += aj;
  }
  free(K);
  *err2 = e2;
  *nrm2 = a2;
  return REF_OK;
}

/* Compression factor, equation (cf), summed over blocks as in Section 3.2:
 * CF = sum_b m_b n_b / sum_b k_b (ms_b + n_b), counting matrix entries.  ms_b is the
 * row count of the stored skeleton: m_b for the ID and SubID, the coarse m_c for
 * SPID (disk storage of Table 2 without the interpolation stencil); pass NULL for
 * ms = m. */
double spid_ref_compression_factor(int32_t nblocks, const int64_t* m,
                                   const int32_t* n, const int32_t* k,
                                   const int64_t* ms) {
  double num = 0.0, den = 0.0;
  for (int32_t b = 0; b < nblocks; b++) {
    double rows = ms ? (double)ms[b] : (double)m[b];
    num += (double)m[b] * (double)n[b];
    den += (double)k[b] * (rows + (double)n[b]);
  }
  return den > 0.0 ? num / den : INFINITY;
}

/* ------------------------------------------------------------------------- */
/* Whole pipeline over a batch of independent blocks (Section 3.2), one      */
/* POSIX thread pool over blocks.                                             */
/*                                                                           */
/* A_ptrs[b]: host pointer to block b (m[b] x n[b], leading dimension         */
/* lda[b]).  Outputs per block b, with offsets off_S[b] = b*k_max,           */
/* off_P = sum_{c<b} k_max*n[c], off_Y = sum_{c<b} l*n[c]:                   */
/*   S[b*k_max ...], k[b], status[b], P (k_max x n[b] column-major), Y,      */
/*   gaps[b*k_max ...], err2[b], nrm2[b].                                    */
/* grids (NULL: Gaussian sketch): grids[7*b ...] is block b's coarse grid;   */
/* the sketch is then B = A(J,:) (SubID, Algorithm 2) and, if ierr2 is not   */
/* NULL, ierr2[b] receives the single-pass error of Algorithm 3.             */
/* ------------------------------------------------------------------------- */
typedef struct {
  int32_t nblocks;
  const int64_t* m;
  const int32_t* n;
  const void* const* A;
  const int64_t* lda;
  int32_t a_dtype, l, k_max;
  double tol, rank_floor;
  uint64_t seed;
  int32_t omega_per_block, omega_prec;
  int32_t *S, *k, *status;
  double *P, *Y, *gaps, *err2, *nrm2;
  const int64_t *off_P, *off_Y;
  const int32_t* grids; /* non-NULL: coarse-grid sketch, grids[7*b ...] */
  double* ierr2;        /* with grids, non-NULL: single-pass error */
  int32_t next; /* next block to take, guarded by mu */
  pthread_mutex_t mu;
  int32_t rc;
} batch_job;

static void run_one_block(batch_job* jb, int32_t b) {
  int64_t m = jb->m[b];
  int32_t n = jb->n[b];
  double* Y = jb->Y + jb->off_Y[b];
  double* P = jb->P + jb->off_P[b];
  uint32_t bkey = jb->omega_per_block ? (uint32_t)(b + 1) : 0u;
  int32_t ly = jb->l; /* rows the selection sees */
  int rc = REF_OK;
  if (jb->grids) {
    /* SubID / SPID: B = A(J,:) with J the block's coarse rows; rows of the  */
    /* l-row output past m_c stay zero (they change no sum of the selection) */
    const int32_t* g = jb->grids + 7 * (int64_t)b;
    int32_t mc = spid_ref_coarse_count(g);
    int32_t* J = mc > 0 ? (int32_t*)malloc(sizeof(int32_t) * (size_t)mc) : NULL;
    if (!J || mc > jb->l || (int64_t)g[0] * g[1] * g[2] * g[3] != m) {
      rc = REF_EINVAL;
    } else {
      spid_ref_coarse_rows(g, J);
      memset(Y, 0, sizeof(double) * (size_t)jb->l * (size_t)n);
      rc = spid_ref_subsample(m, n, jb->A[b], jb->lda[b], jb->a_dtype, J, mc, jb->l, 0, n, Y);
      ly = jb->l;
    }
    free(J);
  } else {
    rc = spid_ref_sketch(m, n, jb->A[b], jb->lda[b], jb->a_dtype, jb->l, jb->seed, bkey,
                         jb->omega_prec, 0, n, Y);
  }
  double* R = (double*)malloc(sizeof(double) * (size_t)jb->k_max * (size_t)n);
  if (rc == REF_OK && R) {
    rc = spid_ref_select(ly, n, Y, jb->k_max, jb->tol, jb->rank_floor,
                         jb->S + (int64_t)b * jb->k_max, jb->k + b, R, NULL,
                         jb->gaps + (int64_t)b * jb->k_max, jb->status + b, NULL);
  }
  if (rc == REF_OK && R)
    rc = spid_ref_coeffs(jb->k[b], jb->k_max, n, R, jb->S + (int64_t)b * jb->k_max, P);
  if (rc == REF_OK && R)
    rc = spid_ref_reconstruct(m, n, jb->A[b], jb->lda[b], jb->a_dtype, jb->k[b],
                              jb->k_max, jb->S + (int64_t)b * jb->k_max, P,
                              jb->err2 + b, jb->nrm2 + b);
  if (rc == REF_OK && R && jb->grids && jb->ierr2) {
    double a2;
    rc = spid_ref_interp_error(jb->grids + 7 * (int64_t)b, m, n, jb->A[b], jb->lda[b],
                               jb->a_dtype, Y, jb->l, jb->k[b], jb->k_max,
                               jb->S + (int64_t)b * jb->k_max, P, jb->ierr2 + b, &a2);
  }
  free(R);
  if (rc != REF_OK || !R) {
    pthread_mutex_lock(&jb->mu);
    jb->rc = REF_EINVAL;
    pthread_mutex_unlock(&jb->mu);
  }
}

static void* batch_worker(void* arg) {
  batch_job* jb = (batch_job*)arg;
  for (;;) {
    pthread_mutex_lock(&jb->mu);
    int32_t b = jb->next++;
    pthread_mutex_unlock(&jb->mu);
    if (b >= jb->nblocks) break;
    run_one_block(jb, b);
  }
  return NULL;
}

int spid_ref_run_batch(int32_t nblocks, const int64_t* m, const int32_t* n,
                       const void* const* A, const int64_t* lda, int32_t a_dtype,
                       int32_t l, int32_t k_max, double tol, double rank_floor,
                       uint64_t seed, int32_t omega_per_block, int32_t omega_prec,
                       const int64_t* off_Y, const int64_t* off_P, int32_t nthreads,
                       double* Y, int32_t* S, int32_t* k, int32_t* status, double* P,
                       double* gaps, double* err2, double* nrm2, const int32_t* grids,
                       double* ierr2) {
  if (nblocks <= 0 || l <= 0 || k_max <= 0) return REF_EINVAL;
  batch_job jb;
  memset(&jb, 0, sizeof jb);
  jb.nblocks = nblocks; jb.m = m; jb.n = n; jb.A = A; jb.lda = lda;
  jb.a_dtype = a_dtype; jb.l = l; jb.k_max = k_max; jb.tol = tol;
  jb.rank_floor = rank_floor; jb.seed = seed; jb.omega_per_block = omega_per_block;
  jb.omega_prec = omega_prec; jb.S = S; jb.k = k; jb.status = status; jb.P = P;
  jb.Y = Y; jb.gaps = gaps; jb.err2 = err2; jb.nrm2 = nrm2; jb.off_P = off_P;
  jb.off_Y = off_Y; jb.grids = grids; jb.ierr2 = ierr2; jb.next = 0; jb.rc = REF_OK;
  pthread_mutex_init(&jb.mu, NULL);
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  pthread_t th[256];
  int started = 0;
  for (int t = 0; t < nthreads; t++)
    if (pthread_create(&th[started], NULL, batch_worker, &jb) == 0) started++;
  if (started == 0) batch_worker(&jb);
  for (int t = 0; t < started; t++) pthread_join(th[t], NULL);
  pthread_mutex_destroy(&jb.mu);
  return jb.rc;
}
