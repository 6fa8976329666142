// spid_device.h -- device helpers of the gfx950 sketched-ID kernels:
// counter-based generator, normal transform, low-precision rounding, wave
// reductions and the MFMA wrappers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spid {

typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
// element-aligned vectors: one load instruction for consecutive elements of a
// column whose start is not 16-byte aligned (gfx950 accepts dword-aligned
// multi-dword global loads)
typedef float f32x4u __attribute__((ext_vector_type(4), aligned(4)));
typedef double f64x2u __attribute__((ext_vector_type(2), aligned(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplications with the key bumped by the Weyl constants
// between rounds.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    if (round) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    // one 32x32->64 product each (v_mad_u64_u32) instead of separate lo/hi multiplies
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1,
                   (uint32_t)p0);
  }
  return c;
}

// Sketch-matrix entries Omega(2q, i) and Omega(2q+1, i): one Philox block at
// counter (i, q, block key, stream 0) under the 64-bit seed, two 53-bit
// uniforms (u1 in (0,1], u2 in [0,1)), Box-Muller in double precision.
// A pointer into global memory (address space 1).  Data pointers that reach a
// kernel through a table in memory are otherwise generic, and the compiler
// then emits flat loads, whose completion shares the counter of LDS
// accesses: every wait for LDS data would also wait for the A loads in
// flight.  Global loads also take the scalar-base addressing form.
template <typename T>
using gptr = const __attribute__((address_space(1))) T*;

__device__ __forceinline__ void omega_words(uint64_t seed, uint32_t bkey, uint32_t i, uint32_t q,
                                            uint64_t& a, uint64_t& b) {
  const uint4 x = philox4x32_10(make_uint4(i, q, bkey, 0u), (uint32_t)seed,
                                (uint32_t)(seed >> 32));
  a = ((uint64_t)(x.x >> 5) << 26) | (uint64_t)(x.y >> 6);
  b = ((uint64_t)(x.z >> 5) << 26) | (uint64_t)(x.w >> 6);
}

// The angle theta = 2 pi u2 is taken in half-revolutions: sincospi(2 u2)
// (2 u2 is exact, its reduction to an octant is exact), about half the
// double-precision operations of sin/cos of a rounded product 2 pi u2, which
// it matches within 1e-15 absolute (the rounding of that product).
__device__ __forceinline__ double2 box_muller_f64(uint64_t a, uint64_t b) {
  const double u1 = (double)(a + 1u) * 0x1p-53;
  const double u2 = (double)b * 0x1p-53;
  const double rho = sqrt(-2.0 * log(u1));
  double s, c;
  sincospi(2.0 * u2, &s, &c);
  return make_double2(rho * c, rho * s);
}

__device__ __forceinline__ double2 omega_pair(uint64_t seed, uint32_t bkey, uint32_t i,
                                              uint32_t q) {
  uint64_t a, b;
  omega_words(seed, bkey, i, q, a, b);
  return box_muller_f64(a, b);
}

// Round-to-nearest-even of a double to bfloat16 precision (8 significant
// bits), result as a double.  Valid for zero and for normal values inside
// the bfloat16 exponent range (the normals of the sketch matrix).
__device__ __forceinline__ double rne_bf16(double x) {
  // keep the top 7 of the 52 stored fraction bits: add half an ulp minus one
  // plus the kept lsb (ties to even), then clear the 45 dropped bits
  uint64_t u = (uint64_t)__double_as_longlong(x);
  const uint64_t drop = (1ull << 45) - 1ull;
  u += ((1ull << 44) - 1ull) + ((u >> 45) & 1ull);
  u &= ~drop;
  return __longlong_as_double((long long)u);
}

// Round-to-nearest-even of a double to OCP fp8 e4m3 ("fn"): 4 significant
// bits for |x| >= 2^-6, quantum 2^-9 below, saturated at +-448.
__device__ __forceinline__ double rne_e4m3(double x) {
  double r;
  if (fabs(x) < 0.015625) {
    r = rint(x * 512.0) * 0.001953125;
  } else {
    uint64_t u = (uint64_t)__double_as_longlong(x);
    const uint64_t drop = (1ull << 49) - 1ull;
    u += ((1ull << 48) - 1ull) + ((u >> 49) & 1ull);
    u &= ~drop;
    r = __longlong_as_double((long long)u);
  }
  return fmin(fmax(r, -448.0), 448.0);
}

// The same roundings of a float (results exactly representable in float).
__device__ __forceinline__ float rne_bf16_f(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xFFFF0000u);
}

__device__ __forceinline__ float rne_e4m3_f(float x) {
  float r;
  if (fabsf(x) < 0.015625f) {
    r = rintf(x * 512.0f) * 0.001953125f;
  } else {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFFu + ((u >> 20) & 1u);
    r = __uint_as_float(u & 0xFFF00000u);
  }
  return fminf(fmaxf(r, -448.0f), 448.0f);
}

// Omega pair rounded to nearest-even bfloat16 (KIND 0) or e4m3 (KIND 1) for
// the low-precision sketches: equal to rounding the double-precision pair of
// omega_pair, evaluated cheaply.  Box-Muller first runs in single precision
// on the hardware transcendentals:
//   ln u1: u1 > 7/8: -(v + v^2/2 + ... + v^8/8) with v = 1 - u1 taken exactly
//          from the integer (truncation 6e-9, rounding 5.5e-7 relative);
//          else log2(fl(u1)) ln 2 (v_log_f32: relative error <= 1.2e-7 over
//          every float input in [2^-53, 1], measured exhaustively on gfx950;
//          input rounding 6e-8 absolute, |ln u1| >= 0.133): relative error
//          <= 6.6e-7, so rho = sqrt(-2 ln u1) is within 3.9e-7 relative;
//   sin / cos of 2 pi u2: v_sin_f32 / v_cos_f32 take revolutions; their error
//          is <= 1.26e-7 absolute over every float in [0, 1) (exhaustive), the
//          rounding of u2 to single adds <= 1.9e-7.
// So |dz| <= 7.6e-7 rho for both values.  With eps = rho 2^-19 (1.9e-6 rho;
// forming z -+ eps in single precision narrows the bracket by at most one ulp
// of z, 6e-8 rho) every value between fl(z - eps) and fl(z + eps) contains the
// double-precision value; when both ends round alike (the rounding is
// monotone) so does it.  Only when a value is that close to a rounding
// boundary is the double-precision pair evaluated.
template <int KIND>
__device__ __forceinline__ float rne_lp_f(float x) {
  if constexpr (KIND == 0) return rne_bf16_f(x);
  else return rne_e4m3_f(x);
}

template <int KIND>
__device__ __forceinline__ void omega_pair_rounded(uint64_t seed, uint32_t bkey, uint32_t i,
                                                   uint32_t q, float& o0, float& o1) {
  uint64_t a, b;
  omega_words(seed, bkey, i, q, a, b);
  float lnu;
  if (a >= 7ull * (1ull << 50)) {
    const float v = (float)((double)((1ull << 53) - 1u - a) * 0x1p-53);
    float p = 1.0f / 8.0f;
    p = __builtin_fmaf(p, v, 1.0f / 7.0f);
    p = __builtin_fmaf(p, v, 1.0f / 6.0f);
    p = __builtin_fmaf(p, v, 1.0f / 5.0f);
    p = __builtin_fmaf(p, v, 0.25f);
    p = __builtin_fmaf(p, v, 1.0f / 3.0f);
    p = __builtin_fmaf(p, v, 0.5f);
    p = __builtin_fmaf(p, v, 1.0f);
    lnu = -v * p;
  } else {
    lnu = __builtin_amdgcn_logf((float)((double)(a + 1u) * 0x1p-53)) * 0.693147180559945309f;
  }
  const float rho = sqrtf(-2.0f * lnu);
  const float u2 = (float)((double)b * 0x1p-53);
  const float z0 = rho * __builtin_amdgcn_cosf(u2);
  const float z1 = rho * __builtin_amdgcn_sinf(u2);
  const float eps = rho * 0x1p-19f + 0x1p-60f;
  const float r0 = rne_lp_f<KIND>(z0), r1 = rne_lp_f<KIND>(z1);
  if (rne_lp_f<KIND>(z0 - eps) == r0 && rne_lp_f<KIND>(z0 + eps) == r0 &&
      rne_lp_f<KIND>(z1 - eps) == r1 && rne_lp_f<KIND>(z1 + eps) == r1) {
    o0 = r0;
    o1 = r1;
    return;
  }
  const double2 z = box_muller_f64(a, b);
  if constexpr (KIND == 0) {
    o0 = (float)rne_bf16(z.x);
    o1 = (float)rne_bf16(z.y);
  } else {
    o0 = (float)rne_e4m3(z.x);
    o1 = (float)rne_e4m3(z.y);
  }
}

// bfloat16 bit pattern of a float (round to nearest even; exact when the
// float already has 8 significant bits).
__device__ __forceinline__ __bf16 to_bf16(float x) { return (__bf16)x; }

// Two floats rounded to nearest-even bfloat16, packed: x0 in bits 0-15, x1 in
// bits 16-31 (one v_cvt_pk_bf16_f32).
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16x2(float x0, float x1) {
  bf16x2 p;
  p[0] = (__bf16)x0;
  p[1] = (__bf16)x1;
  return __builtin_bit_cast(uint32_t, p);
}

// e4m3 byte of a float (hardware conversion, round to nearest even).
__device__ __forceinline__ uint32_t to_e4m3_byte(float x) {
  return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(x, 0.0f, 0, false) & 0xffu;
}

// Workgroup barrier that orders LDS only: waits for this wave's LDS accesses
// (lgkmcnt) and not for outstanding global loads, so prefetched A values stay
// in flight across it.  The "memory" clobber keeps the compiler from moving
// memory accesses across the barrier; register uses of in-flight loads still
// get their own vmcnt waits from the compiler.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// ---------------------------------------------------------------------------
// XCD-aware work-item order.  The hardware deals the workgroups of a launch to
// the 8 XCDs in turn (workgroup w to XCD w % 8), each XCD with its own L2.
// XCD x takes the contiguous items [start[x], start[x + 1]) in order (the host
// cuts the list into 8 ranges of about equal cost), so consecutive items that
// share data (the row ranges of one block, which share its coefficients) meet
// in one L2.  The grid is 8 * the longest range; -1 for the padding workgroups.
// ---------------------------------------------------------------------------
struct XcdSplit {
  int32_t start[9];
};

__device__ __forceinline__ int xcd_item(const XcdSplit& sp) {
  const int x = (int)(blockIdx.x & 7);
  const int it = sp.start[x] + (int)(blockIdx.x >> 3);
  return it < sp.start[x + 1] ? it : -1;
}

// ---------------------------------------------------------------------------
// Wave reductions (64 lanes, fixed butterfly order -> deterministic).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
  return v;
}

// (value, index) argmax: larger value wins, equal values -> lower index.
__device__ __forceinline__ void wave_argmax(double& v, int& idx) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double ov = __shfl_xor(v, off, kWave);
    const int oi = __shfl_xor(idx, off, kWave);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
}

// One exchange level of the same argmax by DPP lane moves within each row of
// 16 lanes (CTRL: the quad permutations, then the half-row and row mirrors).
// The operation (max, lowest index on equal values) is commutative,
// associative and idempotent, so after the four levels every lane of a row
// holds the row's argmax whatever the exchange pattern.
template <int CTRL>
__device__ __forceinline__ void argmax_dpp_level(double& v, int& idx) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, true);
  const int oi = __builtin_amdgcn_mov_dpp(idx, CTRL, 0xf, 0xf, true);
  const double ov = __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                                     (unsigned)lo));
  const bool take = (ov > v) | ((ov == v) & (oi < idx));
  v = take ? ov : v;
  idx = take ? oi : idx;
}

// The same argmax, made wave-uniform: the four DPP levels within each row of
// 16 lanes, then the four row results combined through lane reads (rows in
// ascending order) rather than lane-shuffle rounds through the LDS unit.
__device__ __forceinline__ void wave_argmax_uniform(double& v, int& idx) {
  argmax_dpp_level<0xB1>(v, idx);
  argmax_dpp_level<0x4E>(v, idx);
  argmax_dpp_level<0x141>(v, idx);
  argmax_dpp_level<0x140>(v, idx);
  const long long b = __double_as_longlong(v);
  double bv = v;
  int bi = idx;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int lo = __builtin_amdgcn_readlane((int)b, 16 * r);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 16 * r);
    const double ov = __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                                       (unsigned)lo));
    const int oi = __builtin_amdgcn_readlane(idx, 16 * r);
    if (r == 0) {
      bv = ov;
      bi = oi;
    } else {
      const bool take = (ov > bv) | ((ov == bv) & (oi < bi));
      bv = take ? ov : bv;
      bi = take ? oi : bi;
    }
  }
  v = bv;
  idx = bi;
}

// ---------------------------------------------------------------------------
// MFMA wrappers (gfx950).  Operand layouts (checked on the device):
//   f64 16x16x4 : A lane l -> (row l%16, k l/16); B lane l -> (k l/16, col l%16);
//                 D lane l slot v -> (row l/16 + 4v, col l%16).
//   bf16 16x16x32: A lane l slot v -> (row l%16, k 8(l/16)+v); B likewise with
//                 col l%16; D lane l slot v -> (row 4(l/16)+v, col l%16).
//   f8f6f4 16x16x128 (e4m3, E8M0 scales): A lane l byte v -> (row l%16,
//                 k 16(l/16)+v for v < 16, 64+16(l/16)+v-16 for v >= 16); B
//                 likewise with col l%16; the scale of K block kb (32 k-values)
//                 of row/column c comes from lane c+16kb; D as bf16.
// ---------------------------------------------------------------------------
__device__ __forceinline__ f64x4 mfma_f64(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f32x4 mfma_bf16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// e4m3 x e4m3 with per-lane E8M0 scales (byte 0 of the scale words).
__device__ __forceinline__ f32x4 mfma_fp8_scaled(i32x8 a, i32x8 b, f32x4 c, int sa, int sb) {
  return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 0, 0, 0, sa, 0, sb);
}

}  // namespace spid
