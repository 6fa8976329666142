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
    const uint32_t p0_hi = __umulhi(0xD2511F53u, c.x);
    const uint32_t p0_lo = 0xD2511F53u * c.x;
    const uint32_t p1_hi = __umulhi(0xCD9E8D57u, c.z);
    const uint32_t p1_lo = 0xCD9E8D57u * c.z;
    c = make_uint4(p1_hi ^ c.y ^ k0, p1_lo, p0_hi ^ c.w ^ k1, p0_lo);
  }
  return c;
}

// Sketch-matrix entries Omega(2q, i) and Omega(2q+1, i): one Philox block at
// counter (i, q, block key, stream 0) under the 64-bit seed, two 53-bit
// uniforms (u1 in (0,1], u2 in [0,1)), Box-Muller in double precision.
__device__ __forceinline__ void omega_words(uint64_t seed, uint32_t bkey, uint32_t i, uint32_t q,
                                            uint64_t& a, uint64_t& b) {
  const uint4 x = philox4x32_10(make_uint4(i, q, bkey, 0u), (uint32_t)seed,
                                (uint32_t)(seed >> 32));
  a = ((uint64_t)(x.x >> 5) << 26) | (uint64_t)(x.y >> 6);
  b = ((uint64_t)(x.z >> 5) << 26) | (uint64_t)(x.w >> 6);
}

__device__ __forceinline__ double2 box_muller_f64(uint64_t a, uint64_t b) {
  const double u1 = (double)(a + 1u) * 0x1p-53;
  const double u2 = (double)b * 0x1p-53;
  const double rho = sqrt(-2.0 * log(u1));
  double s, c;
  sincos(6.283185307179586 * u2, &s, &c);
  return make_double2(rho * c, rho * s);
}

__device__ __forceinline__ double2 omega_pair(uint64_t seed, uint32_t bkey, uint32_t i,
                                              uint32_t q) {
  uint64_t a, b;
  omega_words(seed, bkey, i, q, a, b);
  return box_muller_f64(a, b);
}

// The same pair rounded by `rnd` (round-to-nearest-even to bfloat16 or e4m3,
// a monotone map) for the low-precision sketches, evaluated cheaply but with
// the same result.  Box-Muller first runs in single precision: u1 -> ln u1
// (log1p of the exact complement when u1 > 1/2), rho = sqrt(-2 ln u1), the
// angle as sincospi(2 u2).  Error of z = rho (cos, sin) against the
// double-precision evaluation: u2 rounded to single (angle error <= 1.9e-7),
// sincospi (<= 2.4e-7), ln and sqrt (rho relative error <= 2.7e-7), product
// rounding (6e-8 relative): |dz| <= 7.6e-7 rho.  With eps = rho 2^-19
// (1.9e-6 rho) every value within eps of the single-precision z rounds alike
// when z - eps and z + eps do (the map is monotone), so the double-precision
// pair lies in that interval and rounds to the same value.  Only when a value
// is that close to a rounding boundary is the double-precision pair evaluated.
template <typename RND>
__device__ __forceinline__ void omega_pair_rounded(uint64_t seed, uint32_t bkey, uint32_t i,
                                                   uint32_t q, RND rnd, double& o0, double& o1) {
  uint64_t a, b;
  omega_words(seed, bkey, i, q, a, b);
  float lnu;
  if (a >= (1ull << 52)) {
    const float v = (float)((1ull << 53) - 1u - a) * 0x1p-53f;
    lnu = log1pf(-v);
  } else {
    lnu = logf((float)(a + 1u) * 0x1p-53f);
  }
  const float rho = sqrtf(-2.0f * lnu);
  float sn, cs;
  sincospif(2.0f * ((float)b * 0x1p-53f), &sn, &cs);
  const double z0 = (double)(rho * cs), z1 = (double)(rho * sn);
  const double eps = (double)rho * 0x1p-19 + 0x1p-60;
  const double r0 = rnd(z0), r1 = rnd(z1);
  if (rnd(z0 - eps) == r0 && rnd(z0 + eps) == r0 && rnd(z1 - eps) == r1 && rnd(z1 + eps) == r1) {
    o0 = r0;
    o1 = r1;
    return;
  }
  const double2 z = box_muller_f64(a, b);
  o0 = rnd(z.x);
  o1 = rnd(z.y);
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

// bfloat16 bit pattern of a float (round to nearest even; exact when the
// float already has 8 significant bits).
__device__ __forceinline__ __bf16 to_bf16(float x) { return (__bf16)x; }

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
