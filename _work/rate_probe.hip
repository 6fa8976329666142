// Attainable-rate probe for MI355X (gfx950): the ceilings to compare the
// library's kernels with, measured with the library's own device helpers.
// Not part of the library; a stand-alone program:
//
//   paper_2103_01380_amd/rate_probe
//
// prints, one line each:
//   * FP64 MFMA (v_mfma_f64_16x16x4_f64) and BF16 MFMA
//     (v_mfma_f32_16x16x32_bf16) throughput of a loop that does nothing but
//     independent MFMAs from registers, at the FP64 sketch's workgroup shape
//     (8 waves) with 1 and 2 workgroups per compute unit;
//   * HBM read and copy bandwidth of plain streaming kernels (16-byte loads,
//     grid-stride, 4 GiB read / 2 GiB copied);
//   * the sketch matrix's generation rate (Philox4x32-10 + double-precision
//     Box-Muller pairs).
// Every buffer is sized to its grid; every index stays inside it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>

#include "spid_device.h"

using namespace spid;

#define CK(x)                                                                        \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess) {                                                          \
      fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
      exit(1);                                                                       \
    }                                                                                \
  } while (0)

constexpr int kThreads = 512;   // 8 waves per workgroup

// NACC independent accumulators per wave, `iters` rounds of NACC MFMAs.
template <int NACC>
__global__ __launch_bounds__(kThreads) void mfma_f64_loop(double* out, int iters, double a0) {
  f64x4 acc[NACC];
#pragma unroll
  for (int i = 0; i < NACC; ++i) acc[i] = f64x4{0.0, 0.0, 0.0, 0.0};
  const double a = a0 + threadIdx.x, b = a0 * 0.5;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < NACC; ++i) acc[i] = mfma_f64(a, b, acc[i]);
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NACC; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
  out[(size_t)blockIdx.x * kThreads + threadIdx.x] = s;
}

template <int NACC>
__global__ __launch_bounds__(kThreads) void mfma_bf16_loop(float* out, int iters, float a0) {
  f32x4 acc[NACC];
#pragma unroll
  for (int i = 0; i < NACC; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
  bf16x8 a, b;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    a[e] = (__bf16)(a0 + (float)e + (float)threadIdx.x);
    b[e] = (__bf16)(a0 * (float)e);
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < NACC; ++i) acc[i] = mfma_bf16(a, b, acc[i]);
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < NACC; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
  out[(size_t)blockIdx.x * kThreads + threadIdx.x] = s;
}

// Read n16 16-byte pieces once (grid-stride), one partial sum per thread.
__global__ __launch_bounds__(256) void stream_read(const f64x2* __restrict__ src, size_t n16,
                                                   double* __restrict__ part) {
  const size_t tid = (size_t)blockIdx.x * 256 + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * 256;
  double s = 0.0;
  for (size_t i = tid; i < n16; i += stride) {
    const f64x2 v = __builtin_nontemporal_load(src + i);
    s += v[0] + v[1];
  }
  part[tid] = s;
}

__global__ __launch_bounds__(256) void stream_copy(const f64x2* __restrict__ src, size_t n16,
                                                   f64x2* __restrict__ dst) {
  const size_t tid = (size_t)blockIdx.x * 256 + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * 256;
  for (size_t i = tid; i < n16; i += stride) dst[i] = __builtin_nontemporal_load(src + i);
}

__global__ __launch_bounds__(256) void omega_rate(double* out, int iters, uint64_t seed) {
  const uint32_t i0 = blockIdx.x * 256 + threadIdx.x;
  double s = 0.0;
  for (int it = 0; it < iters; ++it) {
    const double2 z = omega_pair(seed, 0u, i0, (uint32_t)it);
    s += z.x + z.y;
  }
  out[i0] = s;
}

__global__ __launch_bounds__(256) void fill(f64x2* p, size_t n16) {
  const size_t stride = (size_t)gridDim.x * 256;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += stride)
    p[i] = f64x2{1.0, (double)(i & 7)};
}

static float time_ms(hipEvent_t e0, hipEvent_t e1) {
  float ms = 0.f;
  CK(hipEventSynchronize(e1));
  CK(hipEventElapsedTime(&ms, e0, e1));
  return ms;
}

int main() {
  int dev = 0, ncu = 0;
  CK(hipGetDevice(&dev));
  CK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  const int max_wg = 2 * ncu;          // MFMA loops: up to 2 workgroups of 512 per CU
  const int og = 8 * ncu;              // generation: 8 workgroups of 256 per CU
  const size_t out_elems = std::max((size_t)max_wg * kThreads, (size_t)og * 256);
  double* out = nullptr;
  CK(hipMalloc(&out, sizeof(double) * out_elems));

  const int iters = 4000;
  for (int per_cu = 1; per_cu <= 2; ++per_cu) {
    const int g = per_cu * ncu;
    // FP64: 6 accumulators per wave (the FP64 sketch's 3 x 2 tiles) and 12
    hipLaunchKernelGGL(mfma_f64_loop<6>, dim3(g), dim3(kThreads), 0, 0, out, 8, 1.0);
    CK(hipEventRecord(e0));
    hipLaunchKernelGGL(mfma_f64_loop<6>, dim3(g), dim3(kThreads), 0, 0, out, iters, 1.0);
    CK(hipEventRecord(e1));
    double fl = 2.0 * 16 * 16 * 4 * 6.0 * iters * (kThreads / 64) * (double)g;
    printf("mfma_f64_16x16x4  %d workgroup(s) of 8 waves per CU,  6 acc/wave: %7.1f TFLOP/s\n",
           per_cu, fl / time_ms(e0, e1) / 1e9);
    CK(hipEventRecord(e0));
    hipLaunchKernelGGL(mfma_f64_loop<12>, dim3(g), dim3(kThreads), 0, 0, out, iters, 1.0);
    CK(hipEventRecord(e1));
    fl *= 2.0;
    printf("mfma_f64_16x16x4  %d workgroup(s) of 8 waves per CU, 12 acc/wave: %7.1f TFLOP/s\n",
           per_cu, fl / time_ms(e0, e1) / 1e9);
    hipLaunchKernelGGL(mfma_bf16_loop<6>, dim3(g), dim3(kThreads), 0, 0, (float*)out, 8, 1.0f);
    CK(hipEventRecord(e0));
    hipLaunchKernelGGL(mfma_bf16_loop<6>, dim3(g), dim3(kThreads), 0, 0, (float*)out, iters, 1.0f);
    CK(hipEventRecord(e1));
    fl = 2.0 * 16 * 16 * 32 * 6.0 * iters * (kThreads / 64) * (double)g;
    printf("mfma_bf16_16x16x32 %d workgroup(s) of 8 waves per CU,  6 acc/wave: %7.1f TFLOP/s\n",
           per_cu, fl / time_ms(e0, e1) / 1e9);
  }

  // HBM: 4 GiB read, 2 GiB copied into a second buffer
  const size_t bytes = (size_t)4 << 30;
  const size_t n16 = bytes / 16;
  f64x2 *src = nullptr, *dst = nullptr;
  CK(hipMalloc(&src, bytes));
  CK(hipMalloc(&dst, bytes / 2));
  const int sgrid = 8 * ncu * 8;   // 8 workgroups of 256 per CU x 8 passes
  double* part = nullptr;
  CK(hipMalloc(&part, sizeof(double) * (size_t)sgrid * 256));
  hipLaunchKernelGGL(fill, dim3(sgrid), dim3(256), 0, 0, src, n16);
  CK(hipDeviceSynchronize());
  for (int rep = 0; rep < 3; ++rep) {
    CK(hipEventRecord(e0));
    hipLaunchKernelGGL(stream_read, dim3(sgrid), dim3(256), 0, 0, src, n16, part);
    CK(hipEventRecord(e1));
    const float ms = time_ms(e0, e1);
    if (rep == 2) printf("HBM read  (4 GiB, 16-byte loads):           %7.1f GB/s\n", bytes / ms / 1e6);
  }
  for (int rep = 0; rep < 3; ++rep) {
    CK(hipEventRecord(e0));
    hipLaunchKernelGGL(stream_copy, dim3(sgrid), dim3(256), 0, 0, src, n16 / 2, dst);
    CK(hipEventRecord(e1));
    const float ms = time_ms(e0, e1);
    if (rep == 2)
      printf("HBM copy  (2 GiB read + 2 GiB written):      %7.1f GB/s\n", bytes / ms / 1e6);
  }

  // sketch-matrix generation: pairs per second over 2 workgroups of 256 per SIMD
  const int oiters = 200;
  hipLaunchKernelGGL(omega_rate, dim3(og), dim3(256), 0, 0, out, 2, 7ull);
  CK(hipEventRecord(e0));
  hipLaunchKernelGGL(omega_rate, dim3(og), dim3(256), 0, 0, out, oiters, 7ull);
  CK(hipEventRecord(e1));
  const double pairs = (double)oiters * 256 * og;
  printf("Omega pairs (Philox4x32-10 + FP64 Box-Muller): %7.1f G pairs/s\n",
         pairs / time_ms(e0, e1) / 1e6);

  CK(hipFree(part));
  CK(hipFree(dst));
  CK(hipFree(src));
  CK(hipFree(out));
  return 0;
}
