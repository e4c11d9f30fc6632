// MFMA issue-rate probe for gfx950: the measured ceilings that the roofline
// fractions of the grouped kernels are read against.  Not part of the
// library; built and run on its own:
//   hipcc -O3 --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         paper_2008_03237_amd/csrc/mfma_rate_probe.hip -o /tmp/mfma_rate && /tmp/mfma_rate
// Each wave issues CH independent accumulation chains of one MFMA for ITERS
// iterations; occ workgroups of 4 waves per CU give occ waves per SIMD.  The
// second of two launches is timed with HIP events.
#include <hip/hip_runtime.h>
#include <cstdio>
typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
constexpr int ITERS = 4096, CH = 8;
__global__ __launch_bounds__(256) void k64(double* out, double a) {
  d4 c[CH]; for (int i = 0; i < CH; ++i) c[i] = d4{0,0,0,0};
  double b = a + threadIdx.x;
  for (int it = 0; it < ITERS; ++it)
#pragma unroll
    for (int i = 0; i < CH; ++i) c[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c[i], 0, 0, 0);
  double s = 0; for (int i = 0; i < CH; ++i) s += c[i][0] + c[i][3];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}
__global__ __launch_bounds__(256) void k32(double* out, float a) {
  f4 c[CH]; for (int i = 0; i < CH; ++i) c[i] = f4{0,0,0,0};
  float b = a + threadIdx.x;
  for (int it = 0; it < ITERS; ++it)
#pragma unroll
    for (int i = 0; i < CH; ++i) c[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c[i], 0, 0, 0);
  float s = 0; for (int i = 0; i < CH; ++i) s += c[i][0] + c[i][3];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}
__global__ __launch_bounds__(256) void kbf16(double* out, short a) {
  f4 c[CH]; for (int i = 0; i < CH; ++i) c[i] = f4{0,0,0,0};
  s4 av = {a, a, a, a}, bv = {(short)(a + threadIdx.x), a, a, a};
  for (int it = 0; it < ITERS; ++it)
#pragma unroll
    for (int i = 0; i < CH; ++i) c[i] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, c[i], 0, 0, 0);
  float s = 0; for (int i = 0; i < CH; ++i) s += c[i][0] + c[i][3];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}
__global__ __launch_bounds__(256) void kbf16x32(double* out, float a) {
  f4 c[CH]; for (int i = 0; i < CH; ++i) c[i] = f4{0,0,0,0};
  b8 av, bv; for (int j = 0; j < 8; ++j) { av[j] = (__bf16)a; bv[j] = (__bf16)(a + threadIdx.x); }
  for (int it = 0; it < ITERS; ++it)
#pragma unroll
    for (int i = 0; i < CH; ++i) c[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c[i], 0, 0, 0);
  float s = 0; for (int i = 0; i < CH; ++i) s += c[i][0] + c[i][3];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}
__global__ __launch_bounds__(256) void k64s(double* out, double a) {
  double c[CH]; for (int i = 0; i < CH; ++i) c[i] = 0.0;
  double b = a + threadIdx.x;
  for (int it = 0; it < ITERS; ++it)
#pragma unroll
    for (int i = 0; i < CH; ++i) c[i] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c[i], 0, 0, 0);
  double s = 0; for (int i = 0; i < CH; ++i) s += c[i];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}
int main() {
  int cu; (void)hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, 0);
  int clk; (void)hipDeviceGetAttribute(&clk, hipDeviceAttributeClockRate, 0);
  double* out; (void)hipMalloc(&out, (size_t)cu * 4 * 256 * sizeof(double));   // grid <= 4 cu
  for (int occ = 1; occ <= 4; ++occ) {
  const int grid = cu * occ;   // occ WGs (4 waves each) per CU
  hipEvent_t e0, e1; (void)hipEventCreate(&e0); (void)hipEventCreate(&e1);
  const char* names[5] = {"f64 16x16x4", "f32 16x16x4", "bf16 16x16x16", "bf16 16x16x32", "f64 4x4x4_4b"};
  const double flops[5] = {2048, 2048, 8192, 16384, 512};
  for (int w = 0; w < 5; ++w) {
    for (int rep = 0; rep < 2; ++rep) {
      (void)hipEventRecord(e0);
      if (w == 0) hipLaunchKernelGGL(k64, dim3(grid), dim3(256), 0, 0, out, 1.0);
      if (w == 1) hipLaunchKernelGGL(k32, dim3(grid), dim3(256), 0, 0, out, 1.0f);
      if (w == 2) hipLaunchKernelGGL(kbf16, dim3(grid), dim3(256), 0, 0, out, (short)0x3f80);
      if (w == 3) hipLaunchKernelGGL(kbf16x32, dim3(grid), dim3(256), 0, 0, out, 1.0f);
      if (w == 4) hipLaunchKernelGGL(k64s, dim3(grid), dim3(256), 0, 0, out, 1.0);
      (void)hipEventRecord(e1); (void)hipEventSynchronize(e1);
      float ms; (void)hipEventElapsedTime(&ms, e0, e1);
      const double n_mfma = (double)grid * 4 * ITERS * CH;   // per wave
      if (rep == 1)
        printf("occ %d %-16s %.3f ms  %.1f TFLOP/s  %.1f cycles/MFMA/SIMD at %.0f MHz (CUs %d)\n", occ, names[w], ms,
               n_mfma * flops[w] / (ms * 1e-3) / 1e12, (ms * 1e-3) * clk * 1e3 / (ITERS * CH * occ), clk / 1e3, cu);
    }
  }
  }
  return 0;
}
