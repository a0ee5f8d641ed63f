// Measurement utility: do matrix-core and vector instructions of different
// waves overlap on one SIMD?  Eight waves per workgroup (two per SIMD):
// waves 0-3 run one kind of work, waves 4-7 another, each as independent
// dependency chains, so a pair's time against the two kinds alone shows
// whether the SIMD runs them concurrently (time near the larger) or in turn
// (time near the sum).
#include <hip/hip_runtime.h>

#include "pa_internal.h"

namespace pa {

// kinds: 0 idle, 1 FP64 16x16x4 MFMA, 2 FP32 16x16x4 MFMA, 3 FP64 FMA,
// 4 FP32 FMA, 5 32-bit integer multiply-add
__global__ void __launch_bounds__(512) k_pipe_probe(int kind_lo, int kind_hi, int iters, double* __restrict__ out) {
  const int w = threadIdx.x >> 6;
  const int kind = w < 4 ? kind_lo : kind_hi;
  double r = 0.0;
  if (kind == 1) {
    d4 a0 = {0, 0, 0, 0}, a1 = a0, a2 = a0, a3 = a0;
    const double x = threadIdx.x * 1e-3, y = 1.0 + threadIdx.x * 1e-4;
    for (int i = 0; i < iters; ++i) {
      a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, a0, 0, 0, 0);
      a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, a1, 0, 0, 0);
      a2 = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, a2, 0, 0, 0);
      a3 = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, a3, 0, 0, 0);
    }
    r = a0[0] + a1[1] + a2[2] + a3[3];
  } else if (kind == 2) {
    f4 a0 = {0, 0, 0, 0}, a1 = a0, a2 = a0, a3 = a0;
    const float x = threadIdx.x * 1e-3f, y = 1.0f + threadIdx.x * 1e-4f;
    for (int i = 0; i < 2 * iters; ++i) {
      a0 = __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, a0, 0, 0, 0);
      a1 = __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, a1, 0, 0, 0);
      a2 = __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, a2, 0, 0, 0);
      a3 = __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, a3, 0, 0, 0);
    }
    r = a0[0] + a1[1] + a2[2] + a3[3];
  } else if (kind == 3) {
    double v[8];
    for (int j = 0; j < 8; ++j) v[j] = threadIdx.x * 1e-3 + j;
    for (int i = 0; i < 4 * iters; ++i)
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = fma(v[j], 0.999999, 1e-7);
    for (int j = 0; j < 8; ++j) r += v[j];
  } else if (kind == 4) {
    float v[8];
    for (int j = 0; j < 8; ++j) v[j] = threadIdx.x * 1e-3f + j;
    for (int i = 0; i < 4 * iters; ++i)
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = fmaf(v[j], 0.999999f, 1e-7f);
    for (int j = 0; j < 8; ++j) r += v[j];
  } else if (kind == 5) {
    unsigned v[8];
    for (int j = 0; j < 8; ++j) v[j] = threadIdx.x + j;
    for (int i = 0; i < 4 * iters; ++i)
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = v[j] * 2654435761u + 12345u;
    for (int j = 0; j < 8; ++j) r += v[j];
  }
  out[(int64_t)blockIdx.x * 512 + threadIdx.x] = r;
}

int launch_pipe_probe(int kind_lo, int kind_hi, int iters, int blocks, double* out, hipStream_t s) {
  k_pipe_probe<<<blocks, 512, 0, s>>>(kind_lo, kind_hi, iters, out);
  return 0;
}

}  // namespace pa
