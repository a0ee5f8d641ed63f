// Device-side building blocks shared by the HIP kernels of the library:
// matrix-core engines, activation functions and FP64 kinematics.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pa {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

enum { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16 = 2, PREC_BF16C = 3 };

// ---------------------------------------------------------------------------
// Matrix-core engines.  One instruction multiplies a 16 x KS block of A by a
// KS x 16 block of B.  Lane l = j + 16*g holds operand elements with
// row/column l%16 and K indices g*KE .. g*KE+KE-1 (KE elements per lane).
// The 16x16 result sits in 4 registers per lane: column l%16, row
// ROW(g, v) for register v.  The FP64 instruction interleaves rows
// (row = g + 4v); the FP32 and BF16 instructions hold 4 consecutive rows
// (row = 4g + v).  Both were checked on gfx950.
// ---------------------------------------------------------------------------
struct EngF64 {
  using T = double;      // activation / stash type
  using acc = d4;
  using frag = double;   // one K element per lane
  static constexpr int KS = 4;
  static constexpr int KE = 1;
  __device__ static inline int row(int g, int v) { return g + 4 * v; }
  __device__ static inline acc mma(frag a, frag b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

struct EngF32 {
  using T = float;
  using acc = f4;
  using frag = float;
  static constexpr int KS = 4;
  static constexpr int KE = 1;
  __device__ static inline int row(int g, int v) { return 4 * g + v; }
  __device__ static inline acc mma(frag a, frag b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

struct EngBF16 {
  using T = float;
  using acc = f4;
  using frag = bf16x8;   // eight K elements per lane
  static constexpr int KS = 32;
  static constexpr int KE = 8;
  __device__ static inline int row(int g, int v) { return 4 * g + v; }
  __device__ static inline acc mma(frag a, frag b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

// ---------------------------------------------------------------------------
// Softplus and its derivatives, in forms that stay accurate for large |y|:
//   F(y)   = max(y, 0) + log(1 + e^{-|y|})
//   F'(y)  = sigma(y)
//   F''(y) = sigma(y) sigma(-y) = e^{-|y|} / (1 + e^{-|y|})^2
// ---------------------------------------------------------------------------
__device__ inline void softplus3(double y, double& f, double& f1, double& f2) {
  const double e = exp(-fabs(y));
  const double d = 1.0 + e;
  const double r = 1.0 / d;
  f = fmax(y, 0.0) + log1p(e);
  f1 = (y >= 0.0) ? r : e * r;
  f2 = e * r * r;
}
__device__ inline void softplus3(float y, float& f, float& f1, float& f2) {
  const float e = expf(-fabsf(y));
  const float d = 1.0f + e;
  const float r = 1.0f / d;
  f = fmaxf(y, 0.0f) + log1pf(e);
  f1 = (y >= 0.0f) ? r : e * r;
  f2 = e * r * r;
}

// Symmetric 3x3 tensors are stored as 6 tensor components in the order
// 11, 22, 33, 23, 13, 12.  VI(I, J) maps a pair of indices to that slot.
__device__ __host__ inline constexpr int VI(int I, int J) {
  return (I == J) ? I : (3 - I - J + 3);
}

}  // namespace pa
