// Device-side building blocks shared by the HIP kernels of the library:
// matrix-core engines, activation functions and FP64 kinematics.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pa {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Network-contraction precisions (the values of pa_precision): FP64, FP32,
// all-BF16, all-BF16 followed by an FP32 pass over the value and gradient,
// and the one-pass mixed form (FP32 value, gradient and reverse sweep, BF16
// Jacobians of layers >= 2).
enum { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16 = 2, PREC_BF16C = 3, PREC_BF16J = 4 };

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
// a / d for d in [1, 3]: hardware reciprocal estimate, two Newton steps and
// a residual correction of the quotient (no range scaling is needed).
__device__ inline double div_unit(double a, double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(fma(-d, r, 1.0), r, r);
  r = fma(fma(-d, r, 1.0), r, r);
  const double q = a * r;
  return fma(fma(-d, q, a), r, q);
}

// log(1 + x) for x in [0, 1] (here x = e^{-|y|}).  For x above sqrt(2) - 1,
// log(1 + x) = ln 2 + log(1 + g) with g = (x - 1)/2 in (-0.293, 0]; then
// log(1 + g) = 2 atanh(s), s = g / (2 + g), |s| <= 0.1716, summed as the odd
// series 2 s sum_k s^{2k} / (2k + 1).  Terms to k = 9 leave a truncation
// below half an ulp.
__device__ inline double log1p_unit(double x) {
  const bool hi = x > 0.41421356237309503;
  const double g = hi ? 0.5 * (x - 1.0) : x;
  const double s = div_unit(g, 2.0 + g);
  const double s2 = s * s;
  double p = 1.0 / 19.0;
  p = fma(p, s2, 1.0 / 17.0);
  p = fma(p, s2, 1.0 / 15.0);
  p = fma(p, s2, 1.0 / 13.0);
  p = fma(p, s2, 1.0 / 11.0);
  p = fma(p, s2, 1.0 / 9.0);
  p = fma(p, s2, 1.0 / 7.0);
  p = fma(p, s2, 1.0 / 5.0);
  p = fma(p, s2, 1.0 / 3.0);
  const double t = 2.0 * s;
  const double r = fma(t * s2, p, t);
  return hi ? 0.6931471805599453 + r : r;
}

__device__ inline void softplus3(double y, double& f, double& f1, double& f2) {
  const double e = exp(-fabs(y));
  const double r = div_unit(1.0, 1.0 + e);
  f = fmax(y, 0.0) + log1p_unit(e);
  f1 = (y >= 0.0) ? r : e * r;
  f2 = e * r * r;
}
// FP32 on the hardware base-2 exponential and logarithm (each within about
// two units of 2^-24 relative, checked on gfx950 over their whole range here,
// the logarithm also just above 1):
//   e^{-t} = 2^a 2^da with a = -t log2 e rounded, da its rounding error (one
//   fused multiply-add) plus t times the low part of log2 e, applied to first
//   order (|da| < 1e-5 for t < 128, where e^{-t} still has FP32 digits);
//   log(1 + e) = log(u) + (1 + e - u)/u for the rounded u = 1 + e, whose
//   rounding error 1 + e - u = e - (u - 1) is exact.
// Measured against FP64 over |y| <= 110: F within 3.6, F' within 4.0 and F''
// within 6.1 units of 2^-24 relative.  y = NaN gives NaN outputs.
__device__ inline void softplus3(float y, float& f, float& f1, float& f2) {
  const float t = fabsf(y);
  const float a = -t * 1.44269502f;
  float da = fmaf(-t, 1.44269502f, -a) - t * 1.925963e-8f;
  da = (t < 128.0f) ? da : 0.0f;  // infinite t: e = 0 without a NaN correction
  const float p = __builtin_amdgcn_exp2f(a);
  const float e = fmaf(p * da, 0.693147182f, p);
  const float u = 1.0f + e;
  float r = __builtin_amdgcn_rcpf(u);
  r = fmaf(fmaf(-u, r, 1.0f), r, r);
  f = fmaxf(y, 0.0f) + fmaf(__builtin_amdgcn_logf(u), 0.693147182f, (e - (u - 1.0f)) * r);
  f1 = (y >= 0.0f) ? r : e * r;
  f2 = e * r * r;
}

// FP64 softplus with two 64-entry tables, for kernels that fill them once
// per workgroup (in LDS) and evaluate many activations:
//   e^{-t} = 2^{-N/64} e^{-r},  N = rint(64 t / ln 2),  |r| <= ln 2 / 128,
// with 2^{-j/64} from the table and e^{-r} from its Taylor polynomial to r^5
// (first dropped term below 4e-17 relative); the reduction t - N ln2/64 is
// exact in its first fused step (|r| < 2^-7) and adds the low part of ln2/64
// in a second.  With j = floor(64 e) (0 .. 64, e <= 1) and a reciprocal w_j of
// the centre of the j-th 64th of [1, 2 + 1/64] (w_0 = 1),
//   log(1 + e) = -log w_j + log(1 + d),  d = (1 + e) w_j - 1 = e w_j + (w_j - 1),
// where d comes from one fused multiply-add of exact operands (w_j - 1 is
// exact), so it is correctly rounded for any stored w_j, and |d| < 1/64;
// log(1 + d) from its series to d^9 (relative truncation below 1e-17).
// F keeps its relative accuracy for large negative y (then j = 0, d = e).
struct SpTab {
  double e[64];   // 2^{-j/64}
  double2 l[65];  // {w_j, -log w_j}
};
__device__ inline void softplus_tab_fill(SpTab& T, int tid, int nthreads) {
  for (int j = tid; j < 65; j += nthreads) {
    if (j < 64) T.e[j] = exp2(-(double)j / 64.0);
    const double w = (j == 0) ? 1.0 : 1.0 / (1.0 + ((double)j + 0.5) / 64.0);
    T.l[j] = make_double2(w, -log(w));
  }
}
__device__ inline void softplus3(double y, double& f, double& f1, double& f2, const SpTab& T) {
  const double t = fmin(fabs(y), 745.5);  // e^{-745.5} is below half the smallest subnormal
  const double kd = __builtin_rint(t * 92.33248261689366);  // 64 / ln 2
  const int N = (int)kd;
  double r = fma(-kd, 0x1.62e42fefa39efp-7, t);
  r = fma(-kd, 0x1.abc9e3b39803fp-62, r);
  const double x = -r;
  double p = 1.0 / 120.0;
  p = fma(p, x, 1.0 / 24.0);
  p = fma(p, x, 1.0 / 6.0);
  p = fma(p, x, 0.5);
  p = fma(p, x, 1.0);
  p = fma(p, x, 1.0);
  const double e = __builtin_ldexp(T.e[N & 63] * p, -(N >> 6));
  const double u = 1.0 + e;
  double rc = __builtin_amdgcn_rcp(u);
  rc = fma(fma(-u, rc, 1.0), rc, rc);
  rc = fma(fma(-u, rc, 1.0), rc, rc);
  const double2 lw = T.l[(int)(e * 64.0)];
  const double d = fma(e, lw.x, lw.x - 1.0);
  double q = 1.0 / 9.0;
  q = fma(q, d, -0.125);
  q = fma(q, d, 1.0 / 7.0);
  q = fma(q, d, -1.0 / 6.0);
  q = fma(q, d, 0.2);
  q = fma(q, d, -0.25);
  q = fma(q, d, 1.0 / 3.0);
  q = fma(q, d, -0.5);
  q = fma(q, d, 1.0);
  f = fmax(y, 0.0) + fma(q, d, lw.y);
  f1 = (y >= 0.0) ? rc : e * rc;
  f2 = e * rc * rc;
}

// FP32 kernels share the call sites of the tabled FP64 form (no table).
__device__ inline void softplus3(float y, float& f, float& f1, float& f2, const SpTab&) { softplus3(y, f, f1, f2); }

// Symmetric 3x3 tensors are stored as 6 tensor components in the order
// 11, 22, 33, 23, 13, 12.  VI(I, J) maps a pair of indices to that slot.
__device__ __host__ inline constexpr int VI(int I, int J) {
  return (I == J) ? I : (3 - I - J + 3);
}

}  // namespace pa
