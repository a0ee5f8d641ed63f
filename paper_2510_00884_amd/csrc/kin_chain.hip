// Kernels for the FP64 kinematic layer (features, invariants) and the chain
// rule that turns network derivatives into P and dP/dF.  One quadrature
// point per lane; all per-point arrays are SoA ([component][n]) so every
// load and store is coalesced.
#include "kinematics.h"
#include "pa_internal.h"

namespace pa {


template <int NSV>
__global__ void __launch_bounds__(256) k_invariants(int64_t n, const double* __restrict__ F,
                                                    ModelConst mc, double* __restrict__ I_raw,
                                                    double* __restrict__ K, double* __restrict__ dKdF,
                                                    int32_t* n_bad) {
  constexpr int NP = Feat<NSV>::NP;
  constexpr int P = Feat<NSV>::P;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = t < n;
  double f[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) f[i] = in ? F[i * n + t] : (i % 4 == 0 ? 1.0 : 0.0);
  Kin k;
  kin_compute<NSV>(f, mc, k);
  count_bad(n_bad, in && !(k.J > 0.0 && finite9(f)));
  if (!in) return;
  if (I_raw) {
    I_raw[0 * n + t] = k.I1;
    I_raw[1 * n + t] = k.I2;
    I_raw[2 * n + t] = k.I3;
    I_raw[3 * n + t] = k.J;
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      I_raw[(4 + q) * n + t] = k.I4[q];
      I_raw[(4 + NP + q) * n + t] = k.I5[q];
    }
  }
  if (K) {
    double kf[P];
    kin_features<NSV>(k, mc, kf);
#pragma unroll
    for (int m = 0; m < P; ++m) K[m * n + t] = kf[m];
  }
  if (dKdF) {
#pragma unroll
    for (int m = 0; m < P; ++m) {
      double d[6];
      kin_dfeature<NSV>(k, mc, m, d);
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int J = 0; J < 3; ++J) {
          const double v = 2.0 * (k.F[3 * i] * d[VI(0, J)] + k.F[3 * i + 1] * d[VI(1, J)] + k.F[3 * i + 2] * d[VI(2, J)]);
          dKdF[((int64_t)m * 9 + 3 * i + J) * n + t] = v;
        }
    }
  }
}

// Network outputs in SoA: row 0 = N, rows 1..P = dN/dK_m, then the packed
// upper triangle of d2N/dK_m dK_n (row-major, m <= n).
// F and the outputs have leading dimension ld (>= n; a batch of a longer
// call), the network outputs n.
template <int NSV>
__global__ void __launch_bounds__(256) k_chain(int64_t n, int64_t ld, const double* __restrict__ F,
                                               const double* __restrict__ Nout, const double* __restrict__ N0,
                                               ModelConst mc, double* __restrict__ psi,
                                               double* __restrict__ Pout, double* __restrict__ Aout,
                                               int32_t* n_bad) {
  constexpr int P = Feat<NSV>::P;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  double f[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) f[i] = F[i * ld + t];
  Kin k;
  kin_compute<NSV>(f, mc, k);
  if (psi) psi[t] = Nout[t] - N0[0];
  if (!Pout && !Aout) return;
  const bool second = Aout != nullptr;
  auto N1 = [&](int m) { return Nout[(int64_t)(1 + m) * n + t]; };
  auto N2 = [&](int i) { return Nout[(int64_t)(1 + P + i) * n + t]; };
  double S[6], CCt[21];
  chain_material_stream<NSV>(k, mc, N1, N2, second, S, CCt);
  push_material(
      k, S, CCt,
      [&](int c, double v) { if (Pout) Pout[(int64_t)c * ld + t] = v; },
      [&](int c, double v) { if (Aout) Aout[(int64_t)c * ld + t] = v; });
  (void)n_bad;
}

// Psi, Kirchhoff stress tau [6][n] and spatial tangent cc [21][n] in Voigt
// slots (11, 22, 33, 23, 13, 12), the tangent as the upper triangle of the
// 6 x 6 matrix in TRI order: the paper's own storage of the constitutive
// update (App. A.1-A.2), 216 instead of 720 bytes per point.
template <int NSV>
__global__ void __launch_bounds__(256) k_chain_voigt(int64_t n, int64_t ld, const double* __restrict__ F,
                                                     const double* __restrict__ Nout, const double* __restrict__ N0,
                                                     ModelConst mc, double* __restrict__ psi,
                                                     double* __restrict__ tau, double* __restrict__ cc) {
  constexpr int P = Feat<NSV>::P;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  double f[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) f[i] = F[i * ld + t];
  Kin k;
  kin_compute<NSV>(f, mc, k);
  if (psi) psi[t] = Nout[t] - N0[0];
  if (!tau && !cc) return;
  const bool second = cc != nullptr;
  auto N1 = [&](int m) { return Nout[(int64_t)(1 + m) * n + t]; };
  auto N2 = [&](int i) { return Nout[(int64_t)(1 + P + i) * n + t]; };
  double S[6], CCt[21];
  chain_material_stream<NSV>(k, mc, N1, N2, second, S, CCt);
  push_spatial(
      k, S, CCt, second,
      [&](int c, double v) { if (tau) tau[(int64_t)c * ld + t] = v; },
      [&](int c, double v) { cc[(int64_t)c * ld + t] = v; });
}

// dPsi/dC (6 slots) and d2Psi/dCdC (21 upper-triangle tensor components) per
// point, SoA [27][n]: the material-form quantities the element kernels
// integrate.  Fully unrolled: the network derivatives are loaded once and the
// feature gradients stay in registers.  Launched in workgroups of 128 threads
// (two waves per SIMD either way; 3.5% faster than 256 on 2^21 points).
template <int NSV>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_material_cc(int64_t n, const double* __restrict__ F,
                                                     const double* __restrict__ Nout, ModelConst mc,
                                                     double* __restrict__ SC) {
  constexpr int P = Feat<NSV>::P;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  double f[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) f[i] = F[i * n + t];
  Kin k;
  kin_compute<NSV>(f, mc, k);
  auto N1 = [&](int m) { return Nout[(int64_t)(1 + m) * n + t]; };
  auto N2 = [&](int i) { return Nout[(int64_t)(1 + P + i) * n + t]; };
  double S[6], CCt[21];
  chain_material_stream<NSV>(k, mc, N1, N2, true, S, CCt);
#pragma unroll
  for (int c = 0; c < 6; ++c) SC[(int64_t)c * n + t] = S[c];
#pragma unroll
  for (int c = 0; c < 21; ++c) SC[(int64_t)(6 + c) * n + t] = CCt[c];
}

// Features only (input to the network kernels).
template <int NSV>
__global__ void __launch_bounds__(256) k_features(int64_t n, int64_t ld, const double* __restrict__ F, ModelConst mc,
                                                  double* __restrict__ K, int32_t* n_bad) {
  constexpr int P = Feat<NSV>::P;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = t < n;
  double f[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) f[i] = in ? F[i * ld + t] : (i % 4 == 0 ? 1.0 : 0.0);
  Kin k;
  kin_compute<NSV>(f, mc, k);
  count_bad(n_bad, in && !(k.J > 0.0 && finite9(f)));
  if (!in) return;
  double kf[P];
  kin_features<NSV>(k, mc, kf);
#pragma unroll
  for (int m = 0; m < P; ++m) K[m * n + t] = kf[m];
}

// ---------------------------------------------------------------- launchers
static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

int launch_invariants(int nsv, int64_t n, const double* F, const ModelConst& mc, double* I_raw,
                      double* K, double* dKdF, int32_t* n_bad, hipStream_t s) {
  if (n == 0) return 0;
  switch (nsv) {
    case 0: k_invariants<0><<<nblk(n, 256), 256, 0, s>>>(n, F, mc, I_raw, K, dKdF, n_bad); break;
    case 1: k_invariants<1><<<nblk(n, 256), 256, 0, s>>>(n, F, mc, I_raw, K, dKdF, n_bad); break;
    case 2: k_invariants<2><<<nblk(n, 256), 256, 0, s>>>(n, F, mc, I_raw, K, dKdF, n_bad); break;
    default: return -1;
  }
  return 0;
}

int launch_features(int nsv, int64_t n, int64_t ld, const double* F, const ModelConst& mc, double* K,
                    int32_t* n_bad, hipStream_t s) {
  if (n == 0) return 0;
  switch (nsv) {
    case 0: k_features<0><<<nblk(n, 256), 256, 0, s>>>(n, ld, F, mc, K, n_bad); break;
    case 1: k_features<1><<<nblk(n, 256), 256, 0, s>>>(n, ld, F, mc, K, n_bad); break;
    case 2: k_features<2><<<nblk(n, 256), 256, 0, s>>>(n, ld, F, mc, K, n_bad); break;
    default: return -1;
  }
  return 0;
}

int launch_material_cc(int nsv, int64_t n, const double* F, const double* Nout, const ModelConst& mc,
                       double* SC, hipStream_t s) {
  if (n == 0) return 0;
  switch (nsv) {
    case 0: k_material_cc<0><<<nblk(n, 128), 128, 0, s>>>(n, F, Nout, mc, SC); break;
    case 1: k_material_cc<1><<<nblk(n, 128), 128, 0, s>>>(n, F, Nout, mc, SC); break;
    case 2: k_material_cc<2><<<nblk(n, 128), 128, 0, s>>>(n, F, Nout, mc, SC); break;
    default: return -1;
  }
  return 0;
}

int launch_chain_voigt(int nsv, int64_t n, int64_t ld, const double* F, const double* Nout, const double* N0,
                       const ModelConst& mc, double* psi, double* tau, double* cc, hipStream_t s) {
  if (n == 0) return 0;
  switch (nsv) {
    case 0: k_chain_voigt<0><<<nblk(n, 256), 256, 0, s>>>(n, ld, F, Nout, N0, mc, psi, tau, cc); break;
    case 1: k_chain_voigt<1><<<nblk(n, 256), 256, 0, s>>>(n, ld, F, Nout, N0, mc, psi, tau, cc); break;
    case 2: k_chain_voigt<2><<<nblk(n, 256), 256, 0, s>>>(n, ld, F, Nout, N0, mc, psi, tau, cc); break;
    default: return -1;
  }
  return 0;
}

// k_chain in workgroups of 128 threads (2^21 points: 0.650 -> 0.614 ms against 256)
int launch_chain(int nsv, int64_t n, int64_t ld, const double* F, const double* Nout, const double* N0,
                 const ModelConst& mc, double* psi, double* P, double* A, int32_t* n_bad, hipStream_t s) {
  if (n == 0) return 0;
  switch (nsv) {
    case 0: k_chain<0><<<nblk(n, 128), 128, 0, s>>>(n, ld, F, Nout, N0, mc, psi, P, A, n_bad); break;
    case 1: k_chain<1><<<nblk(n, 128), 128, 0, s>>>(n, ld, F, Nout, N0, mc, psi, P, A, n_bad); break;
    case 2: k_chain<2><<<nblk(n, 128), 128, 0, s>>>(n, ld, F, Nout, N0, mc, psi, P, A, n_bad); break;
    default: return -1;
  }
  return 0;
}

}  // namespace pa
