// FP64 kinematic layer and chain rule, evaluated per quadrature point in
// registers.
//
// Kinematic layer (App. A.2.1-A.2.2, App. C): C = F^T F, I1 = tr C,
// I2 = (I1^2 - C:C)/2, I3 = det C = J^2, I4_ij = A^i.C A^j,
// I5_ij = A^i.C^2 A^j; isochoric I~ = I * I3^alpha (alpha = -1/3 for I1, I4;
// -2/3 for I2, I5); features
//   K = [I1~ - 3, I2~^{3/2} - 3^{3/2}, (J-1)^2, I4~_ij - A^i.A^j, I5~_ij - A^i.A^j].
//
// Chain rule (eq. nncm-chain) in material (C-space) form: with d_m = dK_m/dC
// and the network derivatives N_m, N_mn,
//   S~ = sum_m N_m d_m,   CC~ = sum_mn N_mn d_m (x) d_n + sum_m N_m d2K_m/dCdC,
//   P = 2 F S~,   AA_iJkL = 2 delta_ik S~_JL + 4 F_iI F_kK CC~_IJKL
// (eq. p-stiffness).  The second derivatives of the isochoric features are
// written out as sums of the tensors I(x)I, I[x]I, c(x)c, c[x]c (c = C^{-1}),
// symmetric outer products and the I5 term A.(XY + YX)B.
//
// J - 1 is formed without cancellation from H = F - I:
//   J - 1 = tr H + (tr^2 H - tr H^2)/2 + det H.
#pragma once

#include "pa_device.h"

namespace pa {

// Wave-aggregated increment of an optional device counter.
__device__ inline void count_bad(int32_t* n_bad, bool bad) {
  if (!n_bad) return;
  const unsigned long long m = __ballot(bad);
  if (m && (threadIdx.x & 63) == (__ffsll((long long)m) - 1)) atomicAdd(n_bad, (int32_t)__popcll(m));
}

__device__ inline bool finite9(const double* F) {
  bool ok = true;
#pragma unroll
  for (int i = 0; i < 9; ++i) ok = ok && isfinite(F[i]);
  return ok;
}

struct ModelConst {
  double A[2][3];      // structural vectors A^1, A^2
  double AdotA[3];     // A^i . A^j for the pairs below
};

// Unordered pairs (i, j), i <= j, of structural vectors in row-major order.
__device__ __host__ constexpr int pair_i(int q, int nsv) {
  int c = 0;
  for (int i = 0; i < nsv; ++i)
    for (int j = i; j < nsv; ++j) {
      if (c == q) return i;
      ++c;
    }
  return 0;
}
__device__ __host__ constexpr int pair_j(int q, int nsv) {
  int c = 0;
  for (int i = 0; i < nsv; ++i)
    for (int j = i; j < nsv; ++j) {
      if (c == q) return j;
      ++c;
    }
  return 0;
}
template <int NSV>
struct Feat {
  static constexpr int NP = NSV * (NSV + 1) / 2;
  static constexpr int P = 3 + 2 * NP;
};

struct Kin {
  double F[9];
  double C[6];
  double c[6];   // C^{-1}
  double I1, I2, I3, J, Jm1, p13, p23;
  double CA[2][3];
  double I4[3], I5[3];
};

template <int NSV>
__host__ __device__ inline void kin_compute(const double* __restrict__ Fin, const ModelConst& mc, Kin& k) {
  constexpr int NP = Feat<NSV>::NP;
  double* F = k.F;
#pragma unroll
  for (int i = 0; i < 9; ++i) F[i] = Fin[i];
  const double H0 = F[0] - 1.0, H4 = F[4] - 1.0, H8 = F[8] - 1.0;
  const double H1 = F[1], H2 = F[2], H3 = F[3], H5 = F[5], H6 = F[6], H7 = F[7];
  const double trH = H0 + H4 + H8;
  const double trH2 = H0 * H0 + H4 * H4 + H8 * H8 + 2.0 * (H1 * H3 + H2 * H6 + H5 * H7);
  const double detH = H0 * (H4 * H8 - H5 * H7) - H1 * (H3 * H8 - H5 * H6) + H2 * (H3 * H7 - H4 * H6);
  k.Jm1 = trH + 0.5 * (trH * trH - trH2) + detH;
  k.J = 1.0 + k.Jm1;
  double* C = k.C;
  C[0] = F[0] * F[0] + F[3] * F[3] + F[6] * F[6];
  C[1] = F[1] * F[1] + F[4] * F[4] + F[7] * F[7];
  C[2] = F[2] * F[2] + F[5] * F[5] + F[8] * F[8];
  C[3] = F[1] * F[2] + F[4] * F[5] + F[7] * F[8];
  C[4] = F[0] * F[2] + F[3] * F[5] + F[6] * F[8];
  C[5] = F[0] * F[1] + F[3] * F[4] + F[6] * F[7];
  k.I1 = C[0] + C[1] + C[2];
  const double CC = C[0] * C[0] + C[1] * C[1] + C[2] * C[2] + 2.0 * (C[3] * C[3] + C[4] * C[4] + C[5] * C[5]);
  k.I2 = 0.5 * (k.I1 * k.I1 - CC);
  k.I3 = k.J * k.J;
  const double r3 = 1.0 / k.I3;
  k.c[0] = (C[1] * C[2] - C[3] * C[3]) * r3;
  k.c[1] = (C[0] * C[2] - C[4] * C[4]) * r3;
  k.c[2] = (C[0] * C[1] - C[5] * C[5]) * r3;
  k.c[3] = (C[4] * C[5] - C[0] * C[3]) * r3;
  k.c[4] = (C[5] * C[3] - C[1] * C[4]) * r3;
  k.c[5] = (C[4] * C[3] - C[2] * C[5]) * r3;
  const double cr = cbrt(k.J);
  k.p13 = 1.0 / (cr * cr);  // I3^{-1/3} = |J|^{-2/3}
  k.p23 = k.p13 * k.p13;
#pragma unroll
  for (int i = 0; i < NSV; ++i) {
    const double a0 = mc.A[i][0], a1 = mc.A[i][1], a2 = mc.A[i][2];
    k.CA[i][0] = C[0] * a0 + C[5] * a1 + C[4] * a2;
    k.CA[i][1] = C[5] * a0 + C[1] * a1 + C[3] * a2;
    k.CA[i][2] = C[4] * a0 + C[3] * a1 + C[2] * a2;
  }
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    const int i = pair_i(q, NSV), j = pair_j(q, NSV);
    k.I4[q] = mc.A[i][0] * k.CA[j][0] + mc.A[i][1] * k.CA[j][1] + mc.A[i][2] * k.CA[j][2];
    k.I5[q] = k.CA[i][0] * k.CA[j][0] + k.CA[i][1] * k.CA[j][1] + k.CA[i][2] * k.CA[j][2];
  }
}

template <int NSV>
__host__ __device__ inline void kin_features(const Kin& k, const ModelConst& mc, double* K) {
  constexpr int NP = Feat<NSV>::NP;
  const double I2t = k.I2 * k.p23;
  K[0] = k.I1 * k.p13 - 3.0;
  K[1] = I2t * sqrt(I2t) - 5.196152422706632;  // 3^{3/2}
  K[2] = k.Jm1 * k.Jm1;
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    K[3 + q] = k.I4[q] * k.p13 - mc.AdotA[q];
    K[3 + NP + q] = k.I5[q] * k.p23 - mc.AdotA[q];
  }
}

// dK_m/dC as a symmetric tensor (6 slots) for feature m.
template <int NSV>
__host__ __device__ inline void kin_dfeature(const Kin& k, const ModelConst& mc, int m, double* d) {
  constexpr int NP = Feat<NSV>::NP;
  const double* c = k.c;
  if (m == 0) {
    const double s = -k.I1 / 3.0;
#pragma unroll
    for (int a = 0; a < 6; ++a) d[a] = k.p13 * ((a < 3 ? 1.0 : 0.0) + s * c[a]);
  } else if (m == 1) {
    const double I2t = k.I2 * k.p23;
    const double f1 = 1.5 * sqrt(I2t);
    const double s = -2.0 * k.I2 / 3.0;
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      const double dI2 = (a < 3 ? k.I1 : 0.0) - k.C[a];
      d[a] = f1 * k.p23 * (dI2 + s * c[a]);
    }
  } else if (m == 2) {
    const double s = k.Jm1 * k.J;
#pragma unroll
    for (int a = 0; a < 6; ++a) d[a] = s * c[a];
  } else {
    const int t = m - 3;
    const bool five = t >= NP;
    const int q = five ? t - NP : t;
    const int i = pair_i(q, NSV), j = pair_j(q, NSV);
    const double* Ai = mc.A[i];
    const double* Aj = mc.A[j];
    double M[6];
    // M = sym(A^i (x) A^j) (I4) or sym(A^i (x) C A^j + C A^i (x) A^j) (I5)
    const double* X = Ai;
    const double* Y = five ? k.CA[j] : Aj;
    M[0] = X[0] * Y[0]; M[1] = X[1] * Y[1]; M[2] = X[2] * Y[2];
    M[3] = 0.5 * (X[1] * Y[2] + X[2] * Y[1]);
    M[4] = 0.5 * (X[0] * Y[2] + X[2] * Y[0]);
    M[5] = 0.5 * (X[0] * Y[1] + X[1] * Y[0]);
    if (five) {
      const double* U = k.CA[i];
      const double* V = Aj;
      M[0] += U[0] * V[0]; M[1] += U[1] * V[1]; M[2] += U[2] * V[2];
      M[3] += 0.5 * (U[1] * V[2] + U[2] * V[1]);
      M[4] += 0.5 * (U[0] * V[2] + U[2] * V[0]);
      M[5] += 0.5 * (U[0] * V[1] + U[1] * V[0]);
    }
    const double pw = five ? k.p23 : k.p13;
    const double s = five ? (-2.0 / 3.0) * k.I5[q] : (-1.0 / 3.0) * k.I4[q];
#pragma unroll
    for (int a = 0; a < 6; ++a) d[a] = pw * (M[a] + s * c[a]);
  }
}

// Index of the upper-triangular 6x6 entry (a <= b).
__device__ __host__ inline constexpr int TRI(int a, int b) {
  return (a <= b) ? (a * 6 - a * (a - 1) / 2 + (b - a)) : (b * 6 - b * (b - 1) / 2 + (a - b));
}

// Pair (I,J) of tensor indices for each of the 6 symmetric slots.
__host__ __device__ inline void slot_pair(int a, int& I, int& J) {
  const int tI[6] = {0, 1, 2, 1, 0, 0};
  const int tJ[6] = {0, 1, 2, 2, 2, 1};
  I = tI[a];
  J = tJ[a];
}

template <int NSV>
__host__ __device__ inline void chain_first_order(const Kin& k, const ModelConst& mc, const double* dN,
                                                  double* CCt);

// Chain rule: given dN (p), d2N (p(p+1)/2 packed row-major upper), compute
// S~ (6) and CC~ (21, upper triangle of the 6x6 in tensor components).
template <int NSV>
__host__ __device__ inline void chain_material(const Kin& k, const ModelConst& mc, const double* dN,
                                      const double* d2N, double* S, double* CCt) {
  constexpr int P = Feat<NSV>::P;
  double D[P][6];
#pragma unroll
  for (int m = 0; m < P; ++m) kin_dfeature<NSV>(k, mc, m, D[m]);
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < P; ++m) s += dN[m] * D[m][a];
    S[a] = s;
  }
#pragma unroll
  for (int t = 0; t < 21; ++t) CCt[t] = 0.0;
  // sum_mn N_mn d_m (x) d_n = sum_m d_m (x) V_m,  V_m = sum_n N_mn d_n
#pragma unroll
  for (int m = 0; m < P; ++m) {
    double V[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int n = 0; n < P; ++n) {
      const int mm = m < n ? m : n, nn = m < n ? n : m;
      const double w = d2N[mm * P - mm * (mm - 1) / 2 + (nn - mm)];
#pragma unroll
      for (int a = 0; a < 6; ++a) V[a] += w * D[n][a];
    }
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
      for (int b = a; b < 6; ++b) CCt[TRI(a, b)] += D[m][a] * V[b];
  }
  chain_first_order<NSV>(k, mc, dN, CCt);
}

// Adds sum_m N_m d2K_m/dCdC to CCt (upper triangle, tensor components).
template <int NSV>
__host__ __device__ inline void chain_first_order(const Kin& k, const ModelConst& mc, const double* dN,
                                                  double* CCt) {
  // second derivatives of the features, weighted by N_m
  const double* c = k.c;
  constexpr int np = Feat<NSV>::NP;
  const double I2t = k.I2 * k.p23;
  const double sq = sqrt(I2t);
  const double f1_2 = 1.5 * sq, f2_2 = 0.75 / sq;
  const double w1 = dN[0] * k.p13;            // K1: N_1 * I3^{-1/3}
  const double w2 = dN[1] * f1_2 * k.p23;     // K2: N_2 f' I3^{-2/3}
  const double w3 = dN[2];
  double U[6], dI2t[6];
  double kcc = (1.0 / 9.0) * w1 * k.I1 + (4.0 / 9.0) * w2 * k.I2 + w3 * (0.5 * k.Jm1 * k.J + 0.5 * k.J * k.J);
  double kbox = (1.0 / 3.0) * w1 * k.I1 + (2.0 / 3.0) * w2 * k.I2 - w3 * k.Jm1 * k.J;
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    const double id = a < 3 ? 1.0 : 0.0;
    const double dI2 = id * k.I1 - k.C[a];
    U[a] = (-1.0 / 3.0) * w1 * id + (-2.0 / 3.0) * w2 * dI2;
    dI2t[a] = k.p23 * (dI2 - (2.0 / 3.0) * k.I2 * c[a]);
  }
#pragma unroll
  for (int q = 0; q < np; ++q) {
    const int i = pair_i(q, NSV), j = pair_j(q, NSV);
    const double w4 = dN[3 + q] * k.p13;
    const double w5 = dN[3 + np + q] * k.p23;
    kcc += (1.0 / 9.0) * w4 * k.I4[q] + (4.0 / 9.0) * w5 * k.I5[q];
    kbox += (1.0 / 3.0) * w4 * k.I4[q] + (2.0 / 3.0) * w5 * k.I5[q];
    const double* Ai = mc.A[i];
    const double* Aj = mc.A[j];
    const double* CAi = k.CA[i];
    const double* CAj = k.CA[j];
    // U += -1/3 w4 sym(Ai Aj) - 2/3 w5 sym(Ai CAj + CAi Aj)
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      int I, J;
      slot_pair(a, I, J);
      const double M4 = 0.5 * (Ai[I] * Aj[J] + Ai[J] * Aj[I]);
      const double M5 = 0.5 * (Ai[I] * CAj[J] + Ai[J] * CAj[I] + CAi[I] * Aj[J] + CAi[J] * Aj[I]);
      U[a] += (-1.0 / 3.0) * w4 * M4 + (-2.0 / 3.0) * w5 * M5;
    }
    // w5 * d2 I5 / dC dC:  sym_IJ sym_KL [A_I B_L d_JK + A_L B_J d_IK]
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      int I, J;
      slot_pair(a, I, J);
#pragma unroll
      for (int b = a; b < 6; ++b) {
        int K, L;
        slot_pair(b, K, L);
        const double e =
            (Ai[I] * Aj[L] * (J == K) + Ai[L] * Aj[J] * (I == K) + Ai[J] * Aj[L] * (I == K) +
             Ai[L] * Aj[I] * (J == K) + Ai[I] * Aj[K] * (J == L) + Ai[K] * Aj[J] * (I == L) +
             Ai[J] * Aj[K] * (I == L) + Ai[K] * Aj[I] * (J == L)) * 0.25;
        CCt[TRI(a, b)] += w5 * e;
      }
    }
  }
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    int I, J;
    slot_pair(a, I, J);
#pragma unroll
    for (int b = a; b < 6; ++b) {
      int K, L;
      slot_pair(b, K, L);
      // c [x] c : (c_IK c_JL + c_IL c_JK)/2 ; identity [x] identity likewise
      const double cIK = c[VI(I, K)], cJL = c[VI(J, L)], cIL = c[VI(I, L)], cJK = c[VI(J, K)];
      const double cbox = 0.5 * (cIK * cJL + cIL * cJK);
      const double ibox = 0.5 * ((I == K) * (J == L) + (I == L) * (J == K));
      const double ixi = (a < 3 && b < 3) ? 1.0 : 0.0;
      double v = U[a] * c[b] + c[a] * U[b] + kcc * c[a] * c[b] + kbox * cbox
               + w2 * (ixi - ibox) + dN[1] * f2_2 * dI2t[a] * dI2t[b];
      CCt[TRI(a, b)] += v;
    }
  }
}

// dK_m/dC for a feature index known only at run time (uniform across the
// wave); every case is a compile-time instance, so nothing is indexed
// dynamically in registers.
template <int NSV>
__host__ __device__ inline void kin_dfeature_rt(const Kin& k, const ModelConst& mc, int m, double* d) {
  switch (m) {
    case 0: kin_dfeature<NSV>(k, mc, 0, d); break;
    case 1: kin_dfeature<NSV>(k, mc, 1, d); break;
    case 2: kin_dfeature<NSV>(k, mc, 2, d); break;
    case 3: if constexpr (Feat<NSV>::P > 3) kin_dfeature<NSV>(k, mc, 3, d); break;
    case 4: if constexpr (Feat<NSV>::P > 4) kin_dfeature<NSV>(k, mc, 4, d); break;
    case 5: if constexpr (Feat<NSV>::P > 5) kin_dfeature<NSV>(k, mc, 5, d); break;
    case 6: if constexpr (Feat<NSV>::P > 6) kin_dfeature<NSV>(k, mc, 6, d); break;
    case 7: if constexpr (Feat<NSV>::P > 7) kin_dfeature<NSV>(k, mc, 7, d); break;
    default: if constexpr (Feat<NSV>::P > 8) kin_dfeature<NSV>(k, mc, 8, d); break;
  }
}

// Same result as chain_material, with the network derivatives read through
// accessors (N1(m) = dN/dK_m, N2(idx) = packed d2N) and the feature
// gradients recomputed inside the loops instead of being held in registers.
template <int NSV, class G1, class G2>
__host__ __device__ inline void chain_material_lean(const Kin& k, const ModelConst& mc, G1 N1, G2 N2,
                                                    double* S, double* CCt) {
  constexpr int P = Feat<NSV>::P;
#pragma unroll
  for (int a = 0; a < 6; ++a) S[a] = 0.0;
#pragma unroll
  for (int t = 0; t < 21; ++t) CCt[t] = 0.0;
#pragma unroll 1
  for (int m = 0; m < P; ++m) {
    double Dm[6];
    kin_dfeature_rt<NSV>(k, mc, m, Dm);
    const double nm = N1(m);
#pragma unroll
    for (int a = 0; a < 6; ++a) S[a] += nm * Dm[a];
    double V[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll 1
    for (int n = 0; n < P; ++n) {
      double Dn[6];
      kin_dfeature_rt<NSV>(k, mc, n, Dn);
      const int mm = m < n ? m : n, nn = m < n ? n : m;
      const double w = N2(mm * P - mm * (mm - 1) / 2 + (nn - mm));
#pragma unroll
      for (int a = 0; a < 6; ++a) V[a] += w * Dn[a];
    }
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
      for (int b = a; b < 6; ++b) CCt[TRI(a, b)] += Dm[a] * V[b];
  }
  double dN[P];
#pragma unroll
  for (int m = 0; m < P; ++m) dN[m] = N1(m);
  chain_first_order<NSV>(k, mc, dN, CCt);
}

// Same result as chain_material with short live ranges, for kernels that
// stream the network outputs from memory: the first-derivative terms are
// applied while the kinematic quantities are live, then the feature
// gradients D_m and S~, then the Gram part sum_m D_m (x) V_m with
// V_m = sum_n N_mn D_n, reading the network Hessian one row at a time (an
// empty compiler barrier keeps each row's loads from being hoisted above the
// previous row's arithmetic).  N1(m) = dN/dK_m, N2(idx) = packed d2N;
// second = false computes S~ only.
template <int NSV, class G1, class G2>
__host__ __device__ inline void chain_material_stream(const Kin& k, const ModelConst& mc, G1 N1, G2 N2,
                                                      bool second, double* S, double* CCt) {
  constexpr int P = Feat<NSV>::P;
  double dN[P];
#pragma unroll
  for (int m = 0; m < P; ++m) dN[m] = N1(m);
#pragma unroll
  for (int t = 0; t < 21; ++t) CCt[t] = 0.0;
  if (second) chain_first_order<NSV>(k, mc, dN, CCt);
  double D[P][6];
#pragma unroll
  for (int a = 0; a < 6; ++a) S[a] = 0.0;
#pragma unroll
  for (int m = 0; m < P; ++m) {
    kin_dfeature<NSV>(k, mc, m, D[m]);
#pragma unroll
    for (int a = 0; a < 6; ++a) S[a] += dN[m] * D[m][a];
  }
  if (!second) return;
#pragma unroll
  for (int m = 0; m < P; ++m) {
    asm volatile("" ::: "memory");
    double wr[P];
#pragma unroll
    for (int n2 = 0; n2 < P; ++n2) {
      const int mm = m < n2 ? m : n2, nn = m < n2 ? n2 : m;
      wr[n2] = N2(mm * P - mm * (mm - 1) / 2 + (nn - mm));
    }
    double V[6];
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      double v = 0.0;
#pragma unroll
      for (int n2 = 0; n2 < P; ++n2) v += wr[n2] * D[n2][a];
      V[a] = v;
    }
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
      for (int b = a; b < 6; ++b) CCt[TRI(a, b)] += D[m][a] * V[b];
  }
}

// Spatial Voigt outputs (App. A.1-A.2): Kirchhoff stress tau = F S F^T and
// spatial tangent cc_ijkl = F_iI F_jJ F_kK F_lL CC_IJKL with S = 2 S~ and
// CC = 4 CC~.  In Voigt slots (11, 22, 33, 23, 13, 12) both are products with
// M[c][b] = sum over the index pairs (K, L) of slot c of F_kK F_lL, (k, l) the
// pair of slot b:  tau = 2 M^T s~,  cc = 4 M^T CC~ M  (upper triangle, TRI).
template <class StoreT, class StoreC>
__host__ __device__ inline void push_spatial(const Kin& k, const double* S, const double* CCt, bool tangent,
                                             StoreT storeT, StoreC storeC) {
  const double* F = k.F;
  double M[6][6];  // M[c][b]
#pragma unroll
  for (int b = 0; b < 6; ++b) {
    int kk, ll;
    slot_pair(b, kk, ll);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      int K, L;
      slot_pair(c, K, L);
      M[c][b] = (K == L) ? F[3 * kk + K] * F[3 * ll + K] : F[3 * kk + K] * F[3 * ll + L] + F[3 * kk + L] * F[3 * ll + K];
    }
  }
#pragma unroll
  for (int b = 0; b < 6; ++b) {
    double t = 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c) t += M[c][b] * S[c];
    storeT(b, 2.0 * t);
  }
  if (!tangent) return;
  double X[6][6];  // X = CC~ M
#pragma unroll
  for (int a = 0; a < 6; ++a)
#pragma unroll
    for (int b = 0; b < 6; ++b) {
      double x = 0.0;
#pragma unroll
      for (int c = 0; c < 6; ++c) x += CCt[TRI(a, c)] * M[c][b];
      X[a][b] = x;
    }
#pragma unroll
  for (int a = 0; a < 6; ++a)
#pragma unroll
    for (int b = a; b < 6; ++b) {
      double y = 0.0;
#pragma unroll
      for (int c = 0; c < 6; ++c) y += M[c][a] * X[c][b];
      storeC(TRI(a, b), 4.0 * y);
    }
}

// P = 2 F S~ and AA_iJkL = 2 delta_ik S~_JL + 4 F_iI F_kK CC~_IJKL.
// Calls sink(index, value) for the 9 stress and 81 tangent components.
template <class StoreP, class StoreA>
__host__ __device__ inline void push_material(const Kin& k, const double* S, const double* CCt,
                                     StoreP storeP, StoreA storeA) {
  const double* F = k.F;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int J = 0; J < 3; ++J) {
      double s = 0.0;
#pragma unroll
      for (int I = 0; I < 3; ++I) s += F[3 * i + I] * S[VI(I, J)];
      storeP(3 * i + J, 2.0 * s);
    }
#pragma unroll
  for (int J = 0; J < 3; ++J)
#pragma unroll
    for (int L = J; L < 3; ++L) {
      double X[3][3];
#pragma unroll
      for (int I = 0; I < 3; ++I)
#pragma unroll
        for (int K = 0; K < 3; ++K) X[I][K] = CCt[TRI(VI(I, J), VI(K, L))];
      double FX[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int K = 0; K < 3; ++K)
          FX[i][K] = F[3 * i + 0] * X[0][K] + F[3 * i + 1] * X[1][K] + F[3 * i + 2] * X[2][K];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) {
          double y = 4.0 * (FX[i][0] * F[3 * kk + 0] + FX[i][1] * F[3 * kk + 1] + FX[i][2] * F[3 * kk + 2]);
          if (i == kk) y += 2.0 * S[VI(J, L)];
          storeA(9 * (3 * i + J) + (3 * kk + L), y);
          if (L != J) storeA(9 * (3 * kk + L) + (3 * i + J), y);
        }
    }
}

}  // namespace pa
