// Narrow networks (width <= 8) on the vector ALUs, one quadrature point per
// lane: the adjoint form of the network derivatives (value forward, reverse
// sweep for the gradient, Jacobian forward for the Hessian
//   d2N/dK dK = sum_k J_k^T diag(lambda_k (.) F''(y_k)) J_k,
// same outputs as Alg. 4 up to rounding) with every weight read at a
// wave-uniform address (scalar loads) and every per-point quantity in
// registers.  Below one 16-row matrix-core tile the matrix instructions
// would mostly multiply the zero padding; here the work is proportional to
// the real width.  FP64 or FP32 arithmetic (the precision of the network
// contractions); inputs and outputs FP64.
#include <type_traits>

#include "pa_internal.h"

namespace pa {

template <int HR, int L, int P, class T, bool HESS>
__global__ void __launch_bounds__(256) k_mlp_valu(const unsigned char* __restrict__ prep, PrepLayout lay, int64_t n,
                                                  const double* __restrict__ Kin, double* __restrict__ out) {
  constexpr int P2 = P * (P + 1) / 2;
  const int H = lay.H;  // row stride of the prepared (zero-padded) tables
  const bool dbl = std::is_same<T, double>::value;
  const T* W1t = (const T*)(prep + (dbl ? lay.d_W1t : lay.f_W1t));  // [P][H]: W1[r][m] at m H + r
  const T* Bt = (const T*)(prep + (dbl ? lay.d_Bt : lay.f_Bt));     // [L][P][H]: layer k at k - 1
  const T* Am = (const T*)(prep + (dbl ? lay.d_Am : lay.f_Am));     // [L][H][H]: A_k[r][s] at ((k-1) H + r) H + s
  const T* cb = (const T*)(prep + (dbl ? lay.d_c : lay.f_c));       // [L][H]
  const T* av = (const T*)(prep + (dbl ? lay.d_a : lay.f_a));       // [H]
  const double* bv = (const double*)(prep + lay.d_b);                // [P], FP64
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;

  double kd[P];
  T k[P];
#pragma unroll
  for (int m = 0; m < P; ++m) {
    kd[m] = Kin[(int64_t)m * n + t];
    k[m] = (T)kd[m];
  }
  // ---- value forward; F' and F'' of every layer kept
  T s[L][HR], tt[L][HR], z[HR], zn[HR];
#pragma unroll
  for (int r = 0; r < HR; ++r) {
    T y = cb[r];
#pragma unroll
    for (int m = 0; m < P; ++m) y += W1t[m * H + r] * k[m];
    softplus3(y, z[r], s[0][r], tt[0][r]);
  }
#pragma unroll
  for (int kk = 1; kk < L; ++kk) {
#pragma unroll
    for (int r = 0; r < HR; ++r) {
      T y = cb[kk * H + r];
#pragma unroll
      for (int q = 0; q < HR; ++q) y += Am[(kk * H + r) * H + q] * z[q];
#pragma unroll
      for (int m = 0; m < P; ++m) y += Bt[(kk * P + m) * H + r] * k[m];
      softplus3(y, zn[r], s[kk][r], tt[kk][r]);
    }
#pragma unroll
    for (int r = 0; r < HR; ++r) z[r] = zn[r];
  }
  double val = 0.0;
#pragma unroll
  for (int r = 0; r < HR; ++r) val += (double)(av[r] * z[r]);
#pragma unroll
  for (int m = 0; m < P; ++m) val += bv[m] * kd[m];
  out[t] = val;

  // ---- reverse sweep: mu_k = lambda_k F'(y_k), gamma_k = lambda_k F''(y_k)
  T mu[HR], g[L][HR];
  T grad[P];
#pragma unroll
  for (int m = 0; m < P; ++m) grad[m] = (T)0;
#pragma unroll
  for (int r = 0; r < HR; ++r) {
    mu[r] = av[r] * s[L - 1][r];
    g[L - 1][r] = av[r] * tt[L - 1][r];
  }
#pragma unroll
  for (int kk = L - 1; kk >= 1; --kk) {
    T lam[HR];
#pragma unroll
    for (int m = 0; m < P; ++m)
#pragma unroll
      for (int r = 0; r < HR; ++r) grad[m] += Bt[(kk * P + m) * H + r] * mu[r];
#pragma unroll
    for (int q = 0; q < HR; ++q) {
      T x = (T)0;
#pragma unroll
      for (int r = 0; r < HR; ++r) x += Am[(kk * H + r) * H + q] * mu[r];
      lam[q] = x;
    }
#pragma unroll
    for (int q = 0; q < HR; ++q) {
      mu[q] = lam[q] * s[kk - 1][q];
      g[kk - 1][q] = lam[q] * tt[kk - 1][q];
    }
  }
#pragma unroll
  for (int m = 0; m < P; ++m) {
#pragma unroll
    for (int r = 0; r < HR; ++r) grad[m] += W1t[m * H + r] * mu[r];
    out[(int64_t)(1 + m) * n + t] = (double)grad[m] + bv[m];
  }
  if constexpr (!HESS) return;

  // ---- Hessian: layer 1 (J_1 = W1), then the Jacobians of layers >= 2
  T hs[P2];
#pragma unroll
  for (int h = 0; h < P2; ++h) hs[h] = (T)0;
  auto add_rows = [&](const T (&Jr)[P], T gr) {  // hs += gr * Jr Jr^T (upper triangle, row-major packed)
    T gj[P];
#pragma unroll
    for (int m = 0; m < P; ++m) gj[m] = gr * Jr[m];
    int h = 0;
#pragma unroll
    for (int m = 0; m < P; ++m)
#pragma unroll
      for (int q = m; q < P; ++q, ++h) hs[h] += gj[m] * Jr[q];
  };
#pragma unroll
  for (int r = 0; r < HR; ++r) {
    T Jr[P];
#pragma unroll
    for (int m = 0; m < P; ++m) Jr[m] = W1t[m * H + r];
    add_rows(Jr, g[0][r]);
  }
  // J_k[r][m] = sum_q A_k[r][q] F'(y_{k-1})_q J_{k-1}[q][m] + B_k[r][m]
  T Jp[L > 2 ? HR : 1][P];  // J of the previous layer (three or more layers)
#pragma unroll
  for (int kk = 1; kk < L; ++kk) {
    T Jc[L > 2 ? HR : 1][P];
#pragma unroll
    for (int r = 0; r < HR; ++r) {
      T Jr[P];
#pragma unroll
      for (int m = 0; m < P; ++m) {
        T x = Bt[(kk * P + m) * H + r];
#pragma unroll
        for (int q = 0; q < HR; ++q) {
          const T sj = (kk == 1) ? s[0][q] * W1t[m * H + q] : s[kk - 1][q] * Jp[L > 2 ? q : 0][m];
          x += Am[(kk * H + r) * H + q] * sj;
        }
        Jr[m] = x;
      }
      add_rows(Jr, g[kk][r]);
      if constexpr (L > 2) {
#pragma unroll
        for (int m = 0; m < P; ++m) Jc[r][m] = Jr[m];
      }
    }
    if constexpr (L > 2) {
#pragma unroll
      for (int r = 0; r < HR; ++r)
#pragma unroll
        for (int m = 0; m < P; ++m) Jp[r][m] = Jc[r][m];
    }
  }
#pragma unroll
  for (int h = 0; h < P2; ++h) out[(int64_t)(1 + P + h) * n + t] = (double)hs[h];
}

template <int HR, int L, int P>
static int launch_valu_t(const PrepLayout& lay, int prec, const unsigned char* prep, int64_t n, const double* K,
                         double* out, int hess, hipStream_t s) {
  const unsigned grid = (unsigned)((n + 255) / 256);
  if (prec == PREC_F64) {
    if (hess) k_mlp_valu<HR, L, P, double, true><<<grid, 256, 0, s>>>(prep, lay, n, K, out);
    else k_mlp_valu<HR, L, P, double, false><<<grid, 256, 0, s>>>(prep, lay, n, K, out);
  } else if (prec == PREC_F32) {
    if (hess) k_mlp_valu<HR, L, P, float, true><<<grid, 256, 0, s>>>(prep, lay, n, K, out);
    else k_mlp_valu<HR, L, P, float, false><<<grid, 256, 0, s>>>(prep, lay, n, K, out);
  } else {
    return -2;
  }
  return 0;
}

template <int HR, int L>
static int launch_valu_p(const PrepLayout& lay, int prec, const unsigned char* prep, int64_t n, const double* K,
                         double* out, int hess, hipStream_t s) {
  switch (lay.P) {
    case 3: return launch_valu_t<HR, L, 3>(lay, prec, prep, n, K, out, hess, s);
    case 5: return launch_valu_t<HR, L, 5>(lay, prec, prep, n, K, out, hess, s);
    case 9: return launch_valu_t<HR, L, 9>(lay, prec, prep, n, K, out, hess, s);
    default: return -2;
  }
}

template <int HR>
static int launch_valu_l(const PrepLayout& lay, int prec, const unsigned char* prep, int64_t n, const double* K,
                         double* out, int hess, hipStream_t s) {
  switch (lay.L) {
    case 2: return launch_valu_p<HR, 2>(lay, prec, prep, n, K, out, hess, s);
    case 3: return launch_valu_p<HR, 3>(lay, prec, prep, n, K, out, hess, s);
    case 4: return launch_valu_p<HR, 4>(lay, prec, prep, n, K, out, hess, s);
    default: return -2;
  }
}

// Real widths 1..8 run the kernel of the next width in {2, 4, 8}: the
// prepared tables are zero beyond the real width, so the extra rows add
// nothing.
int launch_mlp_valu(const PrepLayout& lay, int prec, const unsigned char* prep, int64_t n, const double* K,
                    double* out, int hess, hipStream_t s) {
  if (lay.HR <= 2) return launch_valu_l<2>(lay, prec, prep, n, K, out, hess, s);
  if (lay.HR <= 4) return launch_valu_l<4>(lay, prec, prep, n, K, out, hess, s);
  if (lay.HR <= 8) return launch_valu_l<8>(lay, prec, prep, n, K, out, hess, s);
  return -2;
}

}  // namespace pa
