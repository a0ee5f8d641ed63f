// Inner functions other than the MICNN: the CANN of App. B.1 (eqs. cann-def,
// cann-chain-rule) and the Gent-Thomas energy of eq. (gt), written as
// functions of the features K.  They fill the same output tile as the
// network kernels ([N | dN/dK_m | packed d2N/dK_m dK_n][n], the Hessian
// diagonal in K), so the chain rule, elements and assembly are shared.
//
// CANN parameters (per input m, 8 values): for the four branches (power 1,
// linear), (power 2, linear), (power 1, exp), (power 2, exp) an inner weight
// w1 and an outer weight w2:  N = sum_m sum_k w2 f2(K_m^e; w1), f2 = w1 x or
// exp(w1 x) - 1.  Gent-Thomas parameters (c1, c2, c3):
// N = c1 K_1 + c2 ((2/3) log(K_2 + 3^{3/2}) - log 3) + c3 K_3.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "pa_internal.h"

namespace pa {

namespace {
constexpr double S32C = 5.196152422706632;  // 3^{3/2}

template <int KIND, int P>
__device__ inline void closed_eval(const double* __restrict__ th, const double (&k)[P], double& N, double (&dN)[P],
                                   double (&d2)[P]) {
  N = 0.0;
#pragma unroll
  for (int m = 0; m < P; ++m) { dN[m] = 0.0; d2[m] = 0.0; }
  if constexpr (KIND == MODEL_CANN) {
#pragma unroll
    for (int m = 0; m < P; ++m) {
      const double x = k[m];
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int e = (b & 1) ? 2 : 1;
        const double w1 = th[8 * m + 2 * b], w2 = th[8 * m + 2 * b + 1];
        const double f1 = (e == 1) ? x : x * x;
        const double d1 = (e == 1) ? 1.0 : 2.0 * x;
        const double dd1 = (e == 1) ? 0.0 : 2.0;
        double f2, g2, h2;
        if (b < 2) {
          f2 = w1 * f1; g2 = w1; h2 = 0.0;
        } else {
          const double ex = exp(w1 * f1);
          f2 = ex - 1.0; g2 = w1 * ex; h2 = w1 * w1 * ex;
        }
        N += w2 * f2;
        dN[m] += w2 * g2 * d1;
        d2[m] += w2 * (h2 * d1 * d1 + g2 * dd1);
      }
    }
  } else {  // MODEL_GENT_THOMAS
    const double c1 = th[0], c2 = th[1], c3 = th[2];
    const double u = k[1] + S32C;
    N = c1 * k[0] + c2 * ((2.0 / 3.0) * log(u) - 1.0986122886681098) + c3 * k[2];  // log 3
    dN[0] = c1;
    dN[1] = c2 * (2.0 / 3.0) / u;
    dN[2] = c3;
    d2[1] = -c2 * (2.0 / 3.0) / (u * u);
  }
}

// One thread per point.  With normalisation the reference-state correction
// sum_q kappa_q K_{4,q} is removed here (the network kernels fold it into the
// output weights instead); N(0) is removed by the chain rule.
template <int KIND, int P>
__global__ void __launch_bounds__(256) k_inner_closed(const double* __restrict__ th, const double* __restrict__ hdr,
                                                      int npair, int64_t n, const double* __restrict__ K,
                                                      double* __restrict__ out, int hess) {
  constexpr int P2 = P * (P + 1) / 2;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  double k[P];
#pragma unroll
  for (int m = 0; m < P; ++m) k[m] = K[(int64_t)m * n + t];
  double N, dN[P], d2[P];
  closed_eval<KIND, P>(th, k, N, dN, d2);
  constexpr int NPAIR = (P - 3) / 2;  // the header holds zeros without normalisation
#pragma unroll
  for (int q = 0; q < NPAIR; ++q) {
    const double kap = hdr[1 + q];
    N -= kap * k[3 + q];
    dN[3 + q] -= kap;
  }
  (void)npair;
  out[t] = N;
#pragma unroll
  for (int m = 0; m < P; ++m) out[(int64_t)(1 + m) * n + t] = dN[m];
  if (hess) {
    int h = 0;
#pragma unroll
    for (int m = 0; m < P; ++m)
#pragma unroll
      for (int j = m; j < P; ++j, ++h) out[(int64_t)(1 + P + h) * n + t] = (j == m) ? d2[m] : 0.0;
  }
  (void)P2;
}

// Copies theta and, with normalisation, stores N(0) and kappa_q =
// dN/dK_{4,q}(0) + 2 dN/dK_{5,q}(0) in the header.
template <int KIND, int P>
__global__ void k_prepare_closed(const double* __restrict__ theta, int n_params, double* __restrict__ hdr,
                                 double* __restrict__ th, int normalize, int npair) {
  for (int i = threadIdx.x; i < n_params; i += blockDim.x) th[i] = theta[i];
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int i = 0; i < 8; ++i) hdr[i] = 0.0;
  if (!normalize) return;
  double k[P], N, dN[P], d2[P];
#pragma unroll
  for (int m = 0; m < P; ++m) k[m] = 0.0;
  closed_eval<KIND, P>(theta, k, N, dN, d2);
  hdr[0] = N;
  constexpr int NPAIR = (P - 3) / 2;
#pragma unroll
  for (int q = 0; q < NPAIR; ++q) hdr[1 + q] = dN[3 + q] + 2.0 * dN[3 + NPAIR + q];
  (void)npair;
}
}  // namespace

#define PA_CLOSED_SWITCH(kind, p, CALL)                                \
  do {                                                                 \
    if (kind == MODEL_CANN) {                                          \
      if (p == 3) { constexpr int KI = MODEL_CANN, PI = 3; CALL; }     \
      else if (p == 5) { constexpr int KI = MODEL_CANN, PI = 5; CALL; } \
      else if (p == 9) { constexpr int KI = MODEL_CANN, PI = 9; CALL; } \
      else return -1;                                                  \
    } else if (kind == MODEL_GENT_THOMAS) {                            \
      if (p == 3) { constexpr int KI = MODEL_GENT_THOMAS, PI = 3; CALL; }     \
      else if (p == 5) { constexpr int KI = MODEL_GENT_THOMAS, PI = 5; CALL; } \
      else if (p == 9) { constexpr int KI = MODEL_GENT_THOMAS, PI = 9; CALL; } \
      else return -1;                                                  \
    } else {                                                           \
      return -1;                                                       \
    }                                                                  \
  } while (0)

int launch_prepare_closed(int kind, int p, int n_params, const double* theta, unsigned char* prep, int normalize,
                          int npair, hipStream_t s) {
  const ClosedLayout cl = closed_layout(kind, p);
  double* hdr = (double*)(prep + cl.hdr);
  double* th = (double*)(prep + cl.theta);
  PA_CLOSED_SWITCH(kind, p, (k_prepare_closed<KI, PI><<<1, 64, 0, s>>>(theta, n_params, hdr, th, normalize, npair)));
  return 0;
}

int launch_inner_closed(int kind, int p, const unsigned char* prep, int npair, int64_t n, const double* K,
                        double* out, int hess, hipStream_t s) {
  if (n == 0) return 0;
  const ClosedLayout cl = closed_layout(kind, p);
  const double* hdr = (const double*)(prep + cl.hdr);
  const double* th = (const double*)(prep + cl.theta);
  const unsigned grid = (unsigned)((n + 255) / 256);
  PA_CLOSED_SWITCH(kind, p, (k_inner_closed<KI, PI><<<grid, 256, 0, s>>>(th, hdr, npair, n, K, out, hess)));
  return 0;
}

}  // namespace pa
