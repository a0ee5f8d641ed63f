// Finite-element kernels: isoparametric geometry, deformation gradients at
// the quadrature points, element residual/stiffness integration and coloured
// CSR scatter-assembly (eqs. apprx-k, apprx-r, r-quad, k-quad; Alg. 1-2).
#include "pa_internal.h"

namespace pa {

static inline unsigned nblocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// ---------------------------------------------------------------- shapes
// Reference-coordinate derivatives dN_a/dxi_d at quadrature point q.
template <int NEN>
__device__ inline void ref_grads(int q, double (&dN)[NEN][3], double& wq);

template <>
__device__ inline void ref_grads<8>(int q, double (&dN)[8][3], double& wq) {
  const double g = 0.57735026918962576451;  // 1/sqrt(3)
  const double xi[3] = {(2 * (q & 1) - 1) * g, (2 * ((q >> 1) & 1) - 1) * g, (2 * ((q >> 2) & 1) - 1) * g};
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const double s[3] = {(double)(2 * (a & 1) - 1), (double)(2 * ((a >> 1) & 1) - 1), (double)(2 * ((a >> 2) & 1) - 1)};
    const double f0 = 1.0 + s[0] * xi[0], f1 = 1.0 + s[1] * xi[1], f2 = 1.0 + s[2] * xi[2];
    dN[a][0] = 0.125 * s[0] * f1 * f2;
    dN[a][1] = 0.125 * s[1] * f0 * f2;
    dN[a][2] = 0.125 * s[2] * f0 * f1;
  }
  wq = 1.0;
}

template <>
__device__ inline void ref_grads<10>(int q, double (&dN)[10][3], double& wq) {
  const double al = 0.5854101966249685, be = 0.1381966011250105;
  double L[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) L[v] = (v == q) ? al : be;
  // dL_v/dxi_d: L0 = 1 - xi - eta - zeta, L_{d+1} = xi_d
  auto dL = [](int v, int d) -> double { return v == 0 ? -1.0 : (v == d + 1 ? 1.0 : 0.0); };
  const int ei[6] = {0, 1, 0, 0, 1, 2};
  const int ej[6] = {1, 2, 2, 3, 3, 3};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
#pragma unroll
    for (int v = 0; v < 4; ++v) dN[v][d] = (4.0 * L[v] - 1.0) * dL(v, d);
#pragma unroll
    for (int e = 0; e < 6; ++e) dN[4 + e][d] = 4.0 * (L[ej[e]] * dL(ei[e], d) + L[ei[e]] * dL(ej[e], d));
  }
  wq = 1.0 / 24.0;
}

template <int NEN>
__device__ inline constexpr int nq_of() { return NEN == 8 ? 8 : 4; }

// ---------------------------------------------------------------- geometry
template <int NEN>
__global__ void __launch_bounds__(256) k_geometry(int64_t n_el, int64_t n_nodes, const double* __restrict__ X,
                                                  const int32_t* __restrict__ conn, double* __restrict__ dNdX,
                                                  double* __restrict__ w, int32_t* n_bad) {
  constexpr int NQ = nq_of<NEN>();
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_el * NQ) return;
  const int q = (int)(t / n_el);
  const int64_t e = t % n_el;
  double dN[NEN][3], wq;
  ref_grads<NEN>(q, dN, wq);
  double jac[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // dX_J / dxi_d
#pragma unroll
  for (int a = 0; a < NEN; ++a) {
    const int64_t node = conn[(int64_t)a * n_el + e];
#pragma unroll
    for (int J = 0; J < 3; ++J) {
      const double x = X[J * n_nodes + node];
#pragma unroll
      for (int d = 0; d < 3; ++d) jac[d][J] += dN[a][d] * x;
    }
  }
  const double det = jac[0][0] * (jac[1][1] * jac[2][2] - jac[1][2] * jac[2][1])
                   - jac[0][1] * (jac[1][0] * jac[2][2] - jac[1][2] * jac[2][0])
                   + jac[0][2] * (jac[1][0] * jac[2][1] - jac[1][1] * jac[2][0]);
  const double r = 1.0 / det;
  double inv[3][3];  // inverse of jac (as a matrix d x J): inv[J][d]
  inv[0][0] = (jac[1][1] * jac[2][2] - jac[1][2] * jac[2][1]) * r;
  inv[0][1] = (jac[0][2] * jac[2][1] - jac[0][1] * jac[2][2]) * r;
  inv[0][2] = (jac[0][1] * jac[1][2] - jac[0][2] * jac[1][1]) * r;
  inv[1][0] = (jac[1][2] * jac[2][0] - jac[1][0] * jac[2][2]) * r;
  inv[1][1] = (jac[0][0] * jac[2][2] - jac[0][2] * jac[2][0]) * r;
  inv[1][2] = (jac[0][2] * jac[1][0] - jac[0][0] * jac[1][2]) * r;
  inv[2][0] = (jac[1][0] * jac[2][1] - jac[1][1] * jac[2][0]) * r;
  inv[2][1] = (jac[0][1] * jac[2][0] - jac[0][0] * jac[2][1]) * r;
  inv[2][2] = (jac[0][0] * jac[1][1] - jac[0][1] * jac[1][0]) * r;
#pragma unroll
  for (int a = 0; a < NEN; ++a)
#pragma unroll
    for (int J = 0; J < 3; ++J) {
      const double v = inv[J][0] * dN[a][0] + inv[J][1] * dN[a][1] + inv[J][2] * dN[a][2];
      dNdX[(((int64_t)q * NEN + a) * 3 + J) * n_el + e] = v;
    }
  w[(int64_t)q * n_el + e] = wq * det;
  if (n_bad && !(det > 0.0)) atomicAdd(n_bad, 1);
}

// ---------------------------------------------------------------- F at points
// F_iJ = delta_iJ + sum_a u^a_i dN^a/dX_J; point index q*n_el + e.
template <int NEN>
__global__ void __launch_bounds__(256) k_gather_F(int64_t n_el, const int32_t* __restrict__ conn,
                                                  const double* __restrict__ dNdX, const double* __restrict__ u,
                                                  double* __restrict__ F) {
  constexpr int NQ = nq_of<NEN>();
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = n_el * NQ;
  if (t >= n) return;
  const int q = (int)(t / n_el);
  const int64_t e = t % n_el;
  double f[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
#pragma unroll
  for (int a = 0; a < NEN; ++a) {
    const int64_t node = conn[(int64_t)a * n_el + e];
    const double u0 = u[3 * node], u1 = u[3 * node + 1], u2 = u[3 * node + 2];
#pragma unroll
    for (int J = 0; J < 3; ++J) {
      const double g = dNdX[(((int64_t)q * NEN + a) * 3 + J) * n_el + e];
      f[J] += u0 * g;
      f[3 + J] += u1 * g;
      f[6 + J] += u2 * g;
    }
  }
#pragma unroll
  for (int c = 0; c < 9; ++c) F[(int64_t)c * n + t] = f[c];
}

// ---------------------------------------------------------------- integration
// One thread per (element, node a): rows 3a..3a+2 of K_e and r_e.
//   r^a_i  = sum_q w P_iJ dN^a/dX_J
//   K^ab_ik = sum_q w dN^a/dX_J AA_iJkL dN^b/dX_L
template <int NEN>
__global__ void __launch_bounds__(256) k_integrate(int64_t n_el, const double* __restrict__ dNdX,
                                                   const double* __restrict__ w, const double* __restrict__ P,
                                                   const double* __restrict__ A, double* __restrict__ r_e,
                                                   double* __restrict__ K_e) {
  constexpr int NQ = nq_of<NEN>();
  constexpr int ND = 3 * NEN;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_el * NEN) return;
  const int64_t e = t / NEN;
  const int a = (int)(t % NEN);
  const int64_t n = n_el * NQ;
  double r[3] = {0, 0, 0};
  double K[3][ND];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int c = 0; c < ND; ++c) K[i][c] = 0.0;
  for (int q = 0; q < NQ; ++q) {
    const int64_t pt = (int64_t)q * n_el + e;
    const double wq = w[pt];
    double ga[3];
#pragma unroll
    for (int J = 0; J < 3; ++J) ga[J] = dNdX[(((int64_t)q * NEN + a) * 3 + J) * n_el + e];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double s = 0.0;
#pragma unroll
      for (int J = 0; J < 3; ++J) s += P[(int64_t)(3 * i + J) * n + pt] * ga[J];
      r[i] += wq * s;
    }
    // T_ikL = sum_J ga_J AA_iJkL
    double T[3][3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int L = 0; L < 3; ++L) {
          double s = 0.0;
#pragma unroll
          for (int J = 0; J < 3; ++J) s += ga[J] * A[(int64_t)(9 * (3 * i + J) + 3 * k + L) * n + pt];
          T[i][k][L] = wq * s;
        }
#pragma unroll
    for (int b = 0; b < NEN; ++b) {
      double gb[3];
#pragma unroll
      for (int L = 0; L < 3; ++L) gb[L] = dNdX[(((int64_t)q * NEN + b) * 3 + L) * n_el + e];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) K[i][3 * b + k] += T[i][k][0] * gb[0] + T[i][k][1] * gb[1] + T[i][k][2] * gb[2];
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) r_e[e * ND + 3 * a + i] = r[i];
  if (K_e) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int c = 0; c < ND; ++c) K_e[(e * ND + 3 * a + i) * ND + c] = K[i][c];
  }
}

// ---------------------------------------------------------------- CSR map
template <int NEN>
__global__ void __launch_bounds__(256) k_csr_map(int64_t n_el, const int32_t* __restrict__ conn,
                                                 const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                                 int32_t* __restrict__ e2csr) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_el * NEN * NEN) return;
  const int64_t e = t / (NEN * NEN);
  const int a = (int)((t / NEN) % NEN), b = (int)(t % NEN);
  const int64_t row = 3 * (int64_t)conn[(int64_t)a * n_el + e];
  const int32_t target = 3 * conn[(int64_t)b * n_el + e];
  int64_t lo = row_ptr[row], hi = row_ptr[row + 1];
  const int64_t start = lo;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (col[mid] < target) lo = mid + 1; else hi = mid;
  }
  e2csr[t] = (lo < row_ptr[row + 1] && col[lo] == target) ? (int32_t)(lo - start) : -1;
}

// ---------------------------------------------------------------- assembly
// One launch per colour; thread = (element of the colour, element row).
template <int NEN>
__global__ void __launch_bounds__(256) k_assemble(int64_t e_begin, int64_t e_count, const int32_t* __restrict__ perm,
                                                  int64_t n_el, const int32_t* __restrict__ conn,
                                                  const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ e2csr,
                                                  const double* __restrict__ r_e, const double* __restrict__ K_e,
                                                  double* __restrict__ r, double* __restrict__ vals) {
  constexpr int ND = 3 * NEN;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= e_count * ND) return;
  const int64_t pos = e_begin + t / ND;
  const int64_t e = perm ? (int64_t)perm[pos] : pos;
  const int rho = (int)(t % ND);
  const int a = rho / 3, i = rho % 3;
  const int64_t R = 3 * (int64_t)conn[(int64_t)a * n_el + e] + i;
  if (r) r[R] += r_e[e * ND + rho];
  if (vals) {
    const int64_t base = row_ptr[R];
    const double* Krow = K_e + (e * ND + rho) * ND;
#pragma unroll
    for (int b = 0; b < NEN; ++b) {
      const int32_t off = e2csr[(e * NEN + a) * NEN + b];
      if (off < 0) continue;  // column not in the pattern (cannot happen for a pattern built from conn)
      const int64_t p = base + off;
      vals[p] += Krow[3 * b];
      vals[p + 1] += Krow[3 * b + 1];
      vals[p + 2] += Krow[3 * b + 2];
    }
  }
}

__global__ void k_fill(double* x, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) x[i] = v;
}

// ---------------------------------------------------------------- launchers
#define PA_NEN_SWITCH(nen, CALL8, CALL10) \
  do {                                     \
    if ((nen) == 8) { CALL8; }             \
    else if ((nen) == 10) { CALL10; }      \
    else return -1;                        \
  } while (0)

int launch_geometry(int nen, int64_t n_el, int64_t n_nodes, const double* X, const int32_t* conn,
                    double* dNdX, double* w, int32_t* n_bad, hipStream_t s) {
  if (n_el == 0) return 0;
  const int nq = nen == 8 ? 8 : 4;
  PA_NEN_SWITCH(nen, (k_geometry<8><<<nblocks(n_el * nq, 256), 256, 0, s>>>(n_el, n_nodes, X, conn, dNdX, w, n_bad)),
                (k_geometry<10><<<nblocks(n_el * nq, 256), 256, 0, s>>>(n_el, n_nodes, X, conn, dNdX, w, n_bad)));
  return 0;
}

int launch_gather_F(int nen, int nq, int64_t n_el, const int32_t* conn, const double* dNdX,
                    const double* u, double* F, hipStream_t s) {
  if (n_el == 0) return 0;
  PA_NEN_SWITCH(nen, (k_gather_F<8><<<nblocks(n_el * nq, 256), 256, 0, s>>>(n_el, conn, dNdX, u, F)),
                (k_gather_F<10><<<nblocks(n_el * nq, 256), 256, 0, s>>>(n_el, conn, dNdX, u, F)));
  return 0;
}

int launch_integrate(int nen, int nq, int64_t n_el, const double* dNdX, const double* w,
                     const double* P, const double* A, double* r_e, double* K_e, hipStream_t s) {
  if (n_el == 0) return 0;
  (void)nq;
  PA_NEN_SWITCH(nen, (k_integrate<8><<<nblocks(n_el * 8, 256), 256, 0, s>>>(n_el, dNdX, w, P, A, r_e, K_e)),
                (k_integrate<10><<<nblocks(n_el * 10, 256), 256, 0, s>>>(n_el, dNdX, w, P, A, r_e, K_e)));
  return 0;
}

int launch_csr_map(int nen, int64_t n_el, const int32_t* conn, const int64_t* row_ptr,
                   const int32_t* col, int32_t* e2csr, hipStream_t s) {
  if (n_el == 0) return 0;
  PA_NEN_SWITCH(nen, (k_csr_map<8><<<nblocks(n_el * 64, 256), 256, 0, s>>>(n_el, conn, row_ptr, col, e2csr)),
                (k_csr_map<10><<<nblocks(n_el * 100, 256), 256, 0, s>>>(n_el, conn, row_ptr, col, e2csr)));
  return 0;
}

int launch_assemble(int nen, int64_t e_begin, int64_t e_count, const int32_t* perm, int64_t n_el,
                    const int32_t* conn, const int64_t* row_ptr, const int32_t* e2csr,
                    const double* r_e, const double* K_e, double* r, double* vals, hipStream_t s) {
  if (e_count == 0) return 0;
  PA_NEN_SWITCH(nen,
                (k_assemble<8><<<nblocks(e_count * 24, 256), 256, 0, s>>>(e_begin, e_count, perm, n_el, conn, row_ptr, e2csr, r_e, K_e, r, vals)),
                (k_assemble<10><<<nblocks(e_count * 30, 256), 256, 0, s>>>(e_begin, e_count, perm, n_el, conn, row_ptr, e2csr, r_e, K_e, r, vals)));
  return 0;
}

int launch_fill(double* x, int64_t n, double v, hipStream_t s) {
  if (n == 0) return 0;
  const int64_t b = (n + 255) / 256;
  k_fill<<<(unsigned)(b < 65536 ? b : 65536), 256, 0, s>>>(x, n, v);
  return 0;
}

}  // namespace pa
