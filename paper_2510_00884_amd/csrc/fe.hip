// Finite-element kernels: isoparametric geometry, deformation gradients at
// the quadrature points, element residual/stiffness integration and coloured
// CSR scatter-assembly (eqs. apprx-k, apprx-r, r-quad, k-quad; Alg. 1-2).
#include "pa_internal.h"

namespace pa {

static inline unsigned nblocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// Workgroups are dispatched to the 8 XCDs round-robin (workgroup b runs on
// XCD b mod 8), and each XCD has its own L2.  This bijection on [0, G) gives
// every XCD a contiguous run of logical blocks, so neighbouring blocks (which
// share cache lines at their element boundaries) share an L2.
__device__ inline int64_t xcd_swizzle(int64_t b, int64_t G) {
  constexpr int64_t X = 8;
  const int64_t x = b % X, j = b / X, q = G / X, r = G % X;
  return (x < r) ? x * (q + 1) + j : r * (q + 1) + (x - r) * q + j;
}

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
__host__ __device__ inline constexpr int nq_of() { return NEN == 8 ? 8 : 4; }

// ---------------------------------------------------------------- geometry
// Isoparametric map at reference point q of an element whose node
// coordinates xn(a, J) returns (Sec. 2.1): the reference-coordinate
// derivatives dN, the inverse Jacobian inv[J][d] = (dX/dxi)^{-1} and
// det(dX/dxi); the shape gradients are dN^a/dX_J = sum_d inv[J][d] dN[a][d]
// and the point weight w_q det.  Every kernel that needs the geometry calls
// this, so stored and recomputed gradients agree bit for bit.
template <int NEN, class XN>
__device__ inline double geom_jac(int q, XN&& xn, double (&dN)[NEN][3], double (&inv)[3][3], double& wq) {
  ref_grads<NEN>(q, dN, wq);
  double jac[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // dX_J / dxi_d
#pragma unroll
  for (int a = 0; a < NEN; ++a)
#pragma unroll
    for (int J = 0; J < 3; ++J) {
      const double x = xn(a, J);
#pragma unroll
      for (int d = 0; d < 3; ++d) jac[d][J] += dN[a][d] * x;
    }
  const double det = jac[0][0] * (jac[1][1] * jac[2][2] - jac[1][2] * jac[2][1])
                   - jac[0][1] * (jac[1][0] * jac[2][2] - jac[1][2] * jac[2][0])
                   + jac[0][2] * (jac[1][0] * jac[2][1] - jac[1][1] * jac[2][0]);
  const double r = 1.0 / det;
  inv[0][0] = (jac[1][1] * jac[2][2] - jac[1][2] * jac[2][1]) * r;
  inv[0][1] = (jac[0][2] * jac[2][1] - jac[0][1] * jac[2][2]) * r;
  inv[0][2] = (jac[0][1] * jac[1][2] - jac[0][2] * jac[1][1]) * r;
  inv[1][0] = (jac[1][2] * jac[2][0] - jac[1][0] * jac[2][2]) * r;
  inv[1][1] = (jac[0][0] * jac[2][2] - jac[0][2] * jac[2][0]) * r;
  inv[1][2] = (jac[0][2] * jac[1][0] - jac[0][0] * jac[1][2]) * r;
  inv[2][0] = (jac[1][0] * jac[2][1] - jac[1][1] * jac[2][0]) * r;
  inv[2][1] = (jac[0][1] * jac[2][0] - jac[0][0] * jac[2][1]) * r;
  inv[2][2] = (jac[0][0] * jac[1][1] - jac[0][1] * jac[1][0]) * r;
  return det;
}

__device__ inline double shape_grad(const double (&inv)[3][3], const double (&dNa)[3], int J) {
  return inv[J][0] * dNa[0] + inv[J][1] * dNa[1] + inv[J][2] * dNa[2];
}

template <int NEN>
__global__ void __launch_bounds__(256) k_geometry(int64_t n_el, int64_t n_nodes, const double* __restrict__ X,
                                                  const int32_t* __restrict__ conn, double* __restrict__ dNdX,
                                                  double* __restrict__ w, int32_t* n_bad) {
  constexpr int NQ = nq_of<NEN>();
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_el * NQ) return;
  const int q = (int)(t / n_el);
  const int64_t e = t % n_el;
  double dN[NEN][3], inv[3][3], wq;
  const double det = geom_jac<NEN>(
      q, [&](int a, int J) { return X[J * n_nodes + conn[(int64_t)a * n_el + e]]; }, dN, inv, wq);
#pragma unroll
  for (int a = 0; a < NEN; ++a)
#pragma unroll
    for (int J = 0; J < 3; ++J) dNdX[(((int64_t)q * NEN + a) * 3 + J) * n_el + e] = shape_grad(inv, dN[a], J);
  w[(int64_t)q * n_el + e] = wq * det;
  if (n_bad && !(det > 0.0)) atomicAdd(n_bad, 1);
}

// ---------------------------------------------------------------- F at points
// F_iJ = delta_iJ + sum_a u^a_i dN^a/dX_J; point index q*n_el + e.  GI: the
// shape gradients are recomputed from the node coordinates X [3][n_nodes]
// (24 gathered, mostly cached values per point) instead of streaming the
// stored 24 per point.  NSV >= 0: the network inputs K [p][n] (features of
// App. C with NSV structural vectors) are formed from F in registers too,
// and points with J <= 0 or non-finite F are counted in n_bad.
template <int NEN, bool GI, int NSV>
__global__ void __launch_bounds__(256) k_gather_F(int64_t n_el, int64_t n_nodes, const int32_t* __restrict__ conn,
                                                  const double* __restrict__ dNdX, const double* __restrict__ X,
                                                  const double* __restrict__ u, double* __restrict__ F,
                                                  ModelConst mc, double* __restrict__ K, int32_t* n_bad) {
  constexpr int NQ = nq_of<NEN>();
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = n_el * NQ;
  if (t >= n) return;
  const int q = (int)(t / n_el);
  const int64_t e = t % n_el;
  double f[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  int64_t node[NEN];
#pragma unroll
  for (int a = 0; a < NEN; ++a) node[a] = conn[(int64_t)a * n_el + e];
  double dN[NEN][3], inv[3][3], wq;
  if constexpr (GI) (void)geom_jac<NEN>(q, [&](int a, int J) { return X[J * n_nodes + node[a]]; }, dN, inv, wq);
#pragma unroll
  for (int a = 0; a < NEN; ++a) {
    const double u0 = u[3 * node[a]], u1 = u[3 * node[a] + 1], u2 = u[3 * node[a] + 2];
#pragma unroll
    for (int J = 0; J < 3; ++J) {
      const double g = GI ? shape_grad(inv, dN[a], J) : dNdX[(((int64_t)q * NEN + a) * 3 + J) * n_el + e];
      f[J] += u0 * g;
      f[3 + J] += u1 * g;
      f[6 + J] += u2 * g;
    }
  }
#pragma unroll
  for (int c = 0; c < 9; ++c) F[(int64_t)c * n + t] = f[c];
  if constexpr (NSV >= 0) {
    Kin k;
    kin_compute<NSV>(f, mc, k);
    count_bad(n_bad, !(k.J > 0.0 && finite9(f)));
    double kf[Feat<NSV>::P];
    kin_features<NSV>(k, mc, kf);
#pragma unroll
    for (int m = 0; m < Feat<NSV>::P; ++m) K[m * n + t] = kf[m];
  }
}

// ---------------------------------------------------------------- residual-loss cotangent
// Reverse of r^a_i = sum_q w P_iJ G^a_J (eq. r-quad, material form): for a
// residual cotangent rbar (node-major dofs), the stress cotangent at point
// (q, e) is  Pbar_iJ = w sum_a rbar[3 conn_a + i] G^a_J.  Point index
// q * n_el + e, output [9][n_el nq].
template <int NEN>
__global__ void __launch_bounds__(256) k_residual_cotangent(int64_t n_el, const int32_t* __restrict__ conn,
                                                            const double* __restrict__ dNdX,
                                                            const double* __restrict__ w,
                                                            const double* __restrict__ rbar,
                                                            double* __restrict__ Pbar) {
  constexpr int NQ = nq_of<NEN>();
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = n_el * NQ;
  if (t >= n) return;
  const int q = (int)(t / n_el);
  const int64_t e = t % n_el;
  double f[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int a = 0; a < NEN; ++a) {
    const int64_t node = conn[(int64_t)a * n_el + e];
    const double r0 = rbar[3 * node], r1 = rbar[3 * node + 1], r2 = rbar[3 * node + 2];
#pragma unroll
    for (int J = 0; J < 3; ++J) {
      const double gv = dNdX[(((int64_t)q * NEN + a) * 3 + J) * n_el + e];
      f[J] += r0 * gv;
      f[3 + J] += r1 * gv;
      f[6 + J] += r2 * gv;
    }
  }
  const double wq = w[t];
#pragma unroll
  for (int c = 0; c < 9; ++c) Pbar[(int64_t)c * n + t] = wq * f[c];
}

// Residual loss of eq. (loss) for one time step: dof d is free (group -1),
// fixed on reaction boundary b (group b >= 0) or fixed and unobserved
// (group -2).  L = sum_free r_d^2 + sum_b (R_b - sum_{d in b} r_d)^2.
// Pass 1: per-workgroup partial sums (free squares, then one sum per
// boundary) in a fixed order; pass 2: one workgroup sums the partials in
// workgroup order (bitwise reproducible) and forms L; pass 3: the cotangent
// rbar_d = 2 r_d (free), -2 (R_b - S_b) (boundary b), 0 otherwise.
constexpr int LOSS_BLOCK = 256;
__global__ void __launch_bounds__(LOSS_BLOCK) k_loss_partials(int64_t n_rows, const double* __restrict__ r,
                                                              const int32_t* __restrict__ group, int n_groups,
                                                              double* __restrict__ partials) {
  __shared__ double red[LOSS_BLOCK];
  const int tid = threadIdx.x;
  for (int k = -1; k < n_groups; ++k) {  // k = -1: free squares
    double acc = 0.0;
    for (int64_t d = (int64_t)blockIdx.x * LOSS_BLOCK + tid; d < n_rows; d += (int64_t)gridDim.x * LOSS_BLOCK) {
      const int gdof = group[d];
      if (gdof == k) acc += (k < 0) ? r[d] * r[d] : r[d];
    }
    red[tid] = acc;
    __syncthreads();
    for (int s = LOSS_BLOCK / 2; s > 0; s >>= 1) {
      if (tid < s) red[tid] += red[tid + s];
      __syncthreads();
    }
    if (tid == 0) partials[(int64_t)blockIdx.x * (n_groups + 1) + (k + 1)] = red[0];
    __syncthreads();
  }
}

__global__ void __launch_bounds__(64) k_loss_finish(int nblk, int n_groups, const double* __restrict__ partials,
                                                    const double* __restrict__ R, double* __restrict__ sums,
                                                    double* __restrict__ loss) {
  // one thread per column, partials summed in workgroup order
  const int k = threadIdx.x;
  if (k <= n_groups) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += partials[(int64_t)b * (n_groups + 1) + k];
    sums[k] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double L = sums[0];
    for (int b = 0; b < n_groups; ++b) {
      const double m = R[b] - sums[1 + b];
      L += m * m;
    }
    if (loss) loss[0] = L;
  }
}

// A group id outside [-1, n_groups) is treated as constrained and unobserved
// (as -2): it contributes nothing to the loss (k_loss_partials only matches
// ids -1 .. n_groups-1) and gets a zero cotangent, and no R or sums entry
// beyond n_groups is read.
__global__ void __launch_bounds__(256) k_loss_rbar(int64_t n_rows, int n_groups, const double* __restrict__ r,
                                                   const int32_t* __restrict__ group,
                                                   const double* __restrict__ R, const double* __restrict__ sums,
                                                   double* __restrict__ rbar) {
  const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= n_rows) return;
  const int gdof = group[d];
  rbar[d] = (gdof == -1) ? 2.0 * r[d] : (gdof >= 0 && gdof < n_groups) ? -2.0 * (R[gdof] - sums[1 + gdof]) : 0.0;
}

// ---------------------------------------------------------------- chain rule + integration
// Element kernel over a block of E = 8 elements, 3 nen threads per element:
//  phase A (one thread per point q and row i of its tangent): from F,
//    S~ = dPsi/dC and CC~ = d2Psi/dCdC (tensor components per point, from
//    the material kernel) forms, scaled by the quadrature weight w,
//      P_iJ       = 2 F_iI S~_IJ
//      AA_iJkL    = 2 delta_ik S~_JL + 4 F_iI F_kK CC~_IJKL      (27 per row)
//    into LDS;
//  phase B (one thread per element row rho = 3a + i, row index i uniform
//    across a wave; the block's shape gradients of every point are staged in
//    LDS during phase A, so the loop over points has no barrier):
//      r^a_i   += w P_iJ G^a_J
//      K^ab_ik += (w AA_iJkL G^a_J) G^b_L,                G^a = dN^a/dX
//    the material form of eqs. k-quad and r-quad.
// MODE 0 (tables) writes r_e [nd][n_el] and K_e [nd][nd][n_el]; MODE 1
// (scatter) adds the rows straight into the global r and CSR values (one
// launch per colour, so no two threads touch the same entry); MODE 2
// (element-major tables) writes r_e [n_el][nd] and the symmetric K_e
// [n_el][sym_blocks][3][3], the layout read by the gather assembly.
// Elements per workgroup: eight for hex8 (64 points, so the tangent row of
// phase B is uniform over a wave and the symmetric 45-entry storage
// applies); four for tet10 (measured: 1.93 ms per 56^3 build against 2.14
// with eight and 2.25 with two).
template <int NEN>
__host__ __device__ constexpr int integrate_elems() { return NEN == 10 ? 4 : 8; }
template <int NEN>
__host__ __device__ constexpr int integrate_threads() { return integrate_elems<NEN>() * 3 * NEN; }

// Packed index of entry (al, be) of a symmetric 9 x 9 matrix (upper triangle,
// row-major; 45 entries).
__host__ __device__ constexpr int SYM9(int al, int be) {
  return (al <= be) ? (al * 9 - al * (al - 1) / 2 + (be - al)) : (be * 9 - be * (be - 1) / 2 + (al - be));
}

template <int V>
struct Int {
  static constexpr int value = V;
};

// Symmetric element tangent in node blocks.  K_e is symmetric (AA has major
// symmetry), so of its NEN^2 3 x 3 node blocks only NEN (NEN + 1) / 2 are
// distinct.  Block (a, b) is owned by node a when d = (b - a) mod NEN is
// below NEN / 2, or equals NEN / 2 and a < NEN / 2 (NEN is even); every
// unordered pair has exactly one owner and each node owns NEN / 2 or
// NEN / 2 + 1 blocks.  The owned block (a, d) sits in slot
// sym_slot(a, d) of the element's table, stored row-major with rows of node a.
template <int NEN>
__host__ __device__ constexpr int sym_slot(int a, int d) {
  return d < NEN / 2 ? a * (NEN / 2) + d : NEN * (NEN / 2) + a;
}
template <int NEN>
__host__ __device__ constexpr int sym_blocks() { return NEN * (NEN + 1) / 2; }

// Two phases per block of E elements.  Phase A: one thread per (point, row
// i) pushes S~ and CC~ forward to w P_iJ and w AA_iJkL (AA_iJkL = 2 delta_ik
// S~_JL + 4 F_iI F_kK CC~_IJKL, App. A.1) into LDS.  AA has major symmetry
// (AA_iJkL = AA_kLiJ), so when the row index of phase B is uniform over a
// wavefront (E * NEN a multiple of 64) only its 45 distinct entries are
// stored, which is what lets four blocks share a compute unit's LDS; the
// wave then runs a copy of the point loop specialised for its row, so every
// LDS offset is an immediate.  Phase B: one thread per (row i, node a,
// element) accumulates row 3a + i of K_e and r_e over the points.
template <int NEN, int MODE, bool GI>
__global__ void __launch_bounds__(integrate_threads<NEN>()) __attribute__((amdgpu_waves_per_eu(3))) k_chain_integrate(
    int64_t n_el, int64_t e_begin, int64_t e_count, const int32_t* __restrict__ conn,
    const double* __restrict__ dNdX, const double* __restrict__ w, int64_t n_nodes, const double* __restrict__ X,
    const double* __restrict__ F,
    const double* __restrict__ SC, double* __restrict__ r_e, double* __restrict__ K_e,
    const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ e2csr, double* __restrict__ r,
    double* __restrict__ vals) {
  constexpr int NQ = nq_of<NEN>();
  constexpr int ND = 3 * NEN;
  constexpr int E = integrate_elems<NEN>();
  constexpr int NT = integrate_threads<NEN>();
  constexpr int NPT = E * NQ;      // points per block
  constexpr int NG = E * NEN * 3;  // shape-gradient values per point slice
  constexpr bool SYMA = (E * NEN) % 64 == 0;
  constexpr int NA = SYMA ? 45 : 81;
  static_assert(NG == NT, "one shape-gradient value per thread per point");
  static_assert(3 * NPT <= NT, "one (point, row) pair per thread in phase A");
  // MODE 2 reuses the block's LDS to stage its tables on the way out
  constexpr int NS = 9 * sym_blocks<NEN>();  // symmetric tangent values per element
  constexpr int SP = NS + 1;                 // odd stride between staged elements spreads the LDS banks
  constexpr int LA = NA * NPT, LP = 9 * NPT, LG = NQ * NEN * 3 * E;
  constexpr int LST = MODE == 2 ? E * (SP + ND) : 0;
  __shared__ double lds[LA + LP + LG > LST ? LA + LP + LG : LST];
  double* sA = lds;       // w AA: [SYM9(3i+J, 3k+L)][t] or [3i+J][3k+L][t]
  double* sP = lds + LA;  // w P_iJ: [3i+J][t]
  double(*sG)[NEN][3][E] = reinterpret_cast<double(*)[NEN][3][E]>(lds + LA + LP);
  const int tid = threadIdx.x;
  const int64_t eb = e_begin + xcd_swizzle(blockIdx.x, gridDim.x) * E;
  const int64_t e_end = e_begin + e_count;
  const int64_t n = n_el * NQ;

  // this thread's shape-gradient value of every point slice: (b, J, le);
  // with GI the phase-A threads recompute them from the node coordinates
  const int g_le = tid % E, g_J = (tid / E) % 3, g_b = tid / (3 * E);
  const int64_t g_e = eb + g_le;
  double gv[NQ];
  if constexpr (!GI) {
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      gv[q] = (g_e < e_end) ? dNdX[(((int64_t)q * NEN + g_b) * 3 + g_J) * n_el + g_e] : 0.0;
  }

  // phase A: (point t = q * E + le, row i)
  if (tid < 3 * NPT) {
    const int i = tid % 3, t = tid / 3;
    const int le = t % E, q = t / E;
    const int64_t e = eb + le;
    double Fm[9], S[6], Cc[21], wq = 0.0;
    if (e < e_end) {
      const int64_t pt = (int64_t)q * n_el + e;
#pragma unroll
      for (int c = 0; c < 9; ++c) Fm[c] = F[(int64_t)c * n + pt];
#pragma unroll
      for (int c = 0; c < 6; ++c) S[c] = SC[(int64_t)c * n + pt];
#pragma unroll
      for (int c = 0; c < 21; ++c) Cc[c] = SC[(int64_t)(6 + c) * n + pt];
      if constexpr (GI) {
        // the isoparametric map of this point; row i writes column J = i of
        // the shape gradients
        double dN[NEN][3], inv[3][3], wr;
        const double det = geom_jac<NEN>(
            q, [&](int a, int J) { return X[J * n_nodes + conn[(int64_t)a * n_el + e]]; }, dN, inv, wr);
        wq = wr * det;
#pragma unroll
        for (int a = 0; a < NEN; ++a) sG[q][a][i][le] = shape_grad(inv, dN[a], i);
      } else {
        wq = w[pt];
      }
    } else {
      if constexpr (GI) {
#pragma unroll
        for (int a = 0; a < NEN; ++a) sG[q][a][i][le] = 0.0;
      }
#pragma unroll
      for (int c = 0; c < 9; ++c) Fm[c] = 0.0;
#pragma unroll
      for (int c = 0; c < 6; ++c) S[c] = 0.0;
#pragma unroll
      for (int c = 0; c < 21; ++c) Cc[c] = 0.0;
    }
    // row i of F scaled by 4 w (tangent) and 2 w (stress and the S~ term)
    const double w2 = 2.0 * wq, w4 = 4.0 * wq;
    double Fi[3], Fi4[3];
#pragma unroll
    for (int I = 0; I < 3; ++I) {
      Fi[I] = (i == 0) ? Fm[I] : (i == 1) ? Fm[3 + I] : Fm[6 + I];
      Fi4[I] = w4 * Fi[I];
    }
#pragma unroll
    for (int J = 0; J < 3; ++J) {
      sP[(3 * i + J) * NPT + t] = w2 * (Fi[0] * S[VI(0, J)] + Fi[1] * S[VI(1, J)] + Fi[2] * S[VI(2, J)]);
      // Y_KL = 4 w sum_I F_iI CC~_IJKL
      double Y[3][3];
#pragma unroll
      for (int K = 0; K < 3; ++K)
#pragma unroll
        for (int L = 0; L < 3; ++L)
          Y[K][L] = Fi4[0] * Cc[TRI(VI(0, J), VI(K, L))] + Fi4[1] * Cc[TRI(VI(1, J), VI(K, L))] +
                    Fi4[2] * Cc[TRI(VI(2, J), VI(K, L))];
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int L = 0; L < 3; ++L) {
          // w AA_iJkL = 2 w delta_ik S~_JL + F_kK Y_KL
          double v = (k == i) ? w2 * S[VI(J, L)] : 0.0;
          v = fma(Fm[3 * k], Y[0][L], v);
          v = fma(Fm[3 * k + 1], Y[1][L], v);
          v = fma(Fm[3 * k + 2], Y[2][L], v);
          const int al = 3 * i + J, be = 3 * k + L;
          if constexpr (SYMA) {
            if (al <= be) sA[SYM9(al, be) * NPT + t] = v;
          } else {
            sA[(al * 9 + be) * NPT + t] = v;
          }
        }
    }
  }
  if constexpr (!GI) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) sG[q][g_b][g_J][g_le] = gv[q];
  }
  __syncthreads();

  // phase B: thread (row i, node a, element le), i outermost
  const int le = tid % E, a = (tid / E) % NEN, i = tid / (E * NEN);
  const int rho = 3 * a + i;
  const int64_t e = eb + le;
  // MODE 2 accumulates row i of the blocks node a owns (sym_slot), the
  // others full rows of K_e
  constexpr int HN = NEN / 2;
  constexpr int NACC = MODE == 2 ? 3 * (HN + 1) : ND;
  double acc[NACC];
#pragma unroll
  for (int c = 0; c < NACC; ++c) acc[c] = 0.0;
  double rr = 0.0;
  // IC::value >= 0: the row is that constant; otherwise it is i
  auto points = [&](auto ic) {
    constexpr int IC = decltype(ic)::value;
    const int ii = IC >= 0 ? IC : i;
#pragma unroll 1
    for (int q = 0; q < NQ; ++q) {
      const int lq = q * E + le;
      double ga[3];
#pragma unroll
      for (int J = 0; J < 3; ++J) ga[J] = sG[q][a][J][le];
      rr += sP[(3 * ii) * NPT + lq] * ga[0] + sP[(3 * ii + 1) * NPT + lq] * ga[1] + sP[(3 * ii + 2) * NPT + lq] * ga[2];
      double T[9];  // T_kL = w AA_iJkL G^a_J
#pragma unroll
      for (int c = 0; c < 9; ++c) {
        double x = 0.0;
#pragma unroll
        for (int J = 0; J < 3; ++J) {
          const int idx = (IC >= 0) ? SYM9(3 * IC + J, c) : (3 * ii + J) * 9 + c;
          x += sA[idx * NPT + lq] * ga[J];
        }
        T[c] = x;
      }
      // three multiply-adds straight into the accumulator per entry
      auto add_block = [&](int c, double h0, double h1, double h2) {
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) {
          double x = acc[c + kk];
          x = fma(T[3 * kk], h0, x);
          x = fma(T[3 * kk + 1], h1, x);
          acc[c + kk] = fma(T[3 * kk + 2], h2, x);
        }
      };
      if constexpr (MODE == 2) {
#pragma unroll
        for (int d = 0; d <= HN; ++d) {
          const int b = a + d < NEN ? a + d : a + d - NEN;
          add_block(3 * d, sG[q][b][0][le], sG[q][b][1][le], sG[q][b][2][le]);
        }
      } else {
#pragma unroll
        for (int b = 0; b < NEN; ++b) add_block(3 * b, sG[q][b][0][le], sG[q][b][1][le], sG[q][b][2][le]);
      }
    }
  };
  if constexpr (SYMA) {
    const int iu = __builtin_amdgcn_readfirstlane(i);
    if (iu == 0)
      points(Int<0>{});
    else if (iu == 1)
      points(Int<1>{});
    else
      points(Int<2>{});
  } else {
    points(Int<-1>{});
  }
  if constexpr (MODE == 2) {
    // stage the block's tables in LDS (after every wave has left the point
    // loop), then write them out contiguously: the E elements of a block are
    // consecutive in the element-major tables
    static_assert(E * ND == NT, "one staged residual value per thread");
    double* stK = lds;           // [E][SP]
    double* stR = lds + E * SP;  // [E][ND]
    __syncthreads();
#pragma unroll
    for (int d = 0; d <= HN; ++d) {
      if (d < HN || a < HN) {
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) stK[le * SP + sym_slot<NEN>(a, d) * 9 + 3 * i + kk] = acc[3 * d + kk];
      }
    }
    stR[le * ND + rho] = rr;
    __syncthreads();
    const int64_t nvalid = e_end - eb < E ? e_end - eb : E;
    if (tid < nvalid * ND) r_e[eb * ND + tid] = stR[tid];
    double* dst = K_e + eb * NS;
    for (int t = tid; t < nvalid * NS; t += NT) dst[t] = stK[(t / NS) * SP + t % NS];
    return;
  }
  if (e >= e_end) return;
  if constexpr (MODE == 0) {
    r_e[(int64_t)rho * n_el + e] = rr;
    if (K_e) {
#pragma unroll
      for (int c = 0; c < ND; ++c) K_e[((int64_t)rho * ND + c) * n_el + e] = acc[c];
    }
  } else {
    const int64_t R = 3 * (int64_t)conn[(int64_t)a * n_el + e] + i;
    if (r) r[R] += rr;
    if (vals) {
      const int64_t base = row_ptr[R];
#pragma unroll
      for (int b = 0; b < NEN; ++b) {
        const int32_t off = e2csr[(e * NEN + a) * NEN + b];
        if (off < 0) continue;
        vals[base + off] += acc[3 * b];
        vals[base + off + 1] += acc[3 * b + 1];
        vals[base + off + 2] += acc[3 * b + 2];
      }
    }
  }
}

// ---------------------------------------------------------------- gather assembly
// One wave per node i: rows 3i..3i+2 of the CSR values and of r are the sums,
// over the node's (element e, local node a) pairs in incidence order
// (ascending e), of rows 3a..3a+2 of K_e and r_e (element-major tables, K_e
// in symmetric node blocks, see sym_slot).  The
// three rows are accumulated in LDS and written once, contiguously (the rows
// of one node share one column pattern and follow each other in CSR), so
// every CSR value is written exactly once: no colouring, no atomics, no
// clearing pass, bitwise reproducible.  Lane t of a round adds entry t of the
// element's 3 x nd block; targets within one element are distinct, and the
// LDS operations of one wave complete in issue order, so elements are summed
// one after another.
template <int NEN>
__global__ void __launch_bounds__(256) k_gather_assemble(
    int64_t n_nodes, const int64_t* __restrict__ inc_ptr, const int32_t* __restrict__ inc_ent,
    const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ e2csr, const double* __restrict__ Kw,
    const double* __restrict__ rw, double* __restrict__ r, double* __restrict__ vals, int max_row) {
  constexpr int ND = 3 * NEN, NB = 3 * ND, R = (NB + 63) / 64;
  constexpr int NS = 9 * sym_blocks<NEN>(), HN = NEN / 2;
  constexpr int GB = 4;  // elements whose loads are in flight together (measured: 4 beat 8 and 16)
  extern __shared__ double lds[];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t node = (int64_t)blockIdx.x * (blockDim.x / 64) + wv;
  if (node >= n_nodes) return;  // the whole wave leaves; the kernel has no block barrier
  double* acc = lds + (int64_t)wv * 3 * max_row;
  const int64_t rb = row_ptr[3 * node];
  const int len = (int)(row_ptr[3 * node + 1] - rb);
  if (len > max_row) return;  // caller's bound is wrong: leave the rows untouched rather than overrun LDS
  for (int t = lane; t < 3 * len; t += 64) acc[t] = 0.0;
  // the entry t handled by this lane in round rr: row ii, node block b, column kk
  int tb[R], tl[R], tik[R];
#pragma unroll
  for (int rr = 0; rr < R; ++rr) {
    const int t = lane + 64 * rr;
    const int ii = t / ND, c = t % ND;
    tb[rr] = c / 3;
    tl[rr] = ii * len + c % 3;
    tik[rr] = (ii << 2) | (c % 3);
  }
  double racc = 0.0;
  const int64_t k0 = inc_ptr[node], k1 = inc_ptr[node + 1];
  for (int64_t kc = k0; kc < k1; kc += 64) {
    const int cnt = (int)((k1 - kc) < 64 ? (k1 - kc) : 64);
    const int32_t mine = lane < cnt ? inc_ent[kc + lane] : 0;
    auto load = [&](int j, double (&vv)[R], int (&oo)[R], double& rv) {
      const int32_t ea = __builtin_amdgcn_readlane(mine, j);
      const int64_t e = ea / NEN;
      const int a = ea - (int)e * NEN;
      const double* src = Kw + e * NS;
      const int32_t* off = e2csr + (int64_t)ea * NEN;
#pragma unroll
      for (int rr = 0; rr < R; ++rr) {
        const int t = lane + 64 * rr;
        if (t < NB) {
          // entry (ii, kk) of block (a, b): stored in a's slot, or transposed in b's
          const int b = tb[rr], ii = tik[rr] >> 2, kk = tik[rr] & 3;
          const int d = b >= a ? b - a : b - a + NEN;
          const bool own = d < HN || (d == HN && a < HN);
          const int k = own ? sym_slot<NEN>(a, d) * 9 + 3 * ii + kk : sym_slot<NEN>(b, NEN - d) * 9 + 3 * kk + ii;
          vv[rr] = src[k];
          oo[rr] = off[b];
        }
      }
      rv = lane < 3 ? rw[e * ND + 3 * a + lane] : 0.0;
    };
    // all loads of a batch of elements are in flight together; the batch is
    // then added in incidence order with LDS adds that return nothing (one
    // wave's LDS operations complete in issue order, and the lanes of one
    // add target distinct entries, so the sums are formed in a fixed order)
    for (int j0 = 0; j0 < cnt; j0 += GB) {
      double v[GB][R], rv[GB];
      int o[GB][R];
#pragma unroll
      for (int jj = 0; jj < GB; ++jj)
        if (j0 + jj < cnt) load(j0 + jj, v[jj], o[jj], rv[jj]);
#pragma unroll
      for (int jj = 0; jj < GB; ++jj) {
        if (j0 + jj >= cnt) break;
        racc += rv[jj];
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
          const int t = lane + 64 * rr;
          if (t < NB && o[jj][rr] >= 0) atomicAdd(&acc[tl[rr] + o[jj][rr]], v[jj][rr]);
        }
      }
    }
  }
  if (vals)
    for (int t = lane; t < 3 * len; t += 64) vals[rb + t] = acc[t];
  if (r && lane < 3) r[3 * node + lane] = racc;
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
// One launch per colour; thread = (element of the colour, element row),
// element fastest so the SoA element tables are read coalesced.
template <int NEN>
__global__ void __launch_bounds__(256) k_assemble(int64_t e_begin, int64_t e_count, const int32_t* __restrict__ perm,
                                                  int64_t n_el, const int32_t* __restrict__ conn,
                                                  const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ e2csr,
                                                  const double* __restrict__ r_e, const double* __restrict__ K_e,
                                                  double* __restrict__ r, double* __restrict__ vals) {
  constexpr int ND = 3 * NEN;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= e_count * ND) return;
  const int64_t pos = e_begin + t % e_count;
  const int rho = (int)(t / e_count);
  const int64_t e = perm ? (int64_t)perm[pos] : pos;
  const int a = rho / 3, i = rho % 3;
  const int64_t R = 3 * (int64_t)conn[(int64_t)a * n_el + e] + i;
  if (r) r[R] += r_e[(int64_t)rho * n_el + e];
  if (vals) {
    const int64_t base = row_ptr[R];
#pragma unroll
    for (int b = 0; b < NEN; ++b) {
      const int32_t off = e2csr[(e * NEN + a) * NEN + b];
      if (off < 0) continue;  // column not in the pattern (cannot happen for a pattern built from conn)
      const int64_t p = base + off;
      vals[p] += K_e[((int64_t)rho * ND + 3 * b) * n_el + e];
      vals[p + 1] += K_e[((int64_t)rho * ND + 3 * b + 1) * n_el + e];
      vals[p + 2] += K_e[((int64_t)rho * ND + 3 * b + 2) * n_el + e];
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

int launch_gather_F(int nen, int nq, int64_t n_el, int64_t n_nodes, const int32_t* conn, const double* dNdX,
                    const double* X, const double* u, double* F, int nsv, const ModelConst* mc, double* K,
                    int32_t* n_bad, hipStream_t s) {
  if (n_el == 0) return 0;
  const unsigned grid = nblocks(n_el * nq, 256);
  const ModelConst m0 = mc ? *mc : ModelConst{};
  if (!K) nsv = -1;
#define PA_GF(NEN_, GI_, NSV_) \
  k_gather_F<NEN_, GI_, NSV_><<<grid, 256, 0, s>>>(n_el, n_nodes, conn, dNdX, X, u, F, m0, K, n_bad)
#define PA_GF_NSV(NEN_, GI_)          \
  switch (nsv) {                      \
    case -1: PA_GF(NEN_, GI_, -1); break; \
    case 0: PA_GF(NEN_, GI_, 0); break;   \
    case 1: PA_GF(NEN_, GI_, 1); break;   \
    case 2: PA_GF(NEN_, GI_, 2); break;   \
    default: return -1;               \
  }
  if (nen == 8) {
    if (X) PA_GF_NSV(8, true) else PA_GF_NSV(8, false)
  } else if (nen == 10) {
    if (X) PA_GF_NSV(10, true) else PA_GF_NSV(10, false)
  } else {
    return -1;
  }
#undef PA_GF_NSV
#undef PA_GF
  return 0;
}
int launch_chain_integrate(int nen, int64_t n_el, int64_t e_begin, int64_t e_count, const int32_t* conn,
                           const double* dNdX, const double* w, int64_t n_nodes, const double* X, const double* F,
                           const double* SC, double* r_e, double* K_e, const int64_t* row_ptr, const int32_t* e2csr,
                           double* r, double* vals, int mode, hipStream_t s) {
  if (e_count == 0) return 0;
#define PA_INTEGRATE_GI(NEN_, GI_)                                                                                 \
  {                                                                                                                \
    const unsigned grid = nblocks(e_count, integrate_elems<NEN_>());                                               \
    constexpr int nt = integrate_threads<NEN_>();                                                                  \
    if (mode == 1)                                                                                                 \
      k_chain_integrate<NEN_, 1, GI_><<<grid, nt, 0, s>>>(n_el, e_begin, e_count, conn, dNdX, w, n_nodes, X, F,    \
                                                          SC, r_e, K_e, row_ptr, e2csr, r, vals);                 \
    else if (mode == 2)                                                                                            \
      k_chain_integrate<NEN_, 2, GI_><<<grid, nt, 0, s>>>(n_el, e_begin, e_count, conn, dNdX, w, n_nodes, X, F,    \
                                                          SC, r_e, K_e, row_ptr, e2csr, r, vals);                 \
    else                                                                                                           \
      k_chain_integrate<NEN_, 0, GI_><<<grid, nt, 0, s>>>(n_el, e_begin, e_count, conn, dNdX, w, n_nodes, X, F,    \
                                                          SC, r_e, K_e, row_ptr, e2csr, r, vals);                 \
  }
#define PA_INTEGRATE(NEN_)            \
  if (X) PA_INTEGRATE_GI(NEN_, true)  \
  else PA_INTEGRATE_GI(NEN_, false)
  if (nen == 8) PA_INTEGRATE(8)
  else if (nen == 10) PA_INTEGRATE(10)
  else return -1;
#undef PA_INTEGRATE_GI
#undef PA_INTEGRATE
  return 0;
}

int launch_gather_assemble(int nen, int64_t n_nodes, const int64_t* inc_ptr, const int32_t* inc_ent,
                           const int64_t* row_ptr, const int32_t* e2csr, const double* Kw, const double* rw,
                           double* r, double* vals, int max_row, hipStream_t s) {
  if (n_nodes == 0) return 0;
  const size_t lds = (size_t)4 * 3 * max_row * sizeof(double);
  if (lds > 64 * 1024) return -1;
  PA_NEN_SWITCH(nen,
                (k_gather_assemble<8><<<nblocks(n_nodes, 4), 256, lds, s>>>(n_nodes, inc_ptr, inc_ent, row_ptr, e2csr, Kw, rw, r, vals, max_row)),
                (k_gather_assemble<10><<<nblocks(n_nodes, 4), 256, lds, s>>>(n_nodes, inc_ptr, inc_ent, row_ptr, e2csr, Kw, rw, r, vals, max_row)));
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

int launch_residual_cotangent(int nen, int64_t n_el, const int32_t* conn, const double* dNdX, const double* w,
                              const double* rbar, double* Pbar, hipStream_t s) {
  if (n_el == 0) return 0;
  const int nq = nen == 8 ? 8 : 4;
  PA_NEN_SWITCH(nen, (k_residual_cotangent<8><<<nblocks(n_el * nq, 256), 256, 0, s>>>(n_el, conn, dNdX, w, rbar, Pbar)),
                (k_residual_cotangent<10><<<nblocks(n_el * nq, 256), 256, 0, s>>>(n_el, conn, dNdX, w, rbar, Pbar)));
  return 0;
}

int loss_partial_blocks(int64_t n_rows) {
  const int64_t b = (n_rows + LOSS_BLOCK - 1) / LOSS_BLOCK;
  return (int)(b < 1024 ? (b > 0 ? b : 1) : 1024);
}

int launch_residual_loss(int64_t n_rows, const double* r, const int32_t* group, int n_groups, const double* R,
                         double* partials, double* sums, double* loss, double* rbar, hipStream_t s) {
  if (n_groups < 0 || n_groups > 63) return -1;
  const int nb = loss_partial_blocks(n_rows);
  k_loss_partials<<<nb, LOSS_BLOCK, 0, s>>>(n_rows, r, group, n_groups, partials);
  k_loss_finish<<<1, 64, 0, s>>>(nb, n_groups, partials, R, sums, loss);
  if (rbar && n_rows > 0) k_loss_rbar<<<nblocks(n_rows, 256), 256, 0, s>>>(n_rows, n_groups, r, group, R, sums, rbar);
  return 0;
}

int launch_fill(double* x, int64_t n, double v, hipStream_t s) {
  if (n == 0) return 0;
  const int64_t b = (n + 255) / 256;
  k_fill<<<(unsigned)(b < 65536 ? b : 65536), 256, 0, s>>>(x, n, v);
  return 0;
}

}  // namespace pa
