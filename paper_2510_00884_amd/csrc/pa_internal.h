// Internal host/device interface of the library: prepared-parameter layout
// and kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "kinematics.h"

namespace pa {

// Byte offsets into the prepared-parameter buffer (one per model).
//   hdr:   N0 (double), kappa[3] (double)
//   d_*:   FP64 tables, f_*: FP32 tables
//          a[H], c[L][H] (hidden biases, layer k at k-1), W1t[P][H] (W1
//          transposed), Bt[L][P][H] (skip weights B_k transposed, k >= 2), b[P]
//   x_*:   FP64 matrix-core fragments, y_*: FP32 fragments, z_*: BF16 fragments
//          W1 [MB][S1][64], A [L][MB][SH][64], B [L][MB][S1][64]
//          (bf16: [..][64][8] with SHB/1 K steps)
//          AT (reverse products): lane (i, g) of step s holds A_k[4s + g][16w + i]
//   k0, nout: scratch used to evaluate the network at K = 0 (normalisation)
struct PrepLayout {
  int32_t H, L, P, MB, S1, SH, SHB, NOUT;
  int32_t HR;  // real width (H is the width of the zero-padded tables)
  int64_t hdr;
  int64_t d_a, d_b, d_c, d_W1t, d_Bt;
  int64_t f_a, f_c, f_W1t, f_Bt;
  int64_t x_W1, x_A, x_B;
  int64_t y_W1, y_A, y_B;
  int64_t z_W1, z_A, z_B;
  int64_t x_AT, y_AT;   // transposed hidden weights for reverse products [L][MB][SH][64]
  int64_t x_G1, y_G1;   // layer-1 Gram table W1_rm W1_rn as MFMA A fragments [NPB][MB][4][64]
  int64_t x_ATp, y_ATp; // transposed hidden weights, K steps in accumulator-row order [L][MB][SH][64]
  // BF16 fragments of the all-BF16 adjoint form, K in the permuted neuron
  // order of the 16x16x32 products (position 8g + e of step t: neuron
  // 32t + 4g + e, e < 4; 32t + 16 + 4g + e - 4, e >= 4), [..][64][8]:
  int64_t w_AT;  // [L][MB][SHB]: lane (i, g) of row block mb holds A_k[neuron][16 mb + i]
  int64_t w_GT;  // [L][SHB]: row i = input: W1[neuron][i] (k = 1), B_k[neuron][i]
  int64_t w_G1;  // [NPB][SHB]: row i = packed pair 16 pb + i: W1[neuron][m] W1[neuron][n]
  int64_t d_Am, f_Am;  // A_k row-major [L][H][H] (layer k at k - 1), FP64 and FP32
  int64_t x_GT, y_GT;  // gradient products [L][SH][64], lane (i, g) of step s = 4 mb + v: W1[r][i] (layer 1)
                       // or B_k[r][i], r = 16 mb + row(g, v) (row64 for x_, row32 for y_), zero for i >= P
  int64_t x_AW;        // FP64 [P][MB][SH][64]: layer-2 Jacobian column tables A_2 diag(W1[:, m]),
                       // lane (i, g) of step s = 4 mb + v: A_2[16 ob + i][q] W1[q][m], q = 16 mb + g + 4 v
  int64_t k0, nout;
  int64_t total;
};

// Offsets into the FP64 parameter vector theta.
struct ThetaLayout {
  int32_t H, L, P, has_bias;
  int64_t W1, c1;     // c1 < 0 when absent
  int64_t A[5], B[5], c[5];  // per layer k (index k), 2 <= k <= 4
  int64_t a, b, total;
};

PrepLayout prep_layout(int H, int L, int P);
// Widths below 16 run on one 16-row matrix-core tile: the prepared tables
// hold the network zero-padded to 16 neurons (padded neurons have zero
// incoming, outgoing and output weights, so they change no output).
inline int padded_width(int h) { return h < 16 ? 16 : h; }
// Forward-mode (Alg. 4) kernels exist for 2-3 hidden layers; the
// adjoint-form kernels also for 4.
bool mlp_fwd_supported(int H, int L, int P);

// Inner functions other than the MICNN (closed.hip); values match pa_model_kind.
enum { MODEL_MICNN = 0, MODEL_CANN = 1, MODEL_GENT_THOMAS = 2 };
struct ClosedLayout {
  int64_t hdr, theta, total;  // header (N(0), kappa), parameters
};
inline int closed_num_params(int kind, int p) { return kind == MODEL_CANN ? 8 * p : 3; }
inline ClosedLayout closed_layout(int kind, int p) {
  ClosedLayout c{};
  c.hdr = 0;
  c.theta = 256;
  c.total = 256 + ((8 * (int64_t)closed_num_params(kind, p) + 255) & ~int64_t(255));
  return c;
}
int launch_prepare_closed(int kind, int p, int n_params, const double* theta, unsigned char* prep, int normalize,
                          int npair, hipStream_t s);
int launch_inner_closed(int kind, int p, const unsigned char* prep, int npair, int64_t n, const double* K,
                        double* out, int hess, hipStream_t s);
ThetaLayout theta_layout(int H, int L, int P, int has_bias);

// kinematics / chain (kin_chain.hip)
int launch_invariants(int nsv, int64_t n, const double* F, const ModelConst& mc, double* I_raw,
                      double* K, double* dKdF, int32_t* n_bad, hipStream_t s);
// F (and the outputs of the chain kernels) with leading dimension ld >= n:
// n points of a batch of a longer call; K and Nout are [..][n].
int launch_features(int nsv, int64_t n, int64_t ld, const double* F, const ModelConst& mc, double* K,
                    int32_t* n_bad, hipStream_t s);
int launch_pipe_probe(int kind_lo, int kind_hi, int iters, int blocks, double* out, hipStream_t s);
int launch_material_cc(int nsv, int64_t n, const double* F, const double* Nout, const ModelConst& mc,
                       double* SC, hipStream_t s);
int launch_chain_voigt(int nsv, int64_t n, int64_t ld, const double* F, const double* Nout, const double* N0,
                       const ModelConst& mc, double* psi, double* tau, double* cc, hipStream_t s);
int launch_chain(int nsv, int64_t n, int64_t ld, const double* F, const double* Nout, const double* N0,
                 const ModelConst& mc, double* psi, double* P, double* A, int32_t* n_bad, hipStream_t s);

// network (mlp.hip)
bool mlp_supported(int H, int L, int P);
int launch_prepare(const PrepLayout& lay, const ThetaLayout& tl, const double* theta,
                   unsigned char* prep, int normalize, int npair, hipStream_t s);
int launch_mlp(const PrepLayout& lay, int prec, int algo, const unsigned char* prep, int64_t n,
               const double* K, double* out, int hess, hipStream_t s);
// per-width instantiations (mlp_fwd_h*.hip, mlp_adj_h*.hip)
#define PA_MLP_LAUNCHER(name)                                                                                 \
  int name(const PrepLayout& lay, int prec, const unsigned char* prep, int64_t n, const double* K, double* out, \
           int hess, hipStream_t s);
PA_MLP_LAUNCHER(launch_mlp_fwd_h16)
PA_MLP_LAUNCHER(launch_mlp_fwd_h32)
PA_MLP_LAUNCHER(launch_mlp_fwd_h64)
PA_MLP_LAUNCHER(launch_mlp_adj_h16)
PA_MLP_LAUNCHER(launch_mlp_adj_h32)
PA_MLP_LAUNCHER(launch_mlp_adj_h64)
PA_MLP_LAUNCHER(launch_mlp_valu)
#undef PA_MLP_LAUNCHER

// parameter adjoint (adjoint.hip)
int64_t param_backward_ws(int H, int L, int P, int prec, int64_t n);
int launch_param_backward(const PrepLayout& lay, const ThetaLayout& tl, int nsv, int prec,
                          const unsigned char* prep, const ModelConst& mc, int64_t n, const double* F,
                          const double* P_bar, double* theta_bar, unsigned char* ws, hipStream_t s);

// elements and assembly (fe.hip)
int launch_geometry(int nen, int64_t n_el, int64_t n_nodes, const double* X, const int32_t* conn,
                    double* dNdX, double* w, int32_t* n_bad, hipStream_t s);
// X [3][n_nodes] may be NULL; when given, the kernels recompute the shape
// gradients and weights from it instead of reading dNdX and w
// nsv >= 0 with K non-NULL: also the network inputs K [p][n] and the
// inverted-point count (the features kernel's outputs)
int launch_gather_F(int nen, int nq, int64_t n_el, int64_t n_nodes, const int32_t* conn, const double* dNdX,
                    const double* X, const double* u, double* F, int nsv, const ModelConst* mc, double* K,
                    int32_t* n_bad, hipStream_t s);
int launch_chain_integrate(int nen, int64_t n_el, int64_t e_begin, int64_t e_count, const int32_t* conn,
                           const double* dNdX, const double* w, int64_t n_nodes, const double* X, const double* F,
                           const double* SC, double* r_e, double* K_e, const int64_t* row_ptr, const int32_t* e2csr,
                           double* r, double* vals, int mode, hipStream_t s);
int launch_gather_assemble(int nen, int64_t n_nodes, const int64_t* inc_ptr, const int32_t* inc_ent,
                           const int64_t* row_ptr, const int32_t* e2csr, const double* Kw, const double* rw,
                           double* r, double* vals, int max_row, hipStream_t s);
int launch_csr_map(int nen, int64_t n_el, const int32_t* conn, const int64_t* row_ptr,
                   const int32_t* col, int32_t* e2csr, hipStream_t s);
int launch_assemble(int nen, int64_t e_begin, int64_t e_count, const int32_t* perm, int64_t n_el,
                    const int32_t* conn, const int64_t* row_ptr, const int32_t* e2csr,
                    const double* r_e, const double* K_e, double* r, double* vals, hipStream_t s);
int launch_fill(double* x, int64_t n, double v, hipStream_t s);
int launch_residual_cotangent(int nen, int64_t n_el, const int32_t* conn, const double* dNdX, const double* w,
                              const double* rbar, double* Pbar, hipStream_t s);
int loss_partial_blocks(int64_t n_rows);
int launch_residual_loss(int64_t n_rows, const double* r, const int32_t* group, int n_groups, const double* R,
                         double* partials, double* sums, double* loss, double* rbar, hipStream_t s);

}  // namespace pa
