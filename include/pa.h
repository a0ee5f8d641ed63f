/*
 * pa.h -- C ABI of the MI355X (gfx950) neural-constitutive finite-element
 * hot path (COMMET, arXiv 2510.00884).
 *
 * The library evaluates an invariant-based input-convex neural strain energy
 * Psi at every quadrature point together with its first Piola-Kirchhoff
 * stress P = dPsi/dF and tangent AA = d2Psi/dFdF, integrates element residuals
 * and stiffnesses, scatter-assembles them into CSR by element colouring, and
 * differentiates a stress-calibration loss with respect to the network
 * parameters.
 *
 * Conventions (all entry points)
 * ------------------------------
 * - Pointers are DEVICE pointers unless the comment says "host".  The caller
 *   owns every buffer; the library never allocates on the hot path.  Scratch
 *   memory is passed in as a workspace whose size a *_workspace_bytes helper
 *   reports.
 * - Arrays are structure-of-arrays (SoA): X[component][index], index fastest.
 * - F is row-major per point: F[3*i + J] = F_iJ.  The tangent is
 *   AA[9*(3*i+J) + (3*k+L)] = d2Psi/dF_iJ dF_kL.
 * - Every call is asynchronous on `stream` (a hipStream_t, NULL = default
 *   stream).  Nothing synchronises.  Calls on one stream are ordered.
 * - Argument and shape errors are detected on the host before any launch and
 *   return PA_ERR_ARG without writing anything; pa_last_error() describes the
 *   problem.  A failed launch returns PA_ERR_HIP.  Numerical trouble does not
 *   return an error (that would need a synchronisation): points with J <= 0 or
 *   non-finite values increment *n_bad when n_bad is non-NULL; J = 0 or
 *   non-finite input yields non-finite output.
 * - Inputs and outputs are FP64 in every precision mode; the precision enum
 *   selects the arithmetic of the network contractions only.  Kinematics,
 *   det F, the volumetric terms and the tangent handed to Newton are FP64.
 */
#ifndef PA_H
#define PA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PA_OK = 0,
  PA_ERR_ARG = -1,         /* bad argument or shape; nothing was launched     */
  PA_ERR_UNSUPPORTED = -2, /* no kernel for this width / depth / inputs        */
  PA_ERR_HIP = -3,         /* HIP runtime reported an error at launch          */
  PA_ERR_WORKSPACE = -4    /* workspace NULL or smaller than required          */
} pa_status;

/* Arithmetic of the inner-network contractions (matrix cores).  Every mode
 * takes and returns FP64 arrays; kinematics, chain rule and elements are FP64. */
typedef enum {
  PA_FP64 = 0,      /* FP64 MFMA                                              */
  PA_FP32 = 1,      /* FP32 MFMA, FP32 activations                            */
  PA_BF16 = 2,      /* every contraction (value, gradient and Hessian) on
                       BF16 MFMA inputs with FP32 accumulation and FP32
                       activations                                           */
  PA_BF16_CORR = 3, /* the PA_BF16 pass, then a correction pass that
                       recomputes the value and first-derivative columns with
                       FP32 MFMA and overwrites them; the second-derivative
                       columns keep the BF16 result (both algorithms)         */
  PA_BF16_JAC = 4   /* one mixed pass, PA_ALGO_ADJOINT only: value, reverse
                       sweep, gradient and layer-1 Hessian term in FP32, the
                       Jacobians of layers >= 2 (the bulk of the Hessian work)
                       on the BF16 matrix cores                              */
} pa_precision;

/* How the network's input Hessian is formed.  Both give the same numbers up
 * to rounding order. */
typedef enum {
  PA_ALGO_FORWARD = 0, /* one-pass forward mode of App. B.2 Alg. 4: value,
                          gradient and Hessian columns carried layer by layer */
  PA_ALGO_ADJOINT = 1  /* value forward, value adjoint backward, then the
                          Jacobian forward accumulating the Hessian as
                          sum_k J_k^T diag(lambda_k F''(y_k)) J_k; every
                          precision (PA_BF16 and PA_BF16_CORR: two or three
                          hidden layers)                                      */
} pa_algorithm;

typedef enum { PA_ACT_SOFTPLUS = 0 } pa_activation;

/* Inner function of the constitutive model.  PA_MODEL_MICNN: the network of
 * eq. icnn (width, n_hidden, activation, has_bias, algorithm apply).
 * PA_MODEL_CANN: the CANN of App. B.1 (eq. cann-def) with f0 = identity and,
 * per input, the branches (power 1, linear), (power 2, linear), (power 1,
 * exp), (power 2, exp), each with an inner weight w1 and an outer weight w2
 * (theta: 8 per input, in that order, (w1, w2) per branch; f2 = w1 x or
 * exp(w1 x) - 1).  PA_MODEL_GENT_THOMAS: eq. (gt) on the isotropic
 * features, theta = (c1, c2, c3), N = c1 K1 + c2 ((2/3) log(K2 + 3^{3/2}) -
 * log 3) + c3 K3 ((0.5, 1, 1) is eq. gt).  For the last two, width,
 * n_hidden, activation, has_bias and algorithm are ignored, the precision
 * argument is accepted and the arithmetic is FP64, and the parameter
 * adjoint is not provided. */
typedef enum { PA_MODEL_MICNN = 0, PA_MODEL_CANN = 1, PA_MODEL_GENT_THOMAS = 2 } pa_model_kind;

/* Description of the neural constitutive model (host struct).
 * Kinematic layer (App. A.2 and App. C):
 *   K = [I1~ - 3, I2~^{3/2} - 3^{3/2}, (J-1)^2,
 *        {I4~_ij - A^i.A^j}_{i<=j}, {I5~_ij - A^i.A^j}_{i<=j}]
 * with isochoric invariants I~ = I * I3^{alpha}, alpha = -1/3 for I1, I4 and
 * -2/3 for I2, I5; p = 3 + 2*n_sv(n_sv+1)/2 inputs (3, 5 or 9).
 * Inner network: (M)ICNN of eq. (icnn), App. B.2, with L hidden layers of
 * width h and softplus activation.  Parameter vector (FP64), in this order:
 *   W1 (h x p row-major), c1 (h),
 *   for k = 2..L: A_k (h x h), B_k (h x p), c_k (h),
 *   a (h), b (p);
 * the c_k blocks are absent when has_bias = 0.
 * normalize = 1 subtracts N(0) and kappa_ij K_{4,ij},
 *   kappa_ij = dN/dK_{4,ij}(0) + 2 dN/dK_{5,ij}(0),
 * so that Psi(I) = 0 and P(I) = 0. */
typedef struct {
  int32_t n_sv;        /* number of structural vectors: 0, 1 or 2           */
  double  A[2][3];     /* reference structural vectors A^1, A^2              */
  int32_t n_hidden;    /* L: hidden layers, 2, 3 or 4 (4: PA_ALGO_ADJOINT
                        * with PA_FP64, PA_FP32 or PA_BF16_JAC, and the
                        * parameter adjoint; otherwise PA_ERR_UNSUPPORTED)  */
  int32_t width;       /* h: neurons per hidden layer: 1..16, 32 or 64.
                        * Widths below 16 run zero-padded to 16 neurons
                        * (same outputs, the cost of width 16)              */
  int32_t activation;  /* PA_ACT_SOFTPLUS                                    */
  int32_t normalize;   /* 1: energy- and stress-free reference state        */
  int32_t has_bias;    /* 1: hidden layers carry biases c_k                  */
  int32_t algorithm;   /* pa_algorithm used by the tangent entry points      */
  int32_t kind;        /* a pa_model_kind value; 0 = MICNN                    */
} pa_model_desc;

/* Finite-element mesh on the device.  nen/nq: 8/8 (hex8, 2x2x2 Gauss) or
 * 10/4 (tet10, 4-point rule).  Local node order and quadrature points follow
 * the element conventions documented with pa_mesh_geometry. */
typedef struct {
  int64_t n_el;          /* elements                                         */
  int64_t n_nodes;       /* nodes                                            */
  int32_t nen;           /* nodes per element (8 or 10)                      */
  int32_t nq;            /* quadrature points per element (8 or 4)           */
  const int32_t* conn;   /* [nen][n_el] node ids                             */
  const double*  dNdX;   /* [nq][nen][3][n_el] reference shape gradients     */
  const double*  w;      /* [nq][n_el] Gauss weight * det(dX/dxi)            */
  const double*  X;      /* [3][n_nodes] node coordinates, or NULL.  When
                          * given, the tangent-build kernels recompute the
                          * shape gradients and weights at each point from
                          * X (the same arithmetic as pa_mesh_geometry, so
                          * the same values) instead of reading dNdX and w,
                          * which saves 8(3 nen + 1) bytes of traffic per
                          * point and kernel; dNdX and w are still required
                          * by the other entry points. */
} pa_mesh;

/* CSR matrix over node-major dofs (dof = 3*node + i). */
typedef struct {
  int64_t n_rows;        /* 3 * n_nodes                                      */
  int64_t nnz;
  const int64_t* row_ptr;/* [n_rows + 1]                                     */
  const int32_t* col;    /* [nnz], sorted within each row                    */
  const int32_t* e2csr;  /* [n_el][nen][nen]: offset of column 3*conn[b]
                            within row 3*conn[a] (pa_element_csr_map)         */
} pa_csr;

/* Element colouring: no two elements of one colour share a node. */
typedef struct {
  int32_t n_colours;
  const int64_t* colour_ptr;  /* HOST [n_colours + 1]: ranges into elem_perm */
  const int32_t* elem_perm;   /* [n_el] element ids by colour; NULL = identity
                                 (elements already numbered colour by colour) */
} pa_colouring;

/* Node incidence for the gather assembly (pa_node_incidence). */
typedef struct {
  int64_t n_nodes;
  int64_t n_ent;         /* n_el * nen                                        */
  int32_t max_row;       /* >= the longest CSR row (3 x neighbours of a node)  */
  const int64_t* ptr;    /* [n_nodes + 1] into ent                            */
  const int32_t* ent;    /* [n_ent] e * nen + a, ascending e within a node     */
} pa_incidence;

/* ---------------------------------------------------------------- model */
int32_t pa_num_inputs(const pa_model_desc* desc);
int64_t pa_num_params(const pa_model_desc* desc);
/* 1 if kernels exist for this (width, depth, inputs) with at least one
 * algorithm, else 0 (depth 4: the adjoint form only). */
int32_t pa_supported(const pa_model_desc* desc);
/* Bytes of the prepared-parameter buffer. */
size_t  pa_prepared_bytes(const pa_model_desc* desc);
/* Converts the FP64 parameter vector theta (device, pa_num_params entries)
 * into the device-resident form used by every precision (matrix-core
 * fragment order, FP64/FP32/BF16 copies) and, if desc->normalize, evaluates
 * the network at K = 0 on the device to fold the reference-state constants.
 * `prepared` must hold pa_prepared_bytes(desc) bytes.  theta may be freed
 * once the stream has passed this call. */
int pa_prepare_params(const pa_model_desc* desc, const double* theta, void* prepared,
                      void* stream);

/* ---------------------------------------------------------------- material */
/* Invariants and features (eq. standard-inv-I, App. A.2.1-A.2.2, App. C).
 * F: [9][n_qp].  Outputs (any may be NULL):
 *   I_raw [4 + 2*npair][n_qp]: I1, I2, I3, J, I4 (pairs), I5 (pairs),
 *         npair = n_sv(n_sv+1)/2, pairs (i,j), i <= j, in row-major order;
 *   K     [p][n_qp] features;
 *   dKdF  [p][9][n_qp] feature derivatives dK_m/dF_iJ. */
int pa_invariants(const pa_model_desc* desc, int64_t n_qp, const double* F,
                  double* I_raw, double* K, double* dKdF, void* stream);

size_t pa_material_workspace_bytes(const pa_model_desc* desc, int64_t n_qp);
/* Psi, P and AA at n_qp points (eq. comp-se; eq. nncm-chain; App. A.1).
 * F: [9][n_qp]; psi [n_qp], P [9][n_qp], AA [81][n_qp] (each may be NULL).
 * prec: pa_precision of the network contractions; desc->algorithm selects the
 * Hessian formation.  workspace: pa_material_workspace_bytes(desc, n_qp). */
int pa_energy_stress_tangent(const pa_model_desc* desc, const void* prepared, int prec,
                             int64_t n_qp, const double* F, double* psi, double* P,
                             double* AA, int32_t* n_bad, void* workspace, size_t ws_bytes,
                             void* stream);

/* pa_energy_stress_tangent in batches of `batch` consecutive points (the
 * batch-vectorised evaluation of Alg. 3 / Sec. 3.2): features, network and
 * chain rule run on one batch at a time, so the workspace holds one batch,
 * pa_material_workspace_bytes(desc, min(batch, n_qp)) bytes, however long
 * the call.  F and the outputs are laid out as for pa_energy_stress_tangent
 * ([..][n_qp]); every point's arithmetic is independent of the batch, so the
 * outputs are bitwise the same for every batch size.  batch must be > 0
 * (PA_ERR_ARG otherwise). */
int pa_energy_stress_tangent_batched(const pa_model_desc* desc, const void* prepared, int prec,
                                     int64_t n_qp, int64_t batch, const double* F, double* psi,
                                     double* P, double* AA, int32_t* n_bad, void* workspace,
                                     size_t ws_bytes, void* stream);

/* Psi, Kirchhoff stress tau and spatial tangent cc at n_qp points, the
 * paper's own storage of the constitutive update (App. A.1-A.2, the tau and
 * cc of eqs. stress-cgo and stiffnes-cgo): tau [6][n_qp] and cc [21][n_qp]
 * in Voigt slots (11, 22, 33, 23, 13, 12), cc as the upper triangle of the
 * symmetric 6 x 6 matrix, row by row ((0,0), (0,1), ..., (0,5), (1,1), ...).
 * 216 bytes per point instead of the 720 of P and AA.  psi, tau or cc may be
 * NULL (cc NULL: no network Hessian is formed).  Same workspace as
 * pa_energy_stress_tangent. */
int pa_energy_stress_tangent_voigt(const pa_model_desc* desc, const void* prepared, int prec, int64_t n_qp,
                                   const double* F, double* psi, double* tau, double* cc, int32_t* n_bad,
                                   void* workspace, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- no allocation */
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and outputs as pa_energy_stress_tangent (same arguments, same
 * kernels, same numbers), with the workspace taken from a device array of
 * PA_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends.  Allocates nothing (no hipMalloc, hipFree or
 * allocating library call); the caller still owns F and the outputs.  Its
 * first call on a device looks up that device's copy of the array (with the
 * device current).  Returns PA_ERR_WORKSPACE, launching nothing, when
 * pa_material_workspace_bytes(desc, n_qp) exceeds the array, i.e. for
 * n_qp > pa_noalloc_max_points(desc) (131,072 points with two structural
 * vectors).  Every call on one GPU shares that GPU's array and leaves its
 * contents behind (nothing in it needs clearing: each call overwrites what
 * it reads); calls on one stream are ordered, but calls that overlap in time
 * on one GPU (several streams or host threads) race on the array. */
#define PA_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int pa_energy_stress_tangent_noalloc(const pa_model_desc* desc, const void* prepared, int prec,
                                     int64_t n_qp, const double* F, double* psi, double* P,
                                     double* AA, int32_t* n_bad, void* stream);
/* Largest n_qp pa_energy_stress_tangent_noalloc accepts for this model. */
int64_t pa_noalloc_max_points(const pa_model_desc* desc);

/* ---------------------------------------------------------------- elements */
/* Reference shape gradients and quadrature volumes (eqs. r-quad, k-quad):
 *   X [3][n_nodes] node coordinates, conn [nen][n_el];
 *   dNdX [nq][nen][3][n_el], w [nq][n_el] = Gauss weight * det(dX/dxi);
 *   n_bad counts points with det(dX/dxi) <= 0.
 * hex8: local node a = a0 + 2 a1 + 4 a2 at reference corner
 *   (2a0-1, 2a1-1, 2a2-1); point q = q0 + 2 q1 + 4 q2 at
 *   ((2q0-1), (2q1-1), (2q2-1))/sqrt(3), weights 1.
 * tet10: vertices at (0,0,0), (1,0,0), (0,1,0), (0,0,1), then mid-edge nodes
 *   of edges (0,1), (1,2), (0,2), (0,3), (1,3), (2,3); point q has
 *   barycentric 0.5854101966249685 at vertex q and 0.1381966011250105
 *   elsewhere, weight 1/24. */
int pa_mesh_geometry(int32_t nen, int64_t n_el, int64_t n_nodes, const double* X,
                     const int32_t* conn, double* dNdX, double* w, int32_t* n_bad,
                     void* stream);

size_t pa_element_workspace_bytes(const pa_model_desc* desc, const pa_mesh* mesh);
/* Element residual and stiffness (eqs. apprx-k, apprx-r, r-quad, k-quad;
 * Alg. 2): F_q = I + sum_a u^a (x) dN^a/dX at every point, the constitutive
 * model at all points as one batch, then
 *   r_e[e][3a+i]         = sum_q w P_iJ dN^a/dX_J,
 *   K_e[e][3a+i][3b+k]   = sum_q w dN^a/dX_J AA_iJkL dN^b/dX_L
 * (the material form, equal to the paper's spatial form).
 * u: [3*n_nodes], dof = 3*node + i.  r_e: [n_el][3 nen];
 * K_e: [n_el][3 nen][3 nen] or NULL (residual only). */
int pa_element_residual_stiffness(const pa_model_desc* desc, const void* prepared, int prec,
                                  const pa_mesh* mesh, const double* u, double* r_e,
                                  double* K_e, int32_t* n_bad, void* workspace,
                                  size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- assembly */
/* HOST setup (not on the hot path).  CSR sparsity of the global stiffness
 * over node-major dofs.  conn_host: [n_el][nen] (element-major, host).
 * Call with row_ptr/col NULL to get *nnz; then with row_ptr [3 n_nodes + 1]
 * and col [nnz] host arrays. */
int pa_csr_pattern(int32_t nen, int64_t n_el, int64_t n_nodes, const int32_t* conn_host,
                   int64_t* row_ptr, int32_t* col, int64_t* nnz);
/* HOST setup.  Greedy element colouring (no two elements of one colour share
 * a node).  colour: [n_el] host output; *n_colours set. */
int pa_colour_elements(int32_t nen, int64_t n_el, int64_t n_nodes, const int32_t* conn_host,
                       int32_t* colour, int32_t* n_colours);
/* Device: e2csr[e][a][b] = offset of column 3*conn[b] within row 3*conn[a]
 * (binary search in the sorted row).  Needs csr->row_ptr, csr->col. */
int pa_element_csr_map(const pa_mesh* mesh, const pa_csr* csr, int32_t* e2csr, void* stream);
/* Coloured scatter-assembly (Alg. 1, global accumulation over node-major
 * dofs): for each colour, one launch adds r_e into r and K_e into vals
 * without atomics.  zero_first = 1 clears r and vals first.  r may be NULL
 * (then r_e is ignored); K_e may be NULL (then vals is untouched).
 * r_e, K_e in the layout written by pa_element_residual_stiffness. */
int pa_assemble_csr(const pa_mesh* mesh, const pa_colouring* colouring, const pa_csr* csr,
                    const double* r_e, const double* K_e, double* r, double* vals,
                    int32_t zero_first, void* stream);
/* One Newton tangent build, fused: u -> F -> network -> element rows added
 * straight into r [n_rows] and vals [nnz] colour by colour (no element
 * tables in memory).  Same numbers as pa_element_residual_stiffness followed
 * by pa_assemble_csr (up to summation order within an element).  Requires
 * elements numbered colour by colour (colouring->elem_perm == NULL).  r or
 * vals may be NULL.  workspace: pa_element_workspace_bytes(desc, mesh). */
int pa_tangent_build(const pa_model_desc* desc, const void* prepared, int prec, const pa_mesh* mesh,
                     const pa_colouring* colouring, const pa_csr* csr, const double* u, double* r,
                     double* vals, int32_t* n_bad, void* workspace, size_t ws_bytes, void* stream);

/* HOST setup.  Node incidence: for node i, ent[ptr[i] .. ptr[i+1]) lists
 * e * nen + a for every element e whose local node a is i, in ascending e.
 * ptr: host [n_nodes + 1]; ent: host [n_el * nen] or NULL (then only ptr). */
int pa_node_incidence(int32_t nen, int64_t n_el, int64_t n_nodes, const int32_t* conn_host,
                      int64_t* ptr, int32_t* ent);
/* Workspace of pa_tangent_build_gather: pa_element_workspace_bytes plus the
 * element-major tables r_e [n_el][nd] and the symmetric K_e, nen (nen + 1) / 2
 * distinct 3 x 3 node blocks per element ([n_el][nen (nen + 1) / 2][3][3]). */
size_t pa_gather_workspace_bytes(const pa_model_desc* desc, const pa_mesh* mesh);
/* One Newton tangent build with node-centric assembly (same result as
 * pa_tangent_build up to summation order): elements are integrated in one
 * launch into element-major tables, then one wave per node sums its
 * elements' rows (incidence order) and writes its three CSR rows and r
 * entries once.  Every entry of r and vals is overwritten (no clearing
 * needed); the result is bitwise reproducible and needs no colouring.
 * Needs csr->row_ptr and csr->e2csr; r or vals may be NULL.  Rows longer
 * than inc->max_row are left untouched.  workspace:
 * pa_gather_workspace_bytes(desc, mesh). */
int pa_tangent_build_gather(const pa_model_desc* desc, const void* prepared, int prec, const pa_mesh* mesh,
                            const pa_incidence* inc, const pa_csr* csr, const double* u, double* r,
                            double* vals, int32_t* n_bad, void* workspace, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- adjoint */
size_t pa_param_backward_workspace(const pa_model_desc* desc, int prec, int64_t n_qp);
/* Parameter adjoint of the stress (raw network, normalize must be 0):
 *   theta_bar = sum_q (dP_q/dtheta)^T P_bar_q
 * with P_q = sum_m dN/dK_m(K_q; theta) dK_m/dF(F_q), the stress of the chain
 * rule of eq. nncm-chain with N the network of eq. icnn (App. B.2).  This is
 * the reverse-mode derivative, in the parameters, of the first-derivative
 * part of the App. B.2 network evaluation (the gradient columns of Alg. 4),
 * contracted with lambda_q,m = P_bar_q : dK_m/dF: the gradient of a
 * stress-calibration loss such as mean ||P - P_target||^2 (P_bar = dLoss/dP),
 * which is how the paper's NCMs are fitted to stress data.  Activations are
 * recomputed, not stored.  F, P_bar: [9][n_qp] (caller-owned, read only);
 * theta_bar [n_params] is overwritten (FP64; the reduction over points is in
 * a fixed order, so the result is bitwise reproducible).  prec: PA_FP64 or
 * PA_FP32 (others: PA_ERR_UNSUPPORTED).  workspace:
 * pa_param_backward_workspace bytes (features, lambda and per-workgroup
 * partial gradients), else PA_ERR_WORKSPACE. */
int pa_param_backward(const pa_model_desc* desc, const void* prepared, int prec, int64_t n_qp,
                      const double* F, const double* P_bar, double* theta_bar,
                      void* workspace, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- residual loss */
/* The NN-EUCLID residual loss of eq. (loss) (Sec. "Data generation and NCM
 * training") for one time step, and its cotangent in the residual:
 *   L = sum_{d free} r_d^2 + sum_b (R_b - sum_{d in boundary b} r_d)^2,
 *   r_bar_d = dL/dr_d = 2 r_d (free), -2 (R_b - sum_{boundary b} r) (d on b).
 * r [n_rows]: assembled residual (node-major dofs); dof_group [n_rows] int32:
 * -1 = free (D^free), b in [0, n_groups) = constrained dof of reaction
 * boundary b (D^fix_b), -2 = constrained and not observed; any other value is
 * treated as -2 (no loss term, zero cotangent; the ids are device data, so
 * the library cannot refuse them without a synchronisation).  R: device
 * [n_groups] reaction forces.  loss: device [1] or NULL; r_bar [n_rows] or
 * NULL.  The sums are reduced in a fixed order (bitwise reproducible).
 * n_groups <= 63.  Over several time steps, sum the losses and the
 * parameter gradients. */
size_t pa_residual_loss_workspace(int64_t n_rows, int32_t n_groups);
int pa_residual_loss(int64_t n_rows, const double* r, const int32_t* dof_group, int32_t n_groups,
                     const double* R, double* loss, double* r_bar, void* workspace, size_t ws_bytes,
                     void* stream);
/* Parameter gradient of a residual cotangent: theta_bar = (dr/dtheta)^T r_bar
 * for the raw network (normalize must be 0).  Since r^a_i = sum_q w P_iJ
 * G^a_J (eq. r-quad), the stress cotangent is P_bar_q = w_q sum_a
 * r_bar[a] (x) G^a_q, followed by pa_param_backward at the points' F.
 * u [3 n_nodes]; r_bar [3 n_nodes]; theta_bar [n_params] overwritten.
 * prec: PA_FP64 or PA_FP32. */
size_t pa_residual_param_backward_workspace(const pa_model_desc* desc, const pa_mesh* mesh, int prec);
int pa_residual_param_backward(const pa_model_desc* desc, const void* prepared, int prec, const pa_mesh* mesh,
                               const double* u, const double* r_bar, double* theta_bar, void* workspace,
                               size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- profiling */
/* Per-kernel timing with HIP events recorded on the launch stream around
 * every kernel the library launches (off by default).  pa_profile_enable(1)
 * clears previous records and starts recording; pa_profile_enable(0) stops.
 * pa_profile_count() synchronises on the recorded events and returns the
 * number of distinct kernels; pa_profile_get(i, ...) returns the name (a
 * static string), the summed duration in milliseconds and the number of
 * launches of kernel i. */
int     pa_profile_enable(int32_t on);
int32_t pa_profile_count(void);
int     pa_profile_get(int32_t i, const char** name, double* total_ms, int64_t* launches);

/* Measurement utility (not part of the method): one launch of `blocks`
 * workgroups of eight waves in which waves 0-3 run work of kind kind_lo and
 * waves 4-7 work of kind kind_hi, each as independent dependency chains of
 * `iters` steps: 0 none, 1 FP64 16x16x4 matrix-core products (four chains),
 * 2 FP32 16x16x4 matrix-core products (four chains, twice the steps),
 * 3 FP64 fused multiply-adds (eight chains, four times the steps), 4 FP32
 * fused multiply-adds (likewise), 5 32-bit integer multiply-adds (likewise).
 * Timing pairs of kinds against each kind alone shows whether the two
 * pipes of one SIMD run concurrently.  out: device buffer of blocks * 512
 * doubles (written, one value per thread).  Kinds outside 0..5, iters
 * outside 1..2^20, blocks outside 1..65536 or a NULL out return PA_ERR_ARG
 * before any launch. */
int pa_pipe_probe(int32_t kind_lo, int32_t kind_hi, int32_t iters, int32_t blocks, double* out, void* stream);

/* ---------------------------------------------------------------- misc */
const char* pa_status_string(int status);
/* Message describing the last PA_ERR_* returned on this thread. */
const char* pa_last_error(void);
/* Library version string. */
const char* pa_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PA_H */
