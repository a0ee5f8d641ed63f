// C ABI of the library (include/pa.h): argument checks on the host, then
// asynchronous kernel launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pa.h"
#include "pa_internal.h"

namespace pa {
int host_csr_pattern(int nen, int64_t n_el, int64_t n_nodes, const int32_t* conn, int64_t* row_ptr,
                     int32_t* col, int64_t* nnz_out);
int host_colour(int nen, int64_t n_el, int64_t n_nodes, const int32_t* conn, int32_t* colour,
                int32_t* n_colours);
int host_node_incidence(int nen, int64_t n_el, int64_t n_nodes, const int32_t* conn, int64_t* ptr,
                        int32_t* ent);
}

using namespace pa;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_check(const char* where) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(PA_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
  return PA_OK;
}

inline hipStream_t S(void* s) { return (hipStream_t)s; }

// ---- optional per-kernel event timing
struct ProfRec {
  const char* name;
  hipEvent_t a, b;
};
bool g_prof = false;
std::vector<ProfRec> g_recs;
std::vector<hipEvent_t> g_pool;
size_t g_pool_next = 0;

hipEvent_t pool_event() {
  if (g_pool_next == g_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    g_pool.push_back(e);
  }
  return g_pool[g_pool_next++];
}

struct Prof {
  const char* name;
  hipStream_t s;
  hipEvent_t a = nullptr;
  Prof(const char* n, hipStream_t st) : name(n), s(st) {
    if (g_prof && (a = pool_event())) (void)hipEventRecord(a, s);
  }
  ~Prof() {
    if (!a) return;
    hipEvent_t b = pool_event();
    if (!b) return;
    (void)hipEventRecord(b, s);
    g_recs.push_back({name, a, b});
  }
};

inline int npair_of(int n_sv) { return n_sv * (n_sv + 1) / 2; }

int check_desc(const pa_model_desc* d) {
  if (!d) return fail(PA_ERR_ARG, "desc is NULL");
  if (d->n_sv < 0 || d->n_sv > 2) return fail(PA_ERR_ARG, "n_sv must be 0, 1 or 2 (got %d)", d->n_sv);
  if (d->kind != PA_MODEL_MICNN && d->kind != PA_MODEL_CANN && d->kind != PA_MODEL_GENT_THOMAS)
    return fail(PA_ERR_ARG, "unknown model kind %d", d->kind);
  if (d->kind != PA_MODEL_MICNN) {
    for (int i = 0; i < d->n_sv; ++i)
      for (int j = 0; j < 3; ++j)
        if (!std::isfinite(d->A[i][j])) return fail(PA_ERR_ARG, "structural vector %d is not finite", i);
    return PA_OK;
  }
  if (d->n_hidden < 2) return fail(PA_ERR_ARG, "n_hidden must be >= 2 (got %d)", d->n_hidden);
  if (d->width <= 0 || (d->width > 16 && d->width % 16))
    return fail(PA_ERR_ARG, "width must be 1..16 or a multiple of 16 (got %d)", d->width);
  if (d->activation != PA_ACT_SOFTPLUS) return fail(PA_ERR_ARG, "unknown activation %d", d->activation);
  if (d->algorithm != PA_ALGO_FORWARD && d->algorithm != PA_ALGO_ADJOINT)
    return fail(PA_ERR_ARG, "unknown algorithm %d", d->algorithm);
  for (int i = 0; i < d->n_sv; ++i)
    for (int j = 0; j < 3; ++j)
      if (!std::isfinite(d->A[i][j])) return fail(PA_ERR_ARG, "structural vector %d is not finite", i);
  const int p = 3 + 2 * npair_of(d->n_sv);
  if (!mlp_supported(padded_width(d->width), d->n_hidden, p))
    return fail(PA_ERR_UNSUPPORTED, "no kernel for width %d, %d hidden layers, %d inputs", d->width, d->n_hidden, p);
  return PA_OK;
}

ModelConst model_const(const pa_model_desc* d) {
  ModelConst mc{};
  for (int i = 0; i < d->n_sv; ++i)
    for (int j = 0; j < 3; ++j) mc.A[i][j] = d->A[i][j];
  int q = 0;
  for (int i = 0; i < d->n_sv; ++i)
    for (int j = i; j < d->n_sv; ++j, ++q)
      mc.AdotA[q] = d->A[i][0] * d->A[j][0] + d->A[i][1] * d->A[j][1] + d->A[i][2] * d->A[j][2];
  return mc;
}

inline int p_of(const pa_model_desc* d) { return 3 + 2 * npair_of(d->n_sv); }

inline PrepLayout layout_of(const pa_model_desc* d) {
  PrepLayout l = prep_layout(padded_width(d->width), d->n_hidden, p_of(d));
  l.HR = d->width;
  return l;
}

inline int64_t al(int64_t x) { return (x + 255) & ~int64_t(255); }

// workspace of the material pipeline: K [p][n], N-derivatives [NOUT][n]
int64_t material_ws(const pa_model_desc* d, int64_t n) {
  const int p = p_of(d);
  const int nout = 1 + p + p * (p + 1) / 2;
  return al(8 * (int64_t)p * n) + al(8 * (int64_t)nout * n);
}

int check_prec(int prec) {
  if (prec < PA_FP64 || prec > PA_BF16_JAC) return fail(PA_ERR_ARG, "unknown precision %d", prec);
  return PA_OK;
}

// Header of the prepared buffer (N(0) and the reference-state constants).
const double* hdr_of(const pa_model_desc* d, const void* prepared) {
  const unsigned char* prep = (const unsigned char*)prepared;
  if (d->kind != PA_MODEL_MICNN) return (const double*)(prep + closed_layout(d->kind, p_of(d)).hdr);
  return (const double*)(prep + layout_of(d).hdr);
}

// The inner function's value, gradient and (hess) Hessian at n points.
int run_inner(const pa_model_desc* d, const void* prepared, int prec, int64_t n, const double* K, double* Nout,
              int hess, hipStream_t s) {
  int rc;
  if (d->kind != PA_MODEL_MICNN) {
    Prof pr("inner_closed", s);
    rc = launch_inner_closed(d->kind, p_of(d), (const unsigned char*)prepared, npair_of(d->n_sv), n, K, Nout, hess, s);
    if (rc) return fail(PA_ERR_ARG, "bad inner-function configuration");
    return PA_OK;
  }
  if (prec == PA_BF16_CORR && d->algorithm == PA_ALGO_ADJOINT) {
    // the all-BF16 pass, then the FP32 pass that rewrites the value and
    // gradient columns (the correction pass)
    {
      Prof pr("mlp_adjoint", s);
      rc = launch_mlp(layout_of(d), PA_BF16, d->algorithm, (const unsigned char*)prepared, n, K, Nout, hess, s);
    }
    if (!rc) {
      Prof pr("mlp_correction", s);
      rc = launch_mlp(layout_of(d), PA_FP32, d->algorithm, (const unsigned char*)prepared, n, K, Nout, 0, s);
    }
  } else {
    Prof pr(d->algorithm == PA_ALGO_ADJOINT ? "mlp_adjoint" : "mlp_forward", s);
    rc = launch_mlp(layout_of(d), prec, d->algorithm, (const unsigned char*)prepared, n, K, Nout, hess, s);
  }
  if (rc == -2) return fail(PA_ERR_UNSUPPORTED, "network algorithm %d not available", d->algorithm);
  if (rc) return fail(PA_ERR_ARG, "bad network configuration");
  return PA_OK;
}

// F -> (psi, P, AA) through features, network and chain rule, in batches of
// `batch` consecutive points (batch <= 0: all n at once).  The workspace
// holds one batch; F and the outputs keep their leading dimension n.  Each
// point's arithmetic is independent of the batch, so the outputs are the
// same for every batch size.
int run_material(const pa_model_desc* d, const void* prepared, int prec, int64_t n, const double* F,
                 double* psi, double* P, double* A, int32_t* n_bad, unsigned char* ws, hipStream_t s,
                 bool voigt = false, int64_t batch = 0) {
  const int p = p_of(d);
  const ModelConst mc = model_const(d);
  const int64_t nb = (batch <= 0 || batch > n) ? n : batch;
  double* K = (double*)ws;
  double* Nout = (double*)(ws + al(8 * (int64_t)p * nb));
  const double* hdr = hdr_of(d, prepared);
  auto at = [](double* x, int64_t o) { return x ? x + o : nullptr; };
  for (int64_t b = 0; b < n; b += nb) {
    const int64_t cnt = (n - b < nb) ? n - b : nb;
    {
      Prof pr("features", s);
      if (launch_features(d->n_sv, cnt, n, F + b, mc, K, n_bad, s)) return fail(PA_ERR_ARG, "bad n_sv");
    }
    int rc = run_inner(d, prepared, prec, cnt, K, Nout, A != nullptr, s);
    if (rc) return rc;
    if (voigt) {
      Prof pr("chain_voigt", s);
      if (launch_chain_voigt(d->n_sv, cnt, n, F + b, Nout, hdr, mc, at(psi, b), at(P, b), at(A, b), s))
        return fail(PA_ERR_ARG, "bad n_sv");
    } else {
      Prof pr("chain", s);
      if (launch_chain(d->n_sv, cnt, n, F + b, Nout, hdr, mc, at(psi, b), at(P, b), at(A, b), n_bad, s))
        return fail(PA_ERR_ARG, "bad n_sv");
    }
  }
  return hip_check("material kernels");
}

int check_mesh(const pa_mesh* m) {
  if (!m) return fail(PA_ERR_ARG, "mesh is NULL");
  if (!((m->nen == 8 && m->nq == 8) || (m->nen == 10 && m->nq == 4)))
    return fail(PA_ERR_ARG, "unsupported element: nen=%d nq=%d (hex8: 8/8, tet10: 10/4)", m->nen, m->nq);
  if (m->n_el < 0 || m->n_nodes < 0) return fail(PA_ERR_ARG, "negative mesh size");
  if (m->n_el > 0 && (!m->conn || !m->dNdX || !m->w)) return fail(PA_ERR_ARG, "mesh arrays missing");
  if ((int64_t)m->n_el * m->nq > ((int64_t)1 << 40)) return fail(PA_ERR_ARG, "mesh too large");
  return PA_OK;
}

}  // namespace

extern "C" {

const char* pa_version(void) { return "pa 0.1 (gfx950)"; }

const char* pa_last_error(void) { return g_err.c_str(); }

const char* pa_status_string(int s) {
  switch (s) {
    case PA_OK: return "ok";
    case PA_ERR_ARG: return "invalid argument";
    case PA_ERR_UNSUPPORTED: return "unsupported configuration";
    case PA_ERR_HIP: return "HIP runtime error";
    case PA_ERR_WORKSPACE: return "workspace too small";
    default: return "unknown status";
  }
}

int32_t pa_num_inputs(const pa_model_desc* d) {
  if (!d || d->n_sv < 0 || d->n_sv > 2) return -1;
  return p_of(d);
}

int64_t pa_num_params(const pa_model_desc* d) {
  if (!d || d->n_sv < 0 || d->n_sv > 2) return -1;
  if (d->kind == PA_MODEL_CANN || d->kind == PA_MODEL_GENT_THOMAS) return closed_num_params(d->kind, p_of(d));
  if (d->width <= 0 || d->n_hidden < 1) return -1;
  return theta_layout(d->width, d->n_hidden, p_of(d), d->has_bias ? 1 : 0).total;
}

int32_t pa_supported(const pa_model_desc* d) { return check_desc(d) == PA_OK ? 1 : 0; }

size_t pa_prepared_bytes(const pa_model_desc* d) {
  if (check_desc(d) != PA_OK) return 0;
  if (d->kind != PA_MODEL_MICNN) return (size_t)closed_layout(d->kind, p_of(d)).total;
  return (size_t)layout_of(d).total;
}

int pa_prepare_params(const pa_model_desc* d, const double* theta, void* prepared, void* stream) {
  int rc = check_desc(d);
  if (rc) return rc;
  if (!theta || !prepared) return fail(PA_ERR_ARG, "theta and prepared must be non-NULL");
  if (d->kind != PA_MODEL_MICNN) {
    if (launch_prepare_closed(d->kind, p_of(d), closed_num_params(d->kind, p_of(d)), theta, (unsigned char*)prepared,
                              d->normalize ? 1 : 0, npair_of(d->n_sv), S(stream)))
      return fail(PA_ERR_UNSUPPORTED, "prepare failed");
    return hip_check("pa_prepare_params");
  }
  const PrepLayout lay = layout_of(d);
  const ThetaLayout tl = theta_layout(d->width, d->n_hidden, p_of(d), d->has_bias ? 1 : 0);
  rc = launch_prepare(lay, tl, theta, (unsigned char*)prepared, d->normalize ? 1 : 0, npair_of(d->n_sv), S(stream));
  if (rc) return fail(PA_ERR_UNSUPPORTED, "prepare failed (%d)", rc);
  return hip_check("pa_prepare_params");
}

int pa_invariants(const pa_model_desc* d, int64_t n, const double* F, double* I_raw, double* K,
                  double* dKdF, void* stream) {
  if (!d || d->n_sv < 0 || d->n_sv > 2) return fail(PA_ERR_ARG, "bad desc / n_sv");
  if (n < 0) return fail(PA_ERR_ARG, "n_qp < 0");
  if (n > 0 && !F) return fail(PA_ERR_ARG, "F is NULL");
  if (n == 0) return PA_OK;
  launch_invariants(d->n_sv, n, F, model_const(d), I_raw, K, dKdF, nullptr, S(stream));
  return hip_check("pa_invariants");
}

size_t pa_material_workspace_bytes(const pa_model_desc* d, int64_t n) {
  if (!d || d->n_sv < 0 || d->n_sv > 2 || n < 0) return 0;
  return (size_t)material_ws(d, n);
}

int pa_energy_stress_tangent(const pa_model_desc* d, const void* prepared, int prec, int64_t n,
                             const double* F, double* psi, double* P, double* A, int32_t* n_bad,
                             void* workspace, size_t ws_bytes, void* stream) {
  int rc = check_desc(d);
  if (rc) return rc;
  if ((rc = check_prec(prec))) return rc;
  if (n < 0) return fail(PA_ERR_ARG, "n_qp < 0");
  if (n == 0) return PA_OK;
  if (!prepared || !F) return fail(PA_ERR_ARG, "prepared and F must be non-NULL");
  if (!workspace || (int64_t)ws_bytes < material_ws(d, n))
    return fail(PA_ERR_WORKSPACE, "workspace needs %lld bytes", (long long)material_ws(d, n));
  return run_material(d, prepared, prec, n, F, psi, P, A, n_bad, (unsigned char*)workspace, S(stream));
}

int pa_energy_stress_tangent_batched(const pa_model_desc* d, const void* prepared, int prec, int64_t n,
                                     int64_t batch, const double* F, double* psi, double* P, double* A,
                                     int32_t* n_bad, void* workspace, size_t ws_bytes, void* stream) {
  int rc = check_desc(d);
  if (rc) return rc;
  if ((rc = check_prec(prec))) return rc;
  if (n < 0) return fail(PA_ERR_ARG, "n_qp < 0");
  if (batch <= 0) return fail(PA_ERR_ARG, "batch must be positive (got %lld)", (long long)batch);
  if (n == 0) return PA_OK;
  if (!prepared || !F) return fail(PA_ERR_ARG, "prepared and F must be non-NULL");
  const int64_t nb = batch < n ? batch : n;
  if (!workspace || (int64_t)ws_bytes < material_ws(d, nb))
    return fail(PA_ERR_WORKSPACE, "workspace needs %lld bytes", (long long)material_ws(d, nb));
  return run_material(d, prepared, prec, n, F, psi, P, A, n_bad, (unsigned char*)workspace, S(stream), false, nb);
}

int pa_energy_stress_tangent_voigt(const pa_model_desc* d, const void* prepared, int prec, int64_t n,
                                   const double* F, double* psi, double* tau, double* cc, int32_t* n_bad,
                                   void* workspace, size_t ws_bytes, void* stream) {
  int rc = check_desc(d);
  if (rc) return rc;
  if ((rc = check_prec(prec))) return rc;
  if (n < 0) return fail(PA_ERR_ARG, "n_qp < 0");
  if (n == 0) return PA_OK;
  if (!prepared || !F) return fail(PA_ERR_ARG, "prepared and F must be non-NULL");
  if (!workspace || (int64_t)ws_bytes < material_ws(d, n))
    return fail(PA_ERR_WORKSPACE, "workspace needs %lld bytes", (long long)material_ws(d, n));
  return run_material(d, prepared, prec, n, F, psi, tau, cc, n_bad, (unsigned char*)workspace, S(stream), true);
}

}  // extern "C"

// ---- the allocation-free material call: its workspace is this file-scope
// device array (one copy per GPU, held until the process ends).  In host
// code `scratch` names a host-side stand-in, so kernels and copies use the
// device address that hipGetSymbolAddress returns for the current device.
namespace {
static __device__ __align__(256) unsigned char scratch[PA_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of the current device's scratch array, looked up once per
// device with that device current.
int scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(PA_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(PA_ERR_ARG, "device %d outside 0..%d", dev, kMaxDevices - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(PA_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return PA_OK;
}
}  // namespace

extern "C" {

int pa_energy_stress_tangent_noalloc(const pa_model_desc* d, const void* prepared, int prec, int64_t n,
                                     const double* F, double* psi, double* P, double* A, int32_t* n_bad,
                                     void* stream) {
  int rc = check_desc(d);
  if (rc) return rc;
  if ((rc = check_prec(prec))) return rc;
  if (n < 0) return fail(PA_ERR_ARG, "n_qp < 0");
  if (n == 0) return PA_OK;
  if (!prepared || !F) return fail(PA_ERR_ARG, "prepared and F must be non-NULL");
  const int64_t need = material_ws(d, n);
  if (need > (int64_t)PA_NOALLOC_SCRATCH_BYTES)
    return fail(PA_ERR_WORKSPACE,
                "pa_energy_stress_tangent_noalloc: %lld points need %lld bytes of scratch, the library holds %lld "
                "(at most %lld points for this model)",
                (long long)n, (long long)need, (long long)PA_NOALLOC_SCRATCH_BYTES,
                (long long)pa_noalloc_max_points(d));
  void* ws = nullptr;
  if ((rc = scratch_address(&ws))) return rc;
  return run_material(d, prepared, prec, n, F, psi, P, A, n_bad, (unsigned char*)ws, S(stream));
}

int64_t pa_noalloc_max_points(const pa_model_desc* d) {
  if (!d || d->n_sv < 0 || d->n_sv > 2) return 0;
  // material_ws rounds each of its two arrays up to 256 bytes
  const int p = p_of(d);
  const int64_t per_point = 8 * (int64_t)(p + 1 + p + p * (p + 1) / 2);
  int64_t n = ((int64_t)PA_NOALLOC_SCRATCH_BYTES - 512) / per_point;
  while (n > 0 && material_ws(d, n) > (int64_t)PA_NOALLOC_SCRATCH_BYTES) --n;
  while (material_ws(d, n + 1) <= (int64_t)PA_NOALLOC_SCRATCH_BYTES) ++n;
  return n;
}

int pa_mesh_geometry(int32_t nen, int64_t n_el, int64_t n_nodes, const double* X, const int32_t* conn,
                     double* dNdX, double* w, int32_t* n_bad, void* stream) {
  if (nen != 8 && nen != 10) return fail(PA_ERR_ARG, "nen must be 8 or 10");
  if (n_el < 0 || n_nodes < 0) return fail(PA_ERR_ARG, "negative size");
  if (n_el == 0) return PA_OK;
  if (!X || !conn || !dNdX || !w) return fail(PA_ERR_ARG, "NULL array");
  launch_geometry(nen, n_el, n_nodes, X, conn, dNdX, w, n_bad, S(stream));
  return hip_check("pa_mesh_geometry");
}

size_t pa_element_workspace_bytes(const pa_model_desc* d, const pa_mesh* m) {
  if (!d || !m || d->n_sv < 0 || d->n_sv > 2) return 0;
  const int64_t n = m->n_el * m->nq;
  // F [9][n], S~ and CC~ [27][n], then the material workspace (features,
  // network derivatives)
  return (size_t)(al(8 * 9 * n) + al(8 * 27 * n) + material_ws(d, n));
}

namespace {
// u -> F -> features -> network derivatives (workspace), shared by the
// element entry points.  Returns the network-output pointer.
int element_front(const pa_model_desc* d, const void* prepared, int prec, const pa_mesh* m, const double* u,
                  int32_t* n_bad, unsigned char* ws, hipStream_t s, double** F_out, double** SC_out) {
  const int64_t n = m->n_el * m->nq;
  const int p = p_of(d);
  double* F = (double*)ws;
  double* SC = (double*)(ws + al(8 * 9 * n));
  unsigned char* mws = ws + al(8 * 9 * n) + al(8 * 27 * n);
  double* K = (double*)mws;
  double* Nout = (double*)(mws + al(8 * (int64_t)p * n));
  const ModelConst mc = model_const(d);
  {
    Prof pr("gather_F", s);  // F and the network inputs in one pass
    launch_gather_F(m->nen, m->nq, m->n_el, m->n_nodes, m->conn, m->dNdX, m->X, u, F, d->n_sv, &mc, K, n_bad, s);
  }
  int rc = run_inner(d, prepared, prec, n, K, Nout, 1, s);
  if (rc) return rc;
  {
    Prof pr("material_cc", s);
    launch_material_cc(d->n_sv, n, F, Nout, mc, SC, s);
  }
  *F_out = F;
  *SC_out = SC;
  return PA_OK;
}
}  // namespace

int pa_element_residual_stiffness(const pa_model_desc* d, const void* prepared, int prec, const pa_mesh* m,
                                  const double* u, double* r_e, double* K_e, int32_t* n_bad,
                                  void* workspace, size_t ws_bytes, void* stream) {
  int rc = check_desc(d);
  if (rc) return rc;
  if ((rc = check_prec(prec))) return rc;
  if ((rc = check_mesh(m))) return rc;
  if (m->n_el == 0) return PA_OK;
  if (!prepared || !u || !r_e) return fail(PA_ERR_ARG, "prepared, u and r_e must be non-NULL");
  const int64_t need = (int64_t)pa_element_workspace_bytes(d, m);
  if (!workspace || (int64_t)ws_bytes < need) return fail(PA_ERR_WORKSPACE, "workspace needs %lld bytes", (long long)need);
  hipStream_t s = S(stream);
  double *F, *SC;
  if ((rc = element_front(d, prepared, prec, m, u, n_bad, (unsigned char*)workspace, s, &F, &SC))) return rc;
  {
    Prof pr("integrate", s);
    launch_chain_integrate(m->nen, m->n_el, 0, m->n_el, m->conn, m->dNdX, m->w, m->n_nodes, m->X, F, SC, r_e, K_e, nullptr,
                           nullptr, nullptr, nullptr, 0, s);
  }
  return hip_check("pa_element_residual_stiffness");
}

int pa_tangent_build(const pa_model_desc* d, const void* prepared, int prec, const pa_mesh* m,
                     const pa_colouring* col, const pa_csr* c, const double* u, double* r, double* vals,
                     int32_t* n_bad, void* workspace, size_t ws_bytes, void* stream) {
  int rc = check_desc(d);
  if (rc) return rc;
  if ((rc = check_prec(prec))) return rc;
  if ((rc = check_mesh(m))) return rc;
  if (!col || !c) return fail(PA_ERR_ARG, "colouring and csr must be non-NULL");
  if (col->elem_perm) return fail(PA_ERR_ARG, "pa_tangent_build needs elements numbered colour by colour (elem_perm = NULL)");
  if (col->n_colours < 0 || (col->n_colours > 0 && !col->colour_ptr)) return fail(PA_ERR_ARG, "bad colouring");
  if (col->n_colours > 0 && (col->colour_ptr[0] != 0 || col->colour_ptr[col->n_colours] != m->n_el))
    return fail(PA_ERR_ARG, "colour_ptr must start at 0 and end at n_el");
  for (int i = 0; i < col->n_colours; ++i)
    if (col->colour_ptr[i + 1] < col->colour_ptr[i]) return fail(PA_ERR_ARG, "colour_ptr not monotone");
  if (c->n_rows != 3 * m->n_nodes) return fail(PA_ERR_ARG, "csr has %lld rows, mesh needs %lld", (long long)c->n_rows, (long long)(3 * m->n_nodes));
  if (vals && (!c->row_ptr || !c->e2csr)) return fail(PA_ERR_ARG, "csr row_ptr and e2csr needed for vals");
  if (!r && !vals) return fail(PA_ERR_ARG, "nothing to assemble");
  if (m->n_el == 0) return PA_OK;
  if (!prepared || !u) return fail(PA_ERR_ARG, "prepared and u must be non-NULL");
  const int64_t need = (int64_t)pa_element_workspace_bytes(d, m);
  if (!workspace || (int64_t)ws_bytes < need) return fail(PA_ERR_WORKSPACE, "workspace needs %lld bytes", (long long)need);
  hipStream_t s = S(stream);
  double *F, *SC;
  if ((rc = element_front(d, prepared, prec, m, u, n_bad, (unsigned char*)workspace, s, &F, &SC))) return rc;
  {
    Prof pr("fill", s);
    if (r) launch_fill(r, c->n_rows, 0.0, s);
    if (vals) launch_fill(vals, c->nnz, 0.0, s);
  }
  for (int k = 0; k < col->n_colours; ++k) {
    Prof pr("integrate_scatter", s);
    const int64_t b = col->colour_ptr[k], cnt = col->colour_ptr[k + 1] - b;
    launch_chain_integrate(m->nen, m->n_el, b, cnt, m->conn, m->dNdX, m->w, m->n_nodes, m->X, F, SC, nullptr, nullptr, c->row_ptr,
                           c->e2csr, r, vals, 1, s);
  }
  return hip_check("pa_tangent_build");
}

size_t pa_gather_workspace_bytes(const pa_model_desc* d, const pa_mesh* m) {
  const size_t base = pa_element_workspace_bytes(d, m);
  if (!base) return 0;
  const int64_t nd = 3 * (int64_t)m->nen, nsym = 9 * (int64_t)m->nen * (m->nen + 1) / 2;
  return (size_t)(al((int64_t)base) + al(8 * nd * m->n_el) + al(8 * nsym * m->n_el));
}

int pa_tangent_build_gather(const pa_model_desc* d, const void* prepared, int prec, const pa_mesh* m,
                            const pa_incidence* inc, const pa_csr* c, const double* u, double* r, double* vals,
                            int32_t* n_bad, void* workspace, size_t ws_bytes, void* stream) {
  int rc = check_desc(d);
  if (rc) return rc;
  if ((rc = check_prec(prec))) return rc;
  if ((rc = check_mesh(m))) return rc;
  if (!inc || !c) return fail(PA_ERR_ARG, "incidence and csr must be non-NULL");
  if (inc->n_nodes != m->n_nodes || inc->n_ent != m->n_el * m->nen)
    return fail(PA_ERR_ARG, "incidence does not match the mesh (%lld nodes, %lld entries)", (long long)inc->n_nodes,
                (long long)inc->n_ent);
  if (c->n_rows != 3 * m->n_nodes) return fail(PA_ERR_ARG, "csr has %lld rows, mesh needs %lld", (long long)c->n_rows, (long long)(3 * m->n_nodes));
  if (!r && !vals) return fail(PA_ERR_ARG, "nothing to assemble");
  if (!c->row_ptr || !c->e2csr) return fail(PA_ERR_ARG, "csr row_ptr and e2csr are needed");
  if (m->n_nodes > 0 && (!inc->ptr || (!inc->ent && inc->n_ent > 0))) return fail(PA_ERR_ARG, "incidence arrays missing");
  if (inc->max_row < 0 || (size_t)4 * 3 * inc->max_row * sizeof(double) > 64 * 1024)
    return fail(PA_ERR_UNSUPPORTED, "max_row %d out of range (at most %d)", inc->max_row, 64 * 1024 / (12 * 8));
  if (m->n_el * (int64_t)m->nen >= ((int64_t)1 << 31)) return fail(PA_ERR_ARG, "n_el * nen must fit in 31 bits");
  if (m->n_el == 0) return PA_OK;
  if (!prepared || !u) return fail(PA_ERR_ARG, "prepared and u must be non-NULL");
  const int64_t need = (int64_t)pa_gather_workspace_bytes(d, m);
  if (!workspace || (int64_t)ws_bytes < need) return fail(PA_ERR_WORKSPACE, "workspace needs %lld bytes", (long long)need);
  hipStream_t s = S(stream);
  double *F, *SC;
  unsigned char* ws = (unsigned char*)workspace;
  if ((rc = element_front(d, prepared, prec, m, u, n_bad, ws, s, &F, &SC))) return rc;
  const int64_t nd = 3 * (int64_t)m->nen;
  unsigned char* tab = ws + al((int64_t)pa_element_workspace_bytes(d, m));
  double* rw = (double*)tab;
  double* Kw = (double*)(tab + al(8 * nd * m->n_el));
  {
    Prof pr("integrate_elmajor", s);
    launch_chain_integrate(m->nen, m->n_el, 0, m->n_el, m->conn, m->dNdX, m->w, m->n_nodes, m->X, F, SC, rw, Kw, nullptr, nullptr,
                           nullptr, nullptr, 2, s);
  }
  {
    Prof pr("gather_assemble", s);
    launch_gather_assemble(m->nen, m->n_nodes, inc->ptr, inc->ent, c->row_ptr, c->e2csr, Kw, rw, r, vals,
                           inc->max_row, s);
  }
  return hip_check("pa_tangent_build_gather");
}

size_t pa_residual_loss_workspace(int64_t n_rows, int32_t n_groups) {
  if (n_rows < 0 || n_groups < 0 || n_groups > 63) return 0;
  return (size_t)(al(8 * (int64_t)loss_partial_blocks(n_rows) * (n_groups + 1)) + al(8 * (int64_t)(n_groups + 1)));
}

int pa_residual_loss(int64_t n_rows, const double* r, const int32_t* dof_group, int32_t n_groups, const double* R,
                     double* loss, double* r_bar, void* workspace, size_t ws_bytes, void* stream) {
  if (n_rows < 0 || n_groups < 0 || n_groups > 63) return fail(PA_ERR_ARG, "n_rows < 0 or n_groups outside [0, 63]");
  if ((n_rows > 0 && (!r || !dof_group)) || (n_groups > 0 && !R)) return fail(PA_ERR_ARG, "NULL argument");
  if (!loss && !r_bar) return fail(PA_ERR_ARG, "nothing to compute");
  const int64_t need = (int64_t)pa_residual_loss_workspace(n_rows, n_groups);
  if (!workspace || (int64_t)ws_bytes < need) return fail(PA_ERR_WORKSPACE, "workspace needs %lld bytes", (long long)need);
  unsigned char* ws = (unsigned char*)workspace;
  double* partials = (double*)ws;
  double* sums = (double*)(ws + al(8 * (int64_t)loss_partial_blocks(n_rows) * (n_groups + 1)));
  hipStream_t s = S(stream);
  {
    Prof pr("residual_loss", s);
    if (launch_residual_loss(n_rows, r, dof_group, n_groups, R, partials, sums, loss, r_bar, s))
      return fail(PA_ERR_ARG, "residual loss launch failed");
  }
  return hip_check("pa_residual_loss");
}

size_t pa_residual_param_backward_workspace(const pa_model_desc* d, const pa_mesh* m, int prec) {
  if (!d || !m || d->n_sv < 0 || d->n_sv > 2 || d->width <= 0) return 0;
  const int64_t n = m->n_el * m->nq;
  return (size_t)(al(8 * 9 * n) + al(8 * 9 * n) + param_backward_ws(d->width, d->n_hidden, p_of(d), prec, n));
}

int pa_residual_param_backward(const pa_model_desc* d, const void* prepared, int prec, const pa_mesh* m,
                               const double* u, const double* r_bar, double* theta_bar, void* workspace,
                               size_t ws_bytes, void* stream) {
  int rc = check_desc(d);
  if (rc) return rc;
  if (d->kind != PA_MODEL_MICNN) return fail(PA_ERR_UNSUPPORTED, "the parameter adjoint is provided for the MICNN");
  if (prec != PA_FP64 && prec != PA_FP32) return fail(PA_ERR_UNSUPPORTED, "supports PA_FP64 and PA_FP32");
  if (d->normalize) return fail(PA_ERR_UNSUPPORTED, "differentiates the raw network (normalize = 0)");
  if ((rc = check_mesh(m))) return rc;
  if (!prepared || !theta_bar || (m->n_el > 0 && (!u || !r_bar))) return fail(PA_ERR_ARG, "NULL argument");
  const int64_t n = m->n_el * m->nq;
  const int64_t need = (int64_t)pa_residual_param_backward_workspace(d, m, prec);
  if (!workspace || (int64_t)ws_bytes < need) return fail(PA_ERR_WORKSPACE, "workspace needs %lld bytes", (long long)need);
  hipStream_t s = S(stream);
  unsigned char* ws = (unsigned char*)workspace;
  double* F = (double*)ws;
  double* Pbar = (double*)(ws + al(8 * 9 * n));
  unsigned char* bws = ws + al(8 * 9 * n) + al(8 * 9 * n);
  {
    Prof pr("gather_F", s);
    launch_gather_F(m->nen, m->nq, m->n_el, m->n_nodes, m->conn, m->dNdX, m->X, u, F, -1, nullptr, nullptr, nullptr, s);
  }
  {
    Prof pr("residual_cotangent", s);
    launch_residual_cotangent(m->nen, m->n_el, m->conn, m->dNdX, m->w, r_bar, Pbar, s);
  }
  const PrepLayout lay = layout_of(d);
  const ThetaLayout tl = theta_layout(d->width, d->n_hidden, p_of(d), d->has_bias ? 1 : 0);
  {
    Prof pr("param_backward", s);
    rc = launch_param_backward(lay, tl, d->n_sv, prec, (const unsigned char*)prepared, model_const(d), n, F, Pbar,
                               theta_bar, bws, s);
  }
  if (rc == -2) return fail(PA_ERR_UNSUPPORTED, "no adjoint kernel for this configuration");
  if (rc) return fail(PA_ERR_ARG, "pa_residual_param_backward failed (%d)", rc);
  return hip_check("pa_residual_param_backward");
}

int pa_node_incidence(int32_t nen, int64_t n_el, int64_t n_nodes, const int32_t* conn_host, int64_t* ptr,
                      int32_t* ent) {
  if (nen != 8 && nen != 10) return fail(PA_ERR_ARG, "nen must be 8 or 10");
  if (!conn_host || !ptr || n_el < 0 || n_nodes < 0) return fail(PA_ERR_ARG, "bad arguments");
  if (n_el * (int64_t)nen >= ((int64_t)1 << 31)) return fail(PA_ERR_ARG, "n_el * nen must fit in 31 bits");
  if (host_node_incidence(nen, n_el, n_nodes, conn_host, ptr, ent))
    return fail(PA_ERR_ARG, "connectivity refers to a node outside [0, n_nodes)");
  return PA_OK;
}

int pa_csr_pattern(int32_t nen, int64_t n_el, int64_t n_nodes, const int32_t* conn_host, int64_t* row_ptr,
                   int32_t* col, int64_t* nnz) {
  if (nen != 8 && nen != 10) return fail(PA_ERR_ARG, "nen must be 8 or 10");
  if (!conn_host || !nnz || n_el < 0 || n_nodes < 0) return fail(PA_ERR_ARG, "bad arguments");
  if (3 * n_nodes >= ((int64_t)1 << 31)) return fail(PA_ERR_ARG, "too many dofs for 32-bit column indices");
  if (col && !row_ptr) return fail(PA_ERR_ARG, "col requires row_ptr");
  if (host_csr_pattern(nen, n_el, n_nodes, conn_host, row_ptr, col, nnz))
    return fail(PA_ERR_ARG, "connectivity refers to a node outside [0, n_nodes)");
  return PA_OK;
}

int pa_colour_elements(int32_t nen, int64_t n_el, int64_t n_nodes, const int32_t* conn_host, int32_t* colour,
                       int32_t* n_colours) {
  if (nen != 8 && nen != 10) return fail(PA_ERR_ARG, "nen must be 8 or 10");
  if (!conn_host || !colour || !n_colours || n_el < 0) return fail(PA_ERR_ARG, "bad arguments");
  if (host_colour(nen, n_el, n_nodes, conn_host, colour, n_colours))
    return fail(PA_ERR_ARG, "connectivity refers to a node outside [0, n_nodes)");
  return PA_OK;
}

int pa_element_csr_map(const pa_mesh* m, const pa_csr* c, int32_t* e2csr, void* stream) {
  if (!m || !c || !e2csr) return fail(PA_ERR_ARG, "NULL argument");
  if (m->nen != 8 && m->nen != 10) return fail(PA_ERR_ARG, "nen must be 8 or 10");
  if (!c->row_ptr || !c->col || !m->conn) return fail(PA_ERR_ARG, "csr/conn arrays missing");
  launch_csr_map(m->nen, m->n_el, m->conn, c->row_ptr, c->col, e2csr, S(stream));
  return hip_check("pa_element_csr_map");
}

int pa_assemble_csr(const pa_mesh* m, const pa_colouring* col, const pa_csr* c, const double* r_e,
                    const double* K_e, double* r, double* vals, int32_t zero_first, void* stream) {
  if (!m || !col || !c) return fail(PA_ERR_ARG, "NULL argument");
  if (m->nen != 8 && m->nen != 10) return fail(PA_ERR_ARG, "nen must be 8 or 10");
  if (c->n_rows != 3 * m->n_nodes) return fail(PA_ERR_ARG, "csr has %lld rows, mesh needs %lld", (long long)c->n_rows, (long long)(3 * m->n_nodes));
  if (col->n_colours < 0 || (col->n_colours > 0 && !col->colour_ptr)) return fail(PA_ERR_ARG, "bad colouring");
  if (col->n_colours > 0 && (col->colour_ptr[0] != 0 || col->colour_ptr[col->n_colours] != m->n_el))
    return fail(PA_ERR_ARG, "colour_ptr must start at 0 and end at n_el");
  for (int i = 0; i < col->n_colours; ++i)
    if (col->colour_ptr[i + 1] < col->colour_ptr[i]) return fail(PA_ERR_ARG, "colour_ptr not monotone");
  const bool doK = K_e && vals;
  const bool doR = r_e && r;
  if (doK && (!c->row_ptr || !c->e2csr)) return fail(PA_ERR_ARG, "csr row_ptr and e2csr needed for K");
  hipStream_t s = S(stream);
  if (zero_first) {
    Prof pr("fill", s);
    if (r) launch_fill(r, c->n_rows, 0.0, s);
    if (vals) launch_fill(vals, c->nnz, 0.0, s);
  }
  for (int k = 0; k < col->n_colours; ++k) {
    Prof pr("assemble", s);
    const int64_t b = col->colour_ptr[k], cnt = col->colour_ptr[k + 1] - b;
    launch_assemble(m->nen, b, cnt, col->elem_perm, m->n_el, m->conn, c->row_ptr, c->e2csr,
                    doR ? r_e : nullptr, doK ? K_e : nullptr, doR ? r : nullptr, doK ? vals : nullptr, s);
  }
  return hip_check("pa_assemble_csr");
}

size_t pa_param_backward_workspace(const pa_model_desc* d, int prec, int64_t n) {
  if (!d || d->n_sv < 0 || d->n_sv > 2 || n < 0 || d->width <= 0) return 0;
  return (size_t)param_backward_ws(d->width, d->n_hidden, p_of(d), prec, n);
}

int pa_param_backward(const pa_model_desc* d, const void* prepared, int prec, int64_t n, const double* F,
                      const double* P_bar, double* theta_bar, void* workspace, size_t ws_bytes, void* stream) {
  int rc = check_desc(d);
  if (rc) return rc;
  if (d->kind != PA_MODEL_MICNN) return fail(PA_ERR_UNSUPPORTED, "the parameter adjoint is provided for the MICNN");
  if (prec != PA_FP64 && prec != PA_FP32) return fail(PA_ERR_UNSUPPORTED, "pa_param_backward supports PA_FP64 and PA_FP32");
  if (d->normalize) return fail(PA_ERR_UNSUPPORTED, "pa_param_backward differentiates the raw network (normalize = 0)");
  if (n < 0) return fail(PA_ERR_ARG, "n_qp < 0");
  if (!prepared || !theta_bar || (n > 0 && (!F || !P_bar))) return fail(PA_ERR_ARG, "NULL argument");
  const int64_t need = param_backward_ws(d->width, d->n_hidden, p_of(d), prec, n);
  if (!workspace || (int64_t)ws_bytes < need) return fail(PA_ERR_WORKSPACE, "workspace needs %lld bytes", (long long)need);
  const PrepLayout lay = layout_of(d);
  const ThetaLayout tl = theta_layout(d->width, d->n_hidden, p_of(d), d->has_bias ? 1 : 0);
  hipStream_t s = S(stream);
  {
    Prof pr("param_backward", s);
    rc = launch_param_backward(lay, tl, d->n_sv, prec, (const unsigned char*)prepared, model_const(d), n, F, P_bar,
                               theta_bar, (unsigned char*)workspace, s);
  }
  if (rc == -2) return fail(PA_ERR_UNSUPPORTED, "no adjoint kernel for this configuration");
  if (rc) return fail(PA_ERR_ARG, "pa_param_backward failed (%d)", rc);
  return hip_check("pa_param_backward");
}

int pa_pipe_probe(int32_t kind_lo, int32_t kind_hi, int32_t iters, int32_t blocks, double* out, void* stream) {
  if (kind_lo < 0 || kind_lo > 5 || kind_hi < 0 || kind_hi > 5)
    return fail(PA_ERR_ARG, "probe kinds must lie in 0..5 (got %d, %d)", kind_lo, kind_hi);
  if (iters <= 0 || iters > (1 << 20)) return fail(PA_ERR_ARG, "iters must lie in 1..2^20 (got %d)", iters);
  if (blocks <= 0 || blocks > 65536) return fail(PA_ERR_ARG, "blocks must lie in 1..65536 (got %d)", blocks);
  if (!out) return fail(PA_ERR_ARG, "out must be non-NULL");
  launch_pipe_probe(kind_lo, kind_hi, iters, blocks, out, S(stream));
  return hip_check("pa_pipe_probe");
}

int pa_profile_enable(int32_t on) {
  g_prof = on != 0;
  if (g_prof) {
    g_recs.clear();
    g_pool_next = 0;
  }
  return PA_OK;
}

namespace {
struct Agg {
  double ms = 0.0;
  int64_t n = 0;
};
std::vector<std::pair<std::string, Agg>> g_agg;
}  // namespace

int32_t pa_profile_count(void) {
  std::map<std::string, Agg> m;
  for (auto& r : g_recs) {
    if (hipEventSynchronize(r.b) != hipSuccess) return fail(PA_ERR_HIP, "event synchronise failed");
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return fail(PA_ERR_HIP, "event timing failed");
    Agg& a = m[r.name];
    a.ms += ms;
    a.n += 1;
  }
  g_agg.assign(m.begin(), m.end());
  return (int32_t)g_agg.size();
}

int pa_profile_get(int32_t i, const char** name, double* total_ms, int64_t* launches) {
  if (i < 0 || i >= (int32_t)g_agg.size()) return fail(PA_ERR_ARG, "profile index out of range");
  static thread_local std::string nm;
  nm = g_agg[i].first;
  if (name) *name = nm.c_str();
  if (total_ms) *total_ms = g_agg[i].second.ms;
  if (launches) *launches = g_agg[i].second.n;
  return PA_OK;
}

}  // extern "C"
