// Inner network (MICNN, eq. icnn of App. B.2) with its input gradient and
// Hessian, evaluated by the one-pass forward mode of Alg. 4 on the matrix
// cores of gfx950.
//
// Data layout.  A workgroup owns a tile of 16 quadrature points, which form
// the N dimension (16 columns) of every matrix-core instruction.  The h
// neurons of each hidden layer are split into h/16 blocks of 16 rows; wave w
// computes rows 16w..16w+15 of layers 2..L.  Layer 1 (h x p, cheap) is
// evaluated by every wave for all rows so that its outputs are already in the
// register positions the next instruction reads: the result of one
// instruction (column = point, rows per lane) is fed back as the B operand of
// the next with the K index permuted to match, so activations never leave
// registers between layer 1 and layer 2.  Between layers k >= 2 the activated
// rows are exchanged through LDS.
//
// Columns.  Alg. 4 carries, for every point, the value column z, the p
// gradient columns dz/dK_m and the p(p+1)/2 Hessian columns d2z/dK_m dK_n.
// They are streamed through the layers in that order: the value column
// leaves sigma(y_k) and F''(y_k) in registers, the gradient columns leave
// dy_k/dK_m, and each Hessian column then needs only
//   d2z_k = F'(y_k) (A_k d2z_{k-1}) + F''(y_k) dy_k/dK_m dy_k/dK_n.
// The output layer N = a.z_L + b.K is applied to every column as it leaves
// layer L (cross-lane and cross-wave sums in a fixed order).
#include <type_traits>
#include <utility>

#include "pa_internal.h"
#include "mma_util.h"

namespace pa {

// ---------------------------------------------------------------- layouts
static inline int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

PrepLayout prep_layout(int H, int L, int P) {
  PrepLayout l{};
  l.H = H; l.L = L; l.P = P;
  l.MB = H / 16;
  l.S1 = (P + 3) / 4;
  l.SH = H / 4;
  l.SHB = (H + 31) / 32;
  l.NOUT = 1 + P + P * (P + 1) / 2;
  int64_t o = 0;
  auto take = [&](int64_t bytes) { int64_t r = o; o = align256(o + bytes); return r; };
  l.hdr = take(8 * 8);
  l.d_a = take(8 * H);
  l.d_b = take(8 * P);
  l.d_c = take(8 * (int64_t)L * H);
  l.d_W1t = take(8 * (int64_t)P * H);
  l.d_Bt = take(8 * (int64_t)L * P * H);
  l.f_a = take(4 * H);
  l.f_c = take(4 * (int64_t)L * H);
  l.f_W1t = take(4 * (int64_t)P * H);
  l.f_Bt = take(4 * (int64_t)L * P * H);
  l.x_W1 = take(8 * (int64_t)l.MB * l.S1 * 64);
  l.x_A = take(8 * (int64_t)L * l.MB * l.SH * 64);
  l.x_B = take(8 * (int64_t)L * l.MB * l.S1 * 64);
  l.y_W1 = take(4 * (int64_t)l.MB * l.S1 * 64);
  l.y_A = take(4 * (int64_t)L * l.MB * l.SH * 64);
  l.y_B = take(4 * (int64_t)L * l.MB * l.S1 * 64);
  l.z_W1 = take(16 * (int64_t)l.MB * 64);
  l.z_A = take(16 * (int64_t)L * l.MB * l.SHB * 64);
  l.z_B = take(16 * (int64_t)L * l.MB * 64);
  l.x_AT = take(8 * (int64_t)L * l.MB * l.SH * 64);
  l.y_AT = take(4 * (int64_t)L * l.MB * l.SH * 64);
  {
    const int npb = (P * (P + 1) / 2 + 15) / 16;
    l.x_G1 = take(8 * (int64_t)npb * l.MB * 4 * 64);
    l.y_G1 = take(4 * (int64_t)npb * l.MB * 4 * 64);
  }
  l.x_ATp = take(8 * (int64_t)L * l.MB * l.SH * 64);
  l.y_ATp = take(4 * (int64_t)L * l.MB * l.SH * 64);
  l.k0 = take(8 * (int64_t)P * 16);
  l.nout = take(8 * (int64_t)l.NOUT * 16);
  l.total = o;
  return l;
}

ThetaLayout theta_layout(int H, int L, int P, int has_bias) {
  ThetaLayout t{};
  t.H = H; t.L = L; t.P = P; t.has_bias = has_bias;
  int64_t o = 0;
  t.W1 = o; o += (int64_t)H * P;
  t.c1 = has_bias ? o : -1; o += has_bias ? H : 0;
  for (int k = 2; k <= L; ++k) {
    t.A[k] = o; o += (int64_t)H * H;
    t.B[k] = o; o += (int64_t)H * P;
    t.c[k] = has_bias ? o : -1; o += has_bias ? H : 0;
  }
  t.a = o; o += H;
  t.b = o; o += P;
  t.total = o;
  return t;
}

// ---------------------------------------------------------------- prepare
// Parameter accessors in the theta layout of width t.H; rows and columns at
// or beyond t.H are the zero padding of a narrow network.
__device__ inline double th_w(const double* th, const ThetaLayout& t, int k, int row, int col) {
  if (row >= t.H || (k >= 2 && col >= t.H)) return 0.0;
  return (k == 1) ? th[t.W1 + (int64_t)row * t.P + col] : th[t.A[k] + (int64_t)row * t.H + col];
}
__device__ inline double th_skip(const double* th, const ThetaLayout& t, int k, int row, int m) {
  return row < t.H ? th[t.B[k] + (int64_t)row * t.P + m] : 0.0;
}
__device__ inline double th_c(const double* th, const ThetaLayout& t, int k, int row) {
  const int64_t o = (k == 1) ? t.c1 : t.c[k];
  return (o < 0 || row >= t.H) ? 0.0 : th[o + row];
}

__global__ void k_prep_tables(const double* __restrict__ th, ThetaLayout t, PrepLayout l,
                              unsigned char* __restrict__ prep) {
  const int H = l.H, P = l.P, L = l.L;
  double* d_a = (double*)(prep + l.d_a);
  double* d_b = (double*)(prep + l.d_b);
  double* d_c = (double*)(prep + l.d_c);
  double* d_W1t = (double*)(prep + l.d_W1t);
  double* d_Bt = (double*)(prep + l.d_Bt);
  float* f_a = (float*)(prep + l.f_a);
  float* f_c = (float*)(prep + l.f_c);
  float* f_W1t = (float*)(prep + l.f_W1t);
  float* f_Bt = (float*)(prep + l.f_Bt);
  const int64_t total = H + P + (int64_t)L * H + (int64_t)P * H + (int64_t)L * P * H + 8 + (int64_t)P * 16;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    int64_t j = i;
    if (j < H) { double v = j < t.H ? th[t.a + j] : 0.0; d_a[j] = v; f_a[j] = (float)v; continue; }
    j -= H;
    if (j < P) { d_b[j] = th[t.b + j]; continue; }
    j -= P;
    if (j < (int64_t)L * H) {
      const int k = (int)(j / H) + 1, row = (int)(j % H);
      const double v = th_c(th, t, k, row); d_c[j] = v; f_c[j] = (float)v; continue;
    }
    j -= (int64_t)L * H;
    if (j < (int64_t)P * H) {
      const int m = (int)(j / H), row = (int)(j % H);
      const double v = th_w(th, t, 1, row, m); d_W1t[j] = v; f_W1t[j] = (float)v; continue;
    }
    j -= (int64_t)P * H;
    if (j < (int64_t)L * P * H) {
      const int k = (int)(j / ((int64_t)P * H)) + 1;
      const int m = (int)((j / H) % P), row = (int)(j % H);
      const double v = (k >= 2) ? th_skip(th, t, k, row, m) : 0.0;
      d_Bt[j] = v; f_Bt[j] = (float)v; continue;
    }
    j -= (int64_t)L * P * H;
    if (j < 8) { ((double*)(prep + l.hdr))[j] = 0.0; continue; }
    j -= 8;
    ((double*)(prep + l.k0))[j] = 0.0;
  }
}

// Row of the 16x16 result held by lane group g in register v.
__device__ inline int row64(int g, int v) { return g + 4 * v; }
__device__ inline int row32(int g, int v) { return 4 * g + v; }

__global__ void k_prep_frags(const double* __restrict__ th, ThetaLayout t, PrepLayout l,
                             unsigned char* __restrict__ prep) {
  const int H = l.H, P = l.P, L = l.L, MB = l.MB, S1 = l.S1, SH = l.SH, SHB = l.SHB;
  double* xW1 = (double*)(prep + l.x_W1);
  double* xA = (double*)(prep + l.x_A);
  double* xB = (double*)(prep + l.x_B);
  float* yW1 = (float*)(prep + l.y_W1);
  float* yA = (float*)(prep + l.y_A);
  float* yB = (float*)(prep + l.y_B);
  __bf16* zW1 = (__bf16*)(prep + l.z_W1);
  __bf16* zA = (__bf16*)(prep + l.z_A);
  __bf16* zB = (__bf16*)(prep + l.z_B);
  const int64_t nW1 = (int64_t)MB * S1 * 64;
  const int64_t nA = (int64_t)L * MB * SH * 64;
  const int64_t nB = (int64_t)L * MB * S1 * 64;
  const int64_t nzW1 = (int64_t)MB * 64 * 8;
  const int64_t nzA = (int64_t)L * MB * SHB * 64 * 8;
  const int64_t nzB = (int64_t)L * MB * 64 * 8;
  const int64_t nAT = (int64_t)L * MB * SH * 64;
  double* xAT = (double*)(prep + l.x_AT);
  float* yAT = (float*)(prep + l.y_AT);
  const int P2 = P * (P + 1) / 2, NPB = (P2 + 15) / 16;
  const int64_t nG1 = (int64_t)NPB * MB * 4 * 64;
  double* xG1 = (double*)(prep + l.x_G1);
  float* yG1 = (float*)(prep + l.y_G1);
  const int64_t nATp = (int64_t)L * MB * SH * 64;
  double* xATp = (double*)(prep + l.x_ATp);
  float* yATp = (float*)(prep + l.y_ATp);
  const int64_t total = nW1 + nA + nB + nzW1 + nzA + nzB + nAT + nG1 + nATp;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t j = idx;
    if (j >= total - nATp) {  // [k-1][mb][s = 4 ob + v][lane]: A_k[16 ob + row(g, v)][16 mb + i]
      j -= total - nATp;
      const int lane = (int)(j % 64), s = (int)((j / 64) % SH);
      const int mb = (int)((j / (64 * SH)) % MB), k = (int)(j / (64 * SH * MB)) + 1;
      const int i = lane & 15, g = lane >> 4, ob = s / 4, v = s % 4;
      double v64 = 0.0, v32 = 0.0;
      if (k >= 2) {
        v64 = th_w(th, t, k, 16 * ob + row64(g, v), 16 * mb + i);
        v32 = th_w(th, t, k, 16 * ob + row32(g, v), 16 * mb + i);
      }
      xATp[j] = v64; yATp[j] = (float)v32;
      continue;
    }
    if (j >= total - nATp - nG1) {  // [pb][w][s][lane]: W1_rm W1_rn, pair 16 pb + i, row 16w + row(g, s)
      j -= total - nATp - nG1;
      const int lane = (int)(j % 64), s = (int)((j / 64) % 4);
      const int w = (int)((j / 256) % MB), pb = (int)(j / (256 * MB));
      const int i = lane & 15, g = lane >> 4, pair = 16 * pb + i;
      double v64 = 0.0, v32 = 0.0;
      if (pair < P2) {
        int h = pair, m = 0;
        while (h >= P - m) { h -= P - m; ++m; }
        const int nn = m + h;
        const int r64 = 16 * w + row64(g, s), r32 = 16 * w + row32(g, s);
        v64 = th_w(th, t, 1, r64, m) * th_w(th, t, 1, r64, nn);
        v32 = th_w(th, t, 1, r32, m) * th_w(th, t, 1, r32, nn);
      }
      xG1[j] = v64; yG1[j] = (float)v32;
      continue;
    }
    if (j < nW1) {  // [mb][s][lane]: W1[16mb + i][4s + g]
      const int lane = (int)(j % 64), s = (int)((j / 64) % S1), mb = (int)(j / (64 * S1));
      const int i = lane & 15, g = lane >> 4, col = 4 * s + g;
      const double v = col < P ? th_w(th, t, 1, 16 * mb + i, col) : 0.0;
      xW1[j] = v; yW1[j] = (float)v; continue;
    }
    j -= nW1;
    if (j < nA) {  // [k-1][w][s][lane]: A_k[16w + i][16mb + row(g, v)], s = 4mb + v
      const int lane = (int)(j % 64), s = (int)((j / 64) % SH);
      const int w = (int)((j / (64 * SH)) % MB), k = (int)(j / (64 * SH * MB)) + 1;
      const int i = lane & 15, g = lane >> 4, mb = s / 4, v = s % 4;
      double v64 = 0.0, v32 = 0.0;
      if (k >= 2) {
        v64 = th_w(th, t, k, 16 * w + i, 16 * mb + row64(g, v));
        v32 = th_w(th, t, k, 16 * w + i, 16 * mb + row32(g, v));
      }
      xA[j] = v64; yA[j] = (float)v32; continue;
    }
    j -= nA;
    if (j < nB) {  // [k-1][w][s][lane]: B_k[16w + i][4s + g]
      const int lane = (int)(j % 64), s = (int)((j / 64) % S1);
      const int w = (int)((j / (64 * S1)) % MB), k = (int)(j / (64 * S1 * MB)) + 1;
      const int i = lane & 15, g = lane >> 4, col = 4 * s + g;
      const double v = (k >= 2 && col < P) ? th_skip(th, t, k, 16 * w + i, col) : 0.0;
      xB[j] = v; yB[j] = (float)v; continue;
    }
    j -= nB;
    if (j < nzW1) {  // [mb][lane][e]: W1[16mb + i][8g + e]
      const int e = (int)(j % 8), lane = (int)((j / 8) % 64), mb = (int)(j / 512);
      const int i = lane & 15, g = lane >> 4, col = 8 * g + e;
      zW1[j] = (__bf16)(float)(col < P ? th_w(th, t, 1, 16 * mb + i, col) : 0.0);
      continue;
    }
    j -= nzW1;
    if (j < nzA) {  // [k-1][w][s][lane][e]; source row 32s + 4g + e (e<4), 32s + 16 + 4g + e-4
      const int e = (int)(j % 8), lane = (int)((j / 8) % 64), s = (int)((j / 512) % SHB);
      const int w = (int)((j / (512 * SHB)) % MB), k = (int)(j / (512 * SHB * MB)) + 1;
      const int i = lane & 15, g = lane >> 4;
      const int r = (e < 4) ? 32 * s + 4 * g + e : 32 * s + 16 + 4 * g + (e - 4);
      zA[j] = (__bf16)(float)((k >= 2 && r < H) ? th_w(th, t, k, 16 * w + i, r) : 0.0);
      continue;
    }
    j -= nzA;
    if (j >= nzB) {  // [k-1][w][s][lane]: A_k[4s + g][16w + i] (reverse products)
      j -= nzB;
      const int lane = (int)(j % 64), s = (int)((j / 64) % SH);
      const int w = (int)((j / (64 * SH)) % MB), k = (int)(j / (64 * SH * MB)) + 1;
      const int i = lane & 15, g = lane >> 4;
      const double v = (k >= 2) ? th_w(th, t, k, 4 * s + g, 16 * w + i) : 0.0;
      xAT[j] = v; yAT[j] = (float)v;
      continue;
    }
    {  // [k-1][w][lane][e]: B_k[16w + i][8g + e]
      const int e = (int)(j % 8), lane = (int)((j / 8) % 64);
      const int w = (int)((j / 512) % MB), k = (int)(j / (512 * MB)) + 1;
      const int i = lane & 15, g = lane >> 4, col = 8 * g + e;
      zB[j] = (__bf16)(float)((k >= 2 && col < P) ? th_skip(th, t, k, 16 * w + i, col) : 0.0);
    }
  }
}

// Normalisation: N0 = N(0), kappa_q = dN/dK_{4,q}(0) + 2 dN/dK_{5,q}(0);
// b_{4,q} -= kappa_q so that P(I) = 0; Psi = N - N0.
__global__ void k_prep_fold(PrepLayout l, unsigned char* __restrict__ prep, int normalize, int npair) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double* hdr = (double*)(prep + l.hdr);
  double* d_b = (double*)(prep + l.d_b);
  const double* out = (const double*)(prep + l.nout);
  if (!normalize) { for (int i = 0; i < 8; ++i) hdr[i] = 0.0; return; }
  // the network was evaluated at a single point, so out is [NOUT][1]
  hdr[0] = out[0];
  for (int q = 0; q < npair; ++q) {
    const double kap = out[1 + 3 + q] + 2.0 * out[1 + 3 + npair + q];
    hdr[1 + q] = kap;
    d_b[3 + q] -= kap;
  }
}

// ---------------------------------------------------------------- network kernel
template <int H, int L, int P, int PR>
struct MlpCfg {
  using EV = typename std::conditional<PR == PREC_F64, EngF64,
             typename std::conditional<PR == PREC_F32 || PR == PREC_BF16C, EngF32, EngBF16>::type>::type;
  using EH = typename std::conditional<PR == PREC_F64, EngF64,
             typename std::conditional<PR == PREC_F32, EngF32, EngBF16>::type>::type;
  using T = typename EV::T;
  static constexpr int MB = H / 16;
  static constexpr int NW = MB;
  static constexpr int P2 = P * (P + 1) / 2;
  static constexpr int NOUT = 1 + P + P2;
  static constexpr int CH = (L >= 3) ? 4 : 1;  // columns per LDS exchange chunk
};

template <int H, int L, int P, int PR>
__global__ void __launch_bounds__(64 * (H / 16))
k_mlp_fwd(const unsigned char* __restrict__ prep, PrepLayout lay, int64_t n,
          const double* __restrict__ Kin, double* __restrict__ out, int hess) {
  using C = MlpCfg<H, L, P, PR>;
  using EV = typename C::EV;
  using EH = typename C::EH;
  using T = typename C::T;
  constexpr int MB = C::MB, NW = C::NW, P2 = C::P2, NOUT = C::NOUT, CH = C::CH;
  constexpr int SHV = steps_hidden<EV, H>();
  constexpr int SHH = steps_hidden<EH, H>();
  constexpr int S1V = steps_input<EV, P>();
  constexpr bool SPLIT = !std::is_same<EV, EH>::value;

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, q = lane & 15, g = lane >> 4;
  const int64_t base = (int64_t)blockIdx.x * 16;
  const int64_t qp = base + q;
  const bool valid = qp < n;

  __shared__ T W1s[P][H];
  __shared__ double outp[NW][NOUT][16];
  __shared__ T xbuf[CH][H][16];

  const T* t_W1t = (const T*)(prep + (std::is_same<T, double>::value ? lay.d_W1t : lay.f_W1t));
  const T* t_a = (const T*)(prep + (std::is_same<T, double>::value ? lay.d_a : lay.f_a));
  const T* t_c = (const T*)(prep + (std::is_same<T, double>::value ? lay.d_c : lay.f_c));
  const T* t_Bt = (const T*)(prep + (std::is_same<T, double>::value ? lay.d_Bt : lay.f_Bt));
  const double* d_b = (const double*)(prep + lay.d_b);

  for (int i = tid; i < P * H; i += 64 * NW) W1s[i / H][i % H] = t_W1t[i];

  // ---- input features as B operands of the value engine
  typename EV::frag kB[S1V];
  if constexpr (EV::KS == 4) {
#pragma unroll
    for (int s = 0; s < S1V; ++s) {
      const int m = 4 * s + g;
      kB[s] = (valid && m < P) ? (T)Kin[(int64_t)m * n + qp] : (T)0;
    }
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int m = 8 * g + e;
      kB[0][e] = (__bf16)(float)((valid && m < P) ? Kin[(int64_t)m * n + qp] : 0.0);
    }
  }

  // ---- layer 1, all rows: y1 = W1 K + c1
  T s1[MB][4], t1[MB][4], z1[MB][4];
  {
    const typename EV::frag* fW1 = frag_ptr<EV>(prep, lay, 0);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      typename EV::frag a1[S1V];
#pragma unroll
      for (int s = 0; s < S1V; ++s) a1[s] = fW1[(mb * S1V + s) * 64 + lane];
      typename EV::acc acc = mma_in<EV, P>(a1, kB, zero_acc<EV>());
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * mb + EV::row(g, v);
        const T y = acc[v] + t_c[r];
        T f, f1, f2;
        softplus3(y, f, f1, f2);
        z1[mb][v] = f; s1[mb][v] = f1; t1[mb][v] = f2;
      }
    }
  }

  // ---- weights of layers 2..L for this wave's rows (registers)
  typename EV::frag AV[L - 1][SHV];
  typename EV::frag BV[L - 1][S1V];
  {
    const typename EV::frag* fA = frag_ptr<EV>(prep, lay, 1);
    const typename EV::frag* fB = frag_ptr<EV>(prep, lay, 2);
#pragma unroll
    for (int k = 2; k <= L; ++k) {
#pragma unroll
      for (int s = 0; s < SHV; ++s) AV[k - 2][s] = fA[(((k - 1) * MB + w) * SHV + s) * 64 + lane];
#pragma unroll
      for (int s = 0; s < S1V; ++s) BV[k - 2][s] = fB[(((k - 1) * MB + w) * S1V + s) * 64 + lane];
    }
  }
  T a_own[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) a_own[v] = t_a[16 * w + EV::row(g, v)];

  // stash of layers 2..L (own rows): F'(y), F''(y), dy/dK_m
  T sk[L - 1][4], tk[L - 1][4], dyk[L - 1][P][4];

  __syncthreads();  // W1s ready

  auto emit = [&](int col, const T (&o)[4], const T (&aw)[4]) {
    double pl = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) pl += (double)(aw[v] * o[v]);
    pl = group_sum(pl);
    if (g == 0) outp[w][col][q] = pl;
  };

  // ================= value column
  {
    T src[MB][4];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int v = 0; v < 4; ++v) src[mb][v] = z1[mb][v];
    static_for<L - 1>([&](auto KI) {
      constexpr int k = decltype(KI)::value + 2;
      if constexpr (k >= 3) {
        // gather all rows of layer k-1 from LDS
        __syncthreads();
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int v = 0; v < 4; ++v) src[mb][v] = xbuf[0][16 * mb + EV::row(g, v)][q];
        __syncthreads();
      }
      typename EV::acc acc = mma_src<EV, MB>(AV[k - 2], src, zero_acc<EV>());
      acc = mma_in<EV, P>(BV[k - 2], kB, acc);
      T o[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * w + EV::row(g, v);
        const T y = acc[v] + t_c[(k - 1) * H + r];
        T f, f1, f2;
        softplus3(y, f, f1, f2);
        sk[k - 2][v] = f1; tk[k - 2][v] = f2; o[v] = f;
      }
      if constexpr (k < L) {
#pragma unroll
        for (int v = 0; v < 4; ++v) xbuf[0][16 * w + EV::row(g, v)][q] = o[v];
      } else {
        emit(0, o, a_own);
      }
    });
  }

  // ================= gradient columns dz/dK_m
  constexpr int NGC = (P + CH - 1) / CH;
  static_for<NGC>([&](auto CI) {
    constexpr int c0 = decltype(CI)::value * CH;
    T o[CH][4];
    static_for<CH>([&](auto JI) {
      constexpr int j = decltype(JI)::value;
      constexpr int m = c0 + j;
      if constexpr (m < P) {
        T src[MB][4];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int v = 0; v < 4; ++v) src[mb][v] = s1[mb][v] * W1s[m][16 * mb + EV::row(g, v)];
        typename EV::acc acc = mma_src<EV, MB>(AV[0], src, zero_acc<EV>());
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 16 * w + EV::row(g, v);
          const T d = acc[v] + t_Bt[((int64_t)1 * P + m) * H + r];
          dyk[0][m][v] = d;
          o[j][v] = sk[0][v] * d;
        }
      }
    });
    if constexpr (L == 2) {
      static_for<CH>([&](auto JI) {
        constexpr int j = decltype(JI)::value;
        if constexpr (c0 + j < P) emit(1 + c0 + j, o[j], a_own);
      });
    } else {
      static_for<CH>([&](auto JI) {
        constexpr int j = decltype(JI)::value;
        if constexpr (c0 + j < P) {
#pragma unroll
          for (int v = 0; v < 4; ++v) xbuf[j][16 * w + EV::row(g, v)][q] = o[j][v];
        }
      });
      __syncthreads();
      static_for<CH>([&](auto JI) {
        constexpr int j = decltype(JI)::value;
        constexpr int m = c0 + j;
        if constexpr (m < P) {
          T src[MB][4];
#pragma unroll
          for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int v = 0; v < 4; ++v) src[mb][v] = xbuf[j][16 * mb + EV::row(g, v)][q];
          typename EV::acc acc = mma_src<EV, MB>(AV[1], src, zero_acc<EV>());
          T oo[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = 16 * w + EV::row(g, v);
            const T d = acc[v] + t_Bt[((int64_t)2 * P + m) * H + r];
            dyk[1][m][v] = d;
            oo[v] = sk[1][v] * d;
          }
          emit(1 + m, oo, a_own);
        }
      });
      __syncthreads();
    }
  });

  // ================= Hessian columns d2z/dK_m dK_n (m <= n)
  if (hess) {
  // For the split precision mode the value/gradient stash was produced by the
  // FP32 engine (rows 4g + v) and the BF16 engine uses the same row order.
  typename EH::frag AH[L - 1][SHH];
  if constexpr (SPLIT) {
    const typename EH::frag* fA = frag_ptr<EH>(prep, lay, 1);
#pragma unroll
    for (int k = 2; k <= L; ++k)
#pragma unroll
      for (int s = 0; s < SHH; ++s) AH[k - 2][s] = fA[(((k - 1) * MB + w) * SHH + s) * 64 + lane];
  }
  auto AHk = [&](int k) -> const typename EH::frag* {
    if constexpr (SPLIT) return AH[k - 2]; else return (const typename EH::frag*)AV[k - 2];
  };

  constexpr int NHC = (P2 + CH - 1) / CH;
  static_for<NHC>([&](auto CI) {
    constexpr int h0 = decltype(CI)::value * CH;
    T o[CH][4];
    static_for<CH>([&](auto JI) {
      constexpr int j = decltype(JI)::value;
      constexpr int h = h0 + j;
      if constexpr (h < P2) {
        constexpr int m = hess_m(h, P), nn = hess_n(h, P);
        T src[MB][4];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = 16 * mb + EH::row(g, v);
            src[mb][v] = t1[mb][v] * W1s[m][r] * W1s[nn][r];
          }
        typename EH::acc acc = mma_src<EH, MB>(AHk(2), src, zero_acc<EH>());
#pragma unroll
        for (int v = 0; v < 4; ++v)
          o[j][v] = sk[0][v] * (T)acc[v] + tk[0][v] * dyk[0][m][v] * dyk[0][nn][v];
      }
    });
    if constexpr (L == 2) {
      static_for<CH>([&](auto JI) {
        constexpr int j = decltype(JI)::value;
        if constexpr (h0 + j < P2) emit(1 + P + h0 + j, o[j], a_own);
      });
    } else {
      static_for<CH>([&](auto JI) {
        constexpr int j = decltype(JI)::value;
        if constexpr (h0 + j < P2) {
#pragma unroll
          for (int v = 0; v < 4; ++v) xbuf[j][16 * w + EH::row(g, v)][q] = o[j][v];
        }
      });
      __syncthreads();
      static_for<CH>([&](auto JI) {
        constexpr int j = decltype(JI)::value;
        constexpr int h = h0 + j;
        if constexpr (h < P2) {
          constexpr int m = hess_m(h, P), nn = hess_n(h, P);
          T src[MB][4];
#pragma unroll
          for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int v = 0; v < 4; ++v) src[mb][v] = xbuf[j][16 * mb + EH::row(g, v)][q];
          typename EH::acc acc = mma_src<EH, MB>(AHk(3), src, zero_acc<EH>());
          T oo[4];
#pragma unroll
          for (int v = 0; v < 4; ++v)
            oo[v] = sk[1][v] * (T)acc[v] + tk[1][v] * dyk[1][m][v] * dyk[1][nn][v];
          emit(1 + P + h, oo, a_own);
        }
      });
      __syncthreads();
    }
  });

  }  // hess

  // ================= cross-wave sum in fixed order, skip term b.K, store
  __syncthreads();
  const int nout_written = hess ? NOUT : 1 + P;
  for (int i = tid; i < nout_written * 16; i += 64 * NW) {
    const int c = i / 16, qq = i % 16;
    const int64_t pt = base + qq;
    if (pt >= n) continue;
    double v = 0.0;
#pragma unroll
    for (int ww = 0; ww < NW; ++ww) v += outp[ww][c][qq];
    if (c == 0) {
      for (int m = 0; m < P; ++m) v += d_b[m] * Kin[(int64_t)m * n + pt];
    } else if (c <= P) {
      v += d_b[c - 1];
    }
    out[(int64_t)c * n + pt] = v;
  }
}

// ---------------------------------------------------------------- adjoint-form Hessian
// Same outputs as k_mlp_fwd.  The Hessian of N = a.z_L + b.K in the inputs is
//   d2N/dK dK = sum_k J_k^T diag(lambda_k (.) F''(y_k)) J_k,
// J_k = dy_k/dK (h x p), lambda_k = dN/dz_k, lambda_L = a,
// lambda_{k-1} = A_k^T (lambda_k (.) F'(y_k)),
// because every second derivative of N enters through the curvature of an
// activation (the layers are affine).  Passes per tile:
//   1. value forward (all layers);
//   2. reverse sweep for gamma_k = lambda_k (.) F''(y_k) (one column,
//      products with A_k^T);
//   3. layer 1: J_1 = W1 is constant, so its Gram sum is the matrix product
//      of the prepared table W1_rm W1_rn (pairs x rows) with gamma_1 (rows x
//      points) on the matrix cores;
//   4. Jacobian forward (p columns) for layers 2..L; each column's Gram
//      pairs (n <= m) are summed in registers as soon as the column is
//      formed, so the vector work overlaps the next column's matrix
//      products, and reduced four pairs at a time into the output tile.
// Points on the N dimension, neurons split across waves as in k_mlp_fwd.
// Pair t of the column-major upper triangle (m = column, n <= m).
__host__ __device__ constexpr int colmaj_m(int t) {
  int m = 0;
  while (t > m) { t -= m + 1; ++m; }
  return m;
}
__host__ __device__ constexpr int colmaj_n(int t) { return t - colmaj_m(t) * (colmaj_m(t) + 1) / 2; }
// Packed row-major index of pair (n, m), n <= m.
__host__ __device__ constexpr int packed_index(int n, int m, int P) { return n * P - n * (n - 1) / 2 + (m - n); }

template <int H, int L, int P, int PR, bool HESS, bool PERSIST = !HESS>
__global__ void __launch_bounds__(64 * (H / 16))
k_mlp_adj(const unsigned char* __restrict__ prep, PrepLayout lay, int64_t n,
          const double* __restrict__ Kin, double* __restrict__ out) {
  using E = typename std::conditional<PR == PREC_F64, EngF64, EngF32>::type;
  using T = typename E::T;
  using acc_t = typename E::acc;
  using frag_t = typename E::frag;
  constexpr int MB = H / 16, NW = MB, P2 = P * (P + 1) / 2, NOUT = 1 + P + P2;
  constexpr int SH = H / 4, S1 = (P + 3) / 4, NPB = (P2 + 15) / 16;
  constexpr int CH = (L >= 3) ? 3 : 1;  // gradient columns per LDS exchange chunk
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, q = lane & 15, g = lane >> 4;

  __shared__ T W1s[P][H];          // W1^T
  __shared__ T Bs[L - 1][P][H];    // B_k^T, k = 2..L
  __shared__ double outp[NW][NOUT][16];
  __shared__ T xbuf[CH][H][16];
  __shared__ T l1buf[2][H][16];
  __shared__ T cs[L][H], as_[H];   // biases and output weights

  const bool dbl = std::is_same<T, double>::value;
  const T* t_W1t = (const T*)(prep + (dbl ? lay.d_W1t : lay.f_W1t));
  const T* t_a = (const T*)(prep + (dbl ? lay.d_a : lay.f_a));
  const T* t_c = (const T*)(prep + (dbl ? lay.d_c : lay.f_c));
  const T* t_Bt = (const T*)(prep + (dbl ? lay.d_Bt : lay.f_Bt));
  const double* d_b = (const double*)(prep + lay.d_b);
  const frag_t* fW1 = frag_ptr<E>(prep, lay, 0);
  const frag_t* fA = frag_ptr<E>(prep, lay, 1);
  const frag_t* fB = frag_ptr<E>(prep, lay, 2);
  const frag_t* fAT = (const frag_t*)(prep + (dbl ? lay.x_AT : lay.y_AT));
  const frag_t* fG1 = (const frag_t*)(prep + (dbl ? lay.x_G1 : lay.y_G1));

  // ---- once per workgroup: weight tables in LDS, this wave's fragments and
  // per-row constants in registers (reused by every tile)
  for (int i = tid; i < P * H; i += 64 * NW) W1s[i / H][i % H] = t_W1t[i];
  for (int i = tid; i < (L - 1) * P * H; i += 64 * NW) (&Bs[0][0][0])[i] = t_Bt[(int64_t)P * H + i];
  frag_t a1[S1], AV[L - 1][SH], BV[L - 1][S1];
#pragma unroll
  for (int s = 0; s < S1; ++s) a1[s] = fW1[(w * S1 + s) * 64 + lane];
#pragma unroll
  for (int k = 2; k <= L; ++k) {
#pragma unroll
    for (int s = 0; s < SH; ++s) AV[k - 2][s] = fA[(((k - 1) * MB + w) * SH + s) * 64 + lane];
#pragma unroll
    for (int s = 0; s < S1; ++s) BV[k - 2][s] = fB[(((k - 1) * MB + w) * S1 + s) * 64 + lane];
  }
  // PREC_BF16C: the Jacobian pass of layers >= 2 runs on the BF16 matrix
  // cores (these fragments, K permuted to the FP32 accumulator layout);
  // value, reverse sweep, gradient and the layer-1 Gram stay FP32
  constexpr bool JB = PR == PREC_BF16C;
  constexpr int SHB = (H + 31) / 32;
  bf16x8 AZ[JB ? L - 1 : 1][JB ? SHB : 1];
  if constexpr (JB && HESS) {
    const bf16x8* zA = frag_ptr<EngBF16>(prep, lay, 1);
#pragma unroll
    for (int k = 2; k <= L; ++k)
#pragma unroll
      for (int s = 0; s < SHB; ++s) AZ[k - 2][s] = zA[(((k - 1) * MB + w) * SHB + s) * 64 + lane];
  }
  auto jac_product = [&](int kk, const T (&src)[MB][4]) -> acc_t {
    if constexpr (JB)
      return mma_src<EngBF16, MB>(AZ[kk], src, zero_acc<EngBF16>());
    else
      return mma_src<E, MB>(AV[kk], src, zero_acc<E>());
  };
  for (int i = tid; i < L * H; i += 64 * NW) (&cs[0][0])[i] = t_c[i];
  for (int i = tid; i < H; i += 64 * NW) as_[i] = t_a[i];
  __syncthreads();  // W1s, Bs, cs, as_

  const int64_t ntiles = (n + 15) / 16;
  auto tile_body = [&](int64_t tile) {
    const int64_t base = tile * 16;
    const int64_t qp = base + q;
    const bool valid = qp < n;
    frag_t kB[S1];
#pragma unroll
    for (int s = 0; s < S1; ++s) {
      const int m = 4 * s + g;
      kB[s] = (valid && m < P) ? (T)Kin[(int64_t)m * n + qp] : (T)0;
    }
    // layer 1: own rows, then z_1 and F'(y_1) of every row through LDS
    T t1w[4], s1w[4], z1[MB][4];
    {
      acc_t acc = mma_in<E, P>(a1, kB, zero_acc<E>());
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        T f, f1, f2;
        const int r = 16 * w + E::row(g, v);
        softplus3((T)(acc[v] + cs[0][r]), f, f1, f2);
        t1w[v] = f2;
        s1w[v] = f1;
        l1buf[0][r][q] = f;
        l1buf[1][r][q] = f1;
      }
    }
    __syncthreads();  // l1buf
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int v = 0; v < 4; ++v) z1[mb][v] = l1buf[0][16 * mb + E::row(g, v)][q];

    // ---- 1. value forward (own rows of layers 2..L)
    T sk[L - 1][4], tk[L - 1][4];
    {
      T src[MB][4];
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int v = 0; v < 4; ++v) src[mb][v] = z1[mb][v];
      static_for<L - 1>([&](auto KI) {
        constexpr int k = decltype(KI)::value + 2;
        if constexpr (k >= 3) {
          __syncthreads();
#pragma unroll
          for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int v = 0; v < 4; ++v) src[mb][v] = xbuf[0][16 * mb + E::row(g, v)][q];
          __syncthreads();
        }
        acc_t acc = mma_in<E, P>(BV[k - 2], kB, mma_src<E, MB>(AV[k - 2], src, zero_acc<E>()));
        T o[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          T f, f1, f2;
          softplus3((T)(acc[v] + cs[k - 1][16 * w + E::row(g, v)]), f, f1, f2);
          sk[k - 2][v] = f1; tk[k - 2][v] = f2; o[v] = f;
        }
        if constexpr (k < L) {
#pragma unroll
          for (int v = 0; v < 4; ++v) xbuf[0][16 * w + E::row(g, v)][q] = o[v];
        } else {
          double pl = 0.0;
#pragma unroll
          for (int v = 0; v < 4; ++v) pl += (double)(as_[16 * w + E::row(g, v)] * o[v]);
          pl = group_sum(pl);
          if (g == 0) outp[w][0][q] = pl;
        }
      });
    }

    // ---- 2. reverse sweep: mu_k = lambda_k (.) F'(y_k) and
    // gamma_k = lambda_k (.) F''(y_k), own rows
    T mus[L][4], gam[L][4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const T a = as_[16 * w + E::row(g, v)];
      gam[L - 1][v] = a * tk[L - 2][v];
      mus[L - 1][v] = a * sk[L - 2][v];
    }
    static_for<L - 1>([&](auto KI) {
      constexpr int k = L - decltype(KI)::value;  // L .. 2: lambda_{k-1} = A_k^T mu_k
      __syncthreads();
#pragma unroll
      for (int v = 0; v < 4; ++v) xbuf[0][16 * w + E::row(g, v)][q] = mus[k - 1][v];
      __syncthreads();
      const frag_t* at = fAT + (((k - 1) * MB + w) * SH) * 64 + lane;
      acc_t acc = zero_acc<E>();
#pragma unroll
      for (int s = 0; s < SH; ++s) acc = E::mma(at[s * 64], (frag_t)xbuf[0][4 * s + g][q], acc);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const T l = (T)acc[v];
        if constexpr (k - 1 >= 2) {
          gam[k - 2][v] = l * tk[k - 3][v];
          mus[k - 2][v] = l * sk[k - 3][v];
        } else {
          gam[0][v] = l * t1w[v];
          mus[0][v] = l * s1w[v];
        }
      }
    });

    // ---- 3. gradient: dN/dK_m = b_m + sum_rows mu_1 W1[., m] + sum_k mu_k B_k[., m]
    static_for<(P + 3) / 4>([&](auto BI) {
      constexpr int c0 = decltype(BI)::value * 4;
      double gp[4];
      static_for<4>([&](auto JI) {
        constexpr int j = decltype(JI)::value;
        T x = (T)0;
        if constexpr (c0 + j < P) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = 16 * w + E::row(g, v);
            x += mus[0][v] * W1s[c0 + j][r];
#pragma unroll
            for (int k = 2; k <= L; ++k) x += mus[k - 1][v] * Bs[k - 2][c0 + j][r];
          }
        }
        gp[j] = (double)x;
      });
      const double r = reduce4(gp[0], gp[1], gp[2], gp[3], g);
      if (c0 + g < P) outp[w][1 + c0 + g][q] = r;
    });

    if constexpr (HESS) {
      // ---- 4. layer-1 Gram on the matrix cores: rows of this wave's block,
      // B operand of K step s = gamma_1 at row(g, s) (already in registers)
#pragma unroll
      for (int pb = 0; pb < NPB; ++pb) {
        acc_t acc = zero_acc<E>();
#pragma unroll
        for (int s = 0; s < 4; ++s) acc = E::mma(fG1[((pb * MB + w) * 4 + s) * 64 + lane], (frag_t)gam[0][s], acc);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int pr = 16 * pb + E::row(g, v);
          if (pr < P2) outp[w][1 + P + pr][q] = (double)acc[v];  // table rows are packed pair indices
        }
      }

      // ---- 5. Jacobian forward; Gram pairs of layer k summed as columns form
      T J[P][4];  // dy_k/dK_m, own rows of the current layer
      double pp[4];
      // pair t (column-major) of layer k: sum over the wave's rows, flushed
      // every four pairs into outp at the packed positions of those pairs
      auto pair_sum = [&](auto TI, const T (&gm)[4]) {
        constexpr int t = decltype(TI)::value;
        constexpr int m = colmaj_m(t), nn = colmaj_n(t);
        T x = (T)0;
#pragma unroll
        for (int v = 0; v < 4; ++v) x += gm[v] * J[nn][v] * J[m][v];
        pp[t % 4] = (double)x;
        if constexpr (t % 4 == 3 || t == P2 - 1) {
          constexpr int c0 = t - t % 4;
#pragma unroll
          for (int j = t % 4 + 1; j < 4; ++j) pp[j] = 0.0;
          const double r = reduce4(pp[0], pp[1], pp[2], pp[3], g);
          constexpr int h0 = packed_index(colmaj_n(c0), colmaj_m(c0), P);
          constexpr int h1 = (c0 + 1 < P2) ? packed_index(colmaj_n(c0 + 1), colmaj_m(c0 + 1), P) : 0;
          constexpr int h2 = (c0 + 2 < P2) ? packed_index(colmaj_n(c0 + 2), colmaj_m(c0 + 2), P) : 0;
          constexpr int h3 = (c0 + 3 < P2) ? packed_index(colmaj_n(c0 + 3), colmaj_m(c0 + 3), P) : 0;
          const int h = g == 0 ? h0 : g == 1 ? h1 : g == 2 ? h2 : h3;
          if (c0 + g < P2) outp[w][1 + P + h][q] += r;
        }
      };
      static_for<L - 1>([&](auto KI) {
        constexpr int k = decltype(KI)::value + 2;
        if constexpr (k == 2) {
          static_for<P>([&](auto MI) {
            constexpr int m = decltype(MI)::value;
            T src[MB][4];
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                const int r = 16 * mb + E::row(g, v);
                src[mb][v] = l1buf[1][r][q] * W1s[m][r];
              }
            acc_t acc = jac_product(0, src);
#pragma unroll
            for (int v = 0; v < 4; ++v) J[m][v] = (T)acc[v] + Bs[0][m][16 * w + E::row(g, v)];
            static_for<m + 1>([&](auto NI) {
              pair_sum(std::integral_constant<int, m * (m + 1) / 2 + decltype(NI)::value>{}, gam[1]);
            });
          });
        } else {
          // exchange dz_{k-1}/dK_m = F'(y_{k-1}) J_{k-1} in chunks of CH columns
          static_for<(P + CH - 1) / CH>([&](auto CI) {
            constexpr int c0 = decltype(CI)::value * CH;
            __syncthreads();
            static_for<CH>([&](auto JI) {
              constexpr int m = c0 + decltype(JI)::value;
              if constexpr (m < P) {
#pragma unroll
                for (int v = 0; v < 4; ++v) xbuf[m - c0][16 * w + E::row(g, v)][q] = sk[k - 3][v] * J[m][v];
              }
            });
            __syncthreads();
            static_for<CH>([&](auto JI) {
              constexpr int m = c0 + decltype(JI)::value;
              if constexpr (m < P) {
                T src[MB][4];
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                  for (int v = 0; v < 4; ++v) src[mb][v] = xbuf[m - c0][16 * mb + E::row(g, v)][q];
                acc_t acc = jac_product(k - 2, src);
#pragma unroll
                for (int v = 0; v < 4; ++v) J[m][v] = (T)acc[v] + Bs[k - 2][m][16 * w + E::row(g, v)];
              }
            });
            // Gram pairs of the columns just formed (their partners n <= m are ready)
            static_for<CH>([&](auto JI) {
              constexpr int m = c0 + decltype(JI)::value;
              if constexpr (m < P)
                static_for<m + 1>([&](auto NI) {
                  pair_sum(std::integral_constant<int, m * (m + 1) / 2 + decltype(NI)::value>{}, gam[k - 1]);
                });
            });
          });
        }
      });
    }

    __syncthreads();  // outp complete
    constexpr int nout_written = HESS ? NOUT : 1 + P;
    for (int i = tid; i < nout_written * 16; i += 64 * NW) {
      const int c = i / 16, qq = i % 16;
      const int64_t pt = base + qq;
      if (pt >= n) continue;
      double v = 0.0;
#pragma unroll
      for (int ww = 0; ww < NW; ++ww) v += outp[ww][c][qq];
      if (c == 0) {
        for (int m = 0; m < P; ++m) v += d_b[m] * Kin[(int64_t)m * n + pt];
      } else if (c <= P) {
        v += d_b[c - 1];
      }
      out[(int64_t)c * n + pt] = v;
    }
    __syncthreads();  // outp, l1buf and xbuf free for the next tile
  };
  if constexpr (!PERSIST) {
    tile_body(blockIdx.x);  // one tile per workgroup (see the launcher)
  } else {
    // block-uniform tile loop: every wave of a workgroup runs the same
    // tiles, so the barriers inside tile_body match
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
      // with the Hessian, nothing read in the tile body stays live across tiles
      if constexpr (HESS) asm volatile("" ::: "memory");
      tile_body(tile);
    }
  }
}

// ---------------------------------------------------------------- two hidden layers, one wave per tile
// Same outputs as k_mlp_adj for networks with two hidden layers and width up
// to 32.  One wave owns a whole 16-point tile and every neuron (H/16 row
// blocks), so the layers chain register to register: the K steps of each
// product run in the order of the accumulator rows (row(g, v) of block mb),
// which is where the previous layer's values already sit in the lanes.  No
// barrier after the weight staging and no exchange through LDS; the layer-2
// Jacobian feeds no later layer, so it is formed one row block at a time,
// and the Hessian pairs are accumulated per wave in LDS and written once.
template <int H, int P, int PR, bool HESS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_mlp_adj2(const unsigned char* __restrict__ prep, PrepLayout lay, int64_t n,
           const double* __restrict__ Kin, double* __restrict__ out) {
  using E = typename std::conditional<PR == PREC_F64, EngF64, EngF32>::type;
  using T = typename E::T;
  using acc_t = typename E::acc;
  using frag_t = typename E::frag;
  constexpr int MB = H / 16, P2 = P * (P + 1) / 2;
  constexpr int SH = H / 4, S1 = (P + 3) / 4, NPB = (P2 + 15) / 16;
  constexpr int WPB = 4;  // waves, one tile each, per workgroup
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, q = lane & 15, g = lane >> 4;
  const uint32_t g8 = 8u * (uint32_t)g;

  __shared__ T W1s[P][H], B2s[P][H], c1s[H], c2s[H], as_[H];
  __shared__ double db_s[P];
  __shared__ double hb[HESS ? WPB : 1][HESS ? P2 : 1][16];
  // FP64: the layer-2 and layer-1 matrix-core fragments are staged once per
  // workgroup (LDS latency instead of L2 latency on every tile); FP32 reads
  // them from the prepared tables, which leaves LDS for more resident waves
  constexpr bool LT = PR == PREC_F64;
  constexpr int NW1 = MB * S1 * 64, NA2 = MB * SH * 64, NG1 = HESS ? NPB * MB * 4 * 64 : 1;
  __shared__ frag_t lW1[LT ? NW1 : 1], lA[LT ? NA2 : 1], lB[LT ? NW1 : 1], lATp[LT ? NA2 : 1], lG1[LT ? NG1 : 1];

  const bool dbl = std::is_same<T, double>::value;
  {
    const T* t_W1t = (const T*)(prep + (dbl ? lay.d_W1t : lay.f_W1t));
    const T* t_Bt = (const T*)(prep + (dbl ? lay.d_Bt : lay.f_Bt));
    const T* t_c = (const T*)(prep + (dbl ? lay.d_c : lay.f_c));
    const T* t_a = (const T*)(prep + (dbl ? lay.d_a : lay.f_a));
    for (int i = tid; i < P * H; i += 64 * WPB) {
      W1s[i / H][i % H] = t_W1t[i];
      B2s[i / H][i % H] = t_Bt[(int64_t)P * H + i];
    }
    for (int i = tid; i < H; i += 64 * WPB) {
      c1s[i] = t_c[i];
      c2s[i] = t_c[H + i];
      as_[i] = t_a[i];
    }
    for (int i = tid; i < P; i += 64 * WPB) db_s[i] = ((const double*)(prep + lay.d_b))[i];
    // layer 2 is index 1 of the per-layer fragment tables
    const frag_t* gW1 = frag_ptr<E>(prep, lay, 0);
    const frag_t* gA = frag_ptr<E>(prep, lay, 1) + NA2;
    const frag_t* gB = frag_ptr<E>(prep, lay, 2) + NW1;
    const frag_t* gATp = (const frag_t*)(prep + (dbl ? lay.x_ATp : lay.y_ATp)) + NA2;
    const frag_t* gG1 = (const frag_t*)(prep + (dbl ? lay.x_G1 : lay.y_G1));
    if constexpr (LT) {
      for (int i = tid; i < NW1; i += 64 * WPB) {
        lW1[i] = gW1[i];
        lB[i] = gB[i];
      }
      for (int i = tid; i < NA2; i += 64 * WPB) {
        lA[i] = gA[i];
        lATp[i] = gATp[i];
      }
      if constexpr (HESS)
        for (int i = tid; i < NG1; i += 64 * WPB) lG1[i] = gG1[i];
    }
  }
  const frag_t* fW1 = LT ? lW1 : frag_ptr<E>(prep, lay, 0);
  const frag_t* fA = LT ? lA : frag_ptr<E>(prep, lay, 1) + NA2;
  const frag_t* fB = LT ? lB : frag_ptr<E>(prep, lay, 2) + NW1;
  const frag_t* fATp = LT ? lATp : (const frag_t*)(prep + (dbl ? lay.x_ATp : lay.y_ATp)) + NA2;
  const frag_t* fG1 = LT ? lG1 : (const frag_t*)(prep + (dbl ? lay.x_G1 : lay.y_G1));
  __syncthreads();  // the only barrier: every wave reaches it before any exits
  const double* d_b = db_s;
  const int64_t ntiles = (n + 15) / 16;
  // this lane's inputs of a tile: feature 4 s + g of point q
  auto load_k = [&](int64_t tile, double (&kv)[S1]) {
    const int64_t qq = tile * 16 + q;
#pragma unroll
    for (int s = 0; s < S1; ++s) {
      const int m = 4 * s + g;
      kv[s] = (qq < n && m < P) ? Kin[(int64_t)m * n + qq] : 0.0;
    }
  };
  auto tile_body = [&](int64_t tile, const double (&kin)[S1]) {
  const int64_t base = tile * 16, qp = base + q;
  const bool valid = qp < n;

  frag_t kB[S1];
  double bK = 0.0;  // this lane's share of b . K, in FP64
#pragma unroll
  for (int s = 0; s < S1; ++s) {
    const int m = 4 * s + g;
    kB[s] = (T)kin[s];
    if (m < P) bK += d_b[m] * kin[s];
  }
  // ---- layer 1, every row block
  T z1[MB][4], s1[MB][4], t1[MB][4];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
    frag_t a1[S1];
#pragma unroll
    for (int s = 0; s < S1; ++s) a1[s] = fW1[(mb * S1 + s) * 64 + lane];
    const acc_t acc = mma_in<E, P>(a1, kB, zero_acc<E>());
#pragma unroll
    for (int v = 0; v < 4; ++v) softplus3((T)(acc[v] + c1s[16 * mb + E::row(g, v)]), z1[mb][v], s1[mb][v], t1[mb][v]);
  }
  // ---- layer 2, every row block; value, mu_2 = a F'(y_2), gamma_2 = a F''(y_2)
  T mu2[MB][4], gam2[MB][4];
  double val = 0.0;
#pragma unroll
  for (int ob = 0; ob < MB; ++ob) {
    frag_t AV[SH], BV[S1];
#pragma unroll
    for (int s = 0; s < SH; ++s) AV[s] = fA[(ob * SH + s) * 64 + lane];
#pragma unroll
    for (int s = 0; s < S1; ++s) BV[s] = fB[(ob * S1 + s) * 64 + lane];
    const acc_t acc = mma_in<E, P>(BV, kB, mma_src<E, MB>(AV, z1, zero_acc<E>()));
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * ob + E::row(g, v);
      T f, f1, f2;
      softplus3((T)(acc[v] + c2s[r]), f, f1, f2);
      const T a = as_[r];
      val += (double)(a * f);
      mu2[ob][v] = a * f1;
      gam2[ob][v] = a * f2;
    }
  }
  val = group_sum(val) + group_sum(bK);
  if (g == 0 && valid) out[qp] = val;
  // ---- reverse: lambda_1 = A_2^T mu_2 (K steps in accumulator-row order)
  T mu1[MB][4], gam1[MB][4];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
    acc_t acc = zero_acc<E>();
#pragma unroll
    for (int ob = 0; ob < MB; ++ob)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        acc = E::mma(fATp[(mb * SH + 4 * ob + v) * 64 + lane], (frag_t)mu2[ob][v], acc);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      mu1[mb][v] = (T)acc[v] * s1[mb][v];
      gam1[mb][v] = (T)acc[v] * t1[mb][v];
    }
  }
  // ---- gradient: b + W1^T mu_1 + B_2^T mu_2
  static_for<(P + 3) / 4>([&](auto BI) {
    constexpr int c0 = decltype(BI)::value * 4;
    double gp[4];
    static_for<4>([&](auto JI) {
      constexpr int j = decltype(JI)::value;
      T x = (T)0;
      if constexpr (c0 + j < P) {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = 16 * mb + E::row(g, v);
            x += mu1[mb][v] * W1s[c0 + j][r] + mu2[mb][v] * B2s[c0 + j][r];
          }
      }
      gp[j] = (double)x;
    });
    const double r = reduce4(gp[0], gp[1], gp[2], gp[3], g);
    if (c0 + g < P && valid) out[(int64_t)(1 + c0 + g) * n + qp] = r + d_b[c0 + g];
  });
  if constexpr (HESS) {
    // ---- layer-1 Gram on the matrix cores (table rows are packed pair indices)
#pragma unroll
    for (int pb = 0; pb < NPB; ++pb) {
      acc_t acc = zero_acc<E>();
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int s = 0; s < 4; ++s) acc = E::mma(fG1[((pb * MB + mb) * 4 + s) * 64 + lane], (frag_t)gam1[mb][s], acc);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int pr = 16 * pb + E::row(g, v);
        if (pr < P2) hb[w][pr][q] = (double)acc[v];
      }
    }
    asm volatile("" ::: "memory");
    // ---- layer-2 Jacobian, one row block at a time, Gram pairs as columns form
#pragma unroll 1
    for (int ob = 0; ob < MB; ++ob) {
      // PREC_BF16C: the layer-2 Jacobian contracts over the neurons on the
      // BF16 matrix cores (16x16x32, FP32 accumulation; the K dimension of
      // the prepared BF16 fragments is permuted to the FP32 accumulator
      // layout, so the column sources pack without shuffles); everything
      // else in this kernel is FP32
      constexpr bool JB = PR == PREC_BF16C;
      constexpr int SHB = (H + 31) / 32;
      frag_t AV[JB ? 1 : SH];
      bf16x8 AZ[JB ? SHB : 1];
      if constexpr (JB) {
        const bf16x8* zA = frag_ptr<EngBF16>(prep, lay, 1);
#pragma unroll
        for (int s = 0; s < SHB; ++s) AZ[s] = zA[((1 * MB + ob) * SHB + s) * 64 + lane];
      } else {
#pragma unroll
        for (int s = 0; s < SH; ++s) AV[s] = fA[(ob * SH + s) * 64 + lane];
      }
      T g2[4];  // gamma_2 of row block ob, selected without indexing registers at run time
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        g2[v] = gam2[0][v];
#pragma unroll
        for (int b = 1; b < MB; ++b) g2[v] = (ob == b) ? gam2[b][v] : g2[v];
      }
      // an opaque zero that changes identity every row block, so the
      // products s_1 W1 below are not hoisted out of this loop (they would
      // occupy 2 x 9 x 4 registers per lane)
      int zr = 0;
      asm volatile("" : "+v"(zr));
      // gJ[n] = gamma_2 * (column n of J_2) for the columns formed so far; the
      // column being paired, Jc, is held unscaled, so each pair term is one
      // multiply-add: sum_r gamma_r J_rn J_rm = sum_r gJ_rn Jc_rm
      T gJ[P][4], Jc[4];
      double pp[4];
      auto pair_sum = [&](auto TI) {
        constexpr int t = decltype(TI)::value;
        constexpr int nn = colmaj_n(t);
        T x = (T)0;
#pragma unroll
        for (int v = 0; v < 4; ++v) x += gJ[nn][v] * Jc[v];
        pp[t % 4] = (double)x;
        if constexpr (t % 4 == 3 || t == P2 - 1) {
          constexpr int c0 = t - t % 4;
#pragma unroll
          for (int j = t % 4 + 1; j < 4; ++j) pp[j] = 0.0;
          const double r = reduce4(pp[0], pp[1], pp[2], pp[3], g);
          constexpr int h0 = packed_index(colmaj_n(c0), colmaj_m(c0), P);
          constexpr int h1 = (c0 + 1 < P2) ? packed_index(colmaj_n(c0 + 1), colmaj_m(c0 + 1), P) : 0;
          constexpr int h2 = (c0 + 2 < P2) ? packed_index(colmaj_n(c0 + 2), colmaj_m(c0 + 2), P) : 0;
          constexpr int h3 = (c0 + 3 < P2) ? packed_index(colmaj_n(c0 + 3), colmaj_m(c0 + 3), P) : 0;
          // lane group g's pair index, without a branch: four bytes of one constant
          static_assert(P2 <= 256, "pair indices fit in a byte");
          constexpr uint32_t hpack = (uint32_t)h0 | (uint32_t)h1 << 8 | (uint32_t)h2 << 16 | (uint32_t)h3 << 24;
          const int h = (int)((hpack >> g8) & 0xffu);
          // each lane adds to its own entry, and a wave's LDS operations
          // complete in issue order: a fixed summation order without a wait
          if (c0 + 3 < P2 || c0 + g < P2) __hip_atomic_fetch_add(&hb[w][h][q], r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
      };
      static_for<P>([&](auto MI) {
        constexpr int m = decltype(MI)::value;
        T src[MB][4];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int v = 0; v < 4; ++v) src[mb][v] = s1[mb][v] * W1s[m][16 * mb + E::row(g, v) + zr];
        acc_t acc;
        if constexpr (JB)
          acc = mma_src<EngBF16, MB>(AZ, src, zero_acc<EngBF16>());
        else
          acc = mma_src<E, MB>(AV, src, zero_acc<E>());
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          Jc[v] = (T)acc[v] + B2s[m][16 * ob + E::row(g, v)];
          gJ[m][v] = g2[v] * Jc[v];
        }
        static_for<m + 1>([&](auto NI) { pair_sum(std::integral_constant<int, m * (m + 1) / 2 + decltype(NI)::value>{}); });
      });
    }
    asm volatile("" ::: "memory");
    // ---- the tile's Hessian: 16 consecutive points per packed pair
    for (int i = lane; i < P2 * 16; i += 64) {
      const int h = i / 16, qq = i % 16;
      if (base + qq < n) out[(int64_t)(1 + P + h) * n + base + qq] = hb[w][h][qq];
    }
  }
  };
  if constexpr (LT) {
    // persistent waves (the launcher sizes the grid to the resident
    // workgroups): each takes every (gridDim.x * WPB)-th tile, with the
    // next tile's inputs in flight while the current one is computed (the
    // body issues no other global load, so nothing waits on them early)
    const int64_t stride = (int64_t)gridDim.x * WPB;
    double kn[S1];
    int64_t tile = (int64_t)blockIdx.x * WPB + w;
    if (tile < ntiles) load_k(tile, kn);
    for (; tile < ntiles; tile += stride) {
      asm volatile("" ::: "memory");  // no fragment read is hoisted out of the tile loop
      double kc[S1];
#pragma unroll
      for (int s = 0; s < S1; ++s) kc[s] = kn[s];
      if (tile + stride < ntiles) load_k(tile + stride, kn);
      tile_body(tile, kc);
    }
  } else {
    const int64_t tile = (int64_t)blockIdx.x * WPB + w;
    if (tile < ntiles) {
      double kc[S1];
      load_k(tile, kc);
      tile_body(tile, kc);
    }
  }
}

// ---------------------------------------------------------------- dispatch
template <int H, int L, int P>
static int launch_mlp_t(const PrepLayout& lay, int prec, const unsigned char* prep, int64_t n,
                        const double* K, double* out, int hess, hipStream_t s) {
  const unsigned grid = (unsigned)((n + 15) / 16);
  const unsigned block = 64 * (H / 16);
  switch (prec) {
    case PREC_F64: k_mlp_fwd<H, L, P, PREC_F64><<<grid, block, 0, s>>>(prep, lay, n, K, out, hess); break;
    case PREC_F32: k_mlp_fwd<H, L, P, PREC_F32><<<grid, block, 0, s>>>(prep, lay, n, K, out, hess); break;
    case PREC_BF16: k_mlp_fwd<H, L, P, PREC_BF16><<<grid, block, 0, s>>>(prep, lay, n, K, out, hess); break;
    case PREC_BF16C: k_mlp_fwd<H, L, P, PREC_BF16C><<<grid, block, 0, s>>>(prep, lay, n, K, out, hess); break;
    default: return -1;
  }
  return 0;
}

#define PA_MLP_CONFIGS(X) \
  X(16, 2, 3) X(16, 2, 5) X(16, 2, 9) X(16, 3, 3) X(16, 3, 5) X(16, 3, 9) \
  X(32, 2, 3) X(32, 2, 5) X(32, 2, 9) X(32, 3, 3) X(32, 3, 5) X(32, 3, 9) \
  X(64, 2, 3) X(64, 2, 5) X(64, 2, 9) X(64, 3, 3) X(64, 3, 5) X(64, 3, 9)

// adjoint-form kernels: the forward-mode configurations and four hidden layers
#define PA_MLP_ADJ_CONFIGS(X) PA_MLP_CONFIGS(X) \
  X(16, 4, 3) X(16, 4, 5) X(16, 4, 9) X(32, 4, 3) X(32, 4, 5) X(32, 4, 9) X(64, 4, 3) X(64, 4, 5) X(64, 4, 9)

bool mlp_fwd_supported(int H, int L, int P) {
#define PA_SUP(h, l, p) if (H == h && L == l && P == p) return true;
  PA_MLP_CONFIGS(PA_SUP)
#undef PA_SUP
  return false;
}

bool mlp_supported(int H, int L, int P) {
#define PA_SUP(h, l, p) if (H == h && L == l && P == p) return true;
  PA_MLP_ADJ_CONFIGS(PA_SUP)
#undef PA_SUP
  return false;
}

// Persistent launch: as many workgroups as fit on the device at once (so the
// per-workgroup set-up is paid once per resident group), never more than the
// number of 16-point tiles.
template <class K>
static unsigned persistent_grid(K kernel, int block, int64_t ntiles) {
  static thread_local int cached_dev = -1, cached_cap = 0;
  static thread_local const void* cached_k = nullptr;
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (cached_k != (const void*)kernel || cached_dev != dev) {
    int cus = 0, per_cu = 0;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0);
    cached_cap = (cus > 0 ? cus : 256) * (per_cu > 0 ? per_cu : 1);
    cached_k = (const void*)kernel;
    cached_dev = dev;
  }
  return (unsigned)(ntiles < cached_cap ? ntiles : cached_cap);
}

// Workgroups of a kernel that fit on one CU at once (cached per kernel and device).
template <class K>
static int blocks_per_cu(K kernel, int block) {
  static thread_local const void* cached_k = nullptr;
  static thread_local int cached_dev = -1, cached = 0;
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (cached_k != (const void*)kernel || cached_dev != dev) {
    int per_cu = 0;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0);
    cached = per_cu;
    cached_k = (const void*)kernel;
    cached_dev = dev;
  }
  return cached;
}

template <int H, int L, int P, int PR, bool HESS>
static void launch_adj_one(const PrepLayout& lay, const unsigned char* prep, int64_t n, const double* K,
                           double* out, hipStream_t s) {
  const int block = 64 * (H / 16);
  const int64_t ntiles = (n + 15) / 16;
  if constexpr (!HESS) {
    k_mlp_adj<H, L, P, PR, false><<<persistent_grid(k_mlp_adj<H, L, P, PR, false>, block, ntiles), block, 0, s>>>(
        prep, lay, n, K, out);
  } else {
    // With the Hessian a tile loop keeps values live across tiles and costs
    // occupancy, so a workgroup takes one tile; only where that kernel fits a
    // single workgroup per CU anyway (FP64, large networks) are the
    // workgroups persistent, staging the weights once.
    if constexpr (PR == PREC_F64) {
      if (blocks_per_cu(k_mlp_adj<H, L, P, PR, true, false>, block) <= 1) {
        k_mlp_adj<H, L, P, PR, true, true><<<persistent_grid(k_mlp_adj<H, L, P, PR, true, true>, block, ntiles),
                                             block, 0, s>>>(prep, lay, n, K, out);
        return;
      }
    }
    k_mlp_adj<H, L, P, PR, true, false><<<(unsigned)ntiles, block, 0, s>>>(prep, lay, n, K, out);
  }
}

template <int H, int P, int PR, bool HESS>
static void launch_adj2_one(const PrepLayout& lay, const unsigned char* prep, int64_t n, const double* K,
                            double* out, hipStream_t s) {
  const int64_t nblk = ((n + 15) / 16 + 3) / 4;
  const unsigned grid = PR == PREC_F64 ? persistent_grid(k_mlp_adj2<H, P, PR, HESS>, 256, nblk) : (unsigned)nblk;
  k_mlp_adj2<H, P, PR, HESS><<<grid, 256, 0, s>>>(prep, lay, n, K, out);
}

template <int H, int L, int P>
static int launch_mlp_adj_t(const PrepLayout& lay, int prec, const unsigned char* prep, int64_t n,
                            const double* K, double* out, int hess, hipStream_t s) {
  if constexpr (L == 2 && H <= 32) {
    switch (prec) {
      case PREC_F64:
        if (hess) launch_adj2_one<H, P, PREC_F64, true>(lay, prep, n, K, out, s);
        else launch_adj2_one<H, P, PREC_F64, false>(lay, prep, n, K, out, s);
        return 0;
      case PREC_F32:
        if (hess) launch_adj2_one<H, P, PREC_F32, true>(lay, prep, n, K, out, s);
        else launch_adj2_one<H, P, PREC_F32, false>(lay, prep, n, K, out, s);
        return 0;
      case PREC_BF16C:  // FP32 value and gradient, layer-2 Jacobian in BF16
        if (hess) launch_adj2_one<H, P, PREC_BF16C, true>(lay, prep, n, K, out, s);
        else launch_adj2_one<H, P, PREC_F32, false>(lay, prep, n, K, out, s);
        return 0;
      default: return -2;
    }
  }
  switch (prec) {
    case PREC_F64:
      if (hess) launch_adj_one<H, L, P, PREC_F64, true>(lay, prep, n, K, out, s);
      else launch_adj_one<H, L, P, PREC_F64, false>(lay, prep, n, K, out, s);
      break;
    case PREC_F32:
      if (hess) launch_adj_one<H, L, P, PREC_F32, true>(lay, prep, n, K, out, s);
      else launch_adj_one<H, L, P, PREC_F32, false>(lay, prep, n, K, out, s);
      break;
    case PREC_BF16C:  // FP32 value and gradient, Jacobian pass in BF16
      if (hess) launch_adj_one<H, L, P, PREC_BF16C, true>(lay, prep, n, K, out, s);
      else launch_adj_one<H, L, P, PREC_F32, false>(lay, prep, n, K, out, s);
      break;
    default: return -2;
  }
  return 0;
}

int launch_mlp(const PrepLayout& lay, int prec, int algo, const unsigned char* prep, int64_t n,
               const double* K, double* out, int hess, hipStream_t s) {
  if (n == 0) return 0;
  if (algo == 1) {
#define PA_DISPATCH_ADJ(h, l, p) \
    if (lay.H == h && lay.L == l && lay.P == p) return launch_mlp_adj_t<h, l, p>(lay, prec, prep, n, K, out, hess, s);
    PA_MLP_ADJ_CONFIGS(PA_DISPATCH_ADJ)
#undef PA_DISPATCH_ADJ
    return -2;
  }
  if (algo != 0) return -2;
#define PA_DISPATCH(h, l, p) \
  if (lay.H == h && lay.L == l && lay.P == p) return launch_mlp_t<h, l, p>(lay, prec, prep, n, K, out, hess, s);
  PA_MLP_CONFIGS(PA_DISPATCH)
#undef PA_DISPATCH
  return -2;
}

int launch_prepare(const PrepLayout& lay, const ThetaLayout& tl, const double* theta,
                   unsigned char* prep, int normalize, int npair, hipStream_t s) {
  k_prep_tables<<<64, 256, 0, s>>>(theta, tl, lay, prep);
  k_prep_frags<<<256, 256, 0, s>>>(theta, tl, lay, prep);
  if (normalize) {
    const int algo = mlp_fwd_supported(lay.H, lay.L, lay.P) ? 0 : 1;
    int rc = launch_mlp(lay, PREC_F64, algo, prep, 1, (const double*)(prep + lay.k0),
                        (double*)(prep + lay.nout), 1, s);
    if (rc) return rc;
  }
  k_prep_fold<<<1, 64, 0, s>>>(lay, prep, normalize, npair);
  return 0;
}

}  // namespace pa
