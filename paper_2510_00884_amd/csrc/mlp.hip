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
  l.H = H; l.L = L; l.P = P; l.HR = H;
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
  {
    const int npb = (P * (P + 1) / 2 + 15) / 16;
    l.w_AT = take(16 * (int64_t)L * l.MB * l.SHB * 64);
    l.w_GT = take(16 * (int64_t)L * l.SHB * 64);
    l.w_G1 = take(16 * (int64_t)npb * l.SHB * 64);
  }
  l.d_Am = take(8 * (int64_t)L * H * H);
  l.f_Am = take(4 * (int64_t)L * H * H);
  l.x_AW = take(8 * (int64_t)P * l.MB * l.SH * 64);
  l.x_GT = take(8 * (int64_t)L * l.SH * 64);
  l.y_GT = take(4 * (int64_t)L * l.SH * 64);
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

// K position 8g + e of BF16 product step t -> neuron (the accumulator-row
// order of the previous product's result).
__device__ inline int kperm_row(int t, int g, int e) { return e < 4 ? 32 * t + 4 * g + e : 32 * t + 16 + 4 * g + e - 4; }

// Tables of the one-wave-per-tile kernels: the all-BF16 fragments (w_*),
// row-major A_k for the vector-ALU kernels (d_Am, f_Am), the FP64 layer-2
// Jacobian column tables (x_AW) and the gradient tables (x_GT, y_GT).
__global__ void k_prep_onewave(const double* __restrict__ th, ThetaLayout t, PrepLayout l,
                            unsigned char* __restrict__ prep) {
  const int H = l.H, P = l.P, L = l.L, MB = l.MB, SHB = l.SHB;
  const int P2 = P * (P + 1) / 2, NPB = (P2 + 15) / 16;
  __bf16* wAT = (__bf16*)(prep + l.w_AT);
  __bf16* wGT = (__bf16*)(prep + l.w_GT);
  __bf16* wG1 = (__bf16*)(prep + l.w_G1);
  const int64_t nAT = (int64_t)L * MB * SHB * 512, nGT = (int64_t)L * SHB * 512, nG1 = (int64_t)NPB * SHB * 512;
  const int64_t nAm = (int64_t)L * H * H, nAW = (int64_t)P * MB * l.SH * 64, nXG = (int64_t)L * l.SH * 64;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < nAT + nGT + nG1 + nAm + nAW + nXG;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t j = idx;
    if (j >= nAT + nGT + nG1 + nAm + nAW) {  // [k-1][s = 4 mb + v][lane]: W1[r][i] or B_k[r][i]
      j -= nAT + nGT + nG1 + nAm + nAW;
      const int ln = (int)(j % 64), s = (int)((j / 64) % l.SH), k = (int)(j / (64 * l.SH)) + 1;
      const int i = ln & 15, gg = ln >> 4;
      const int r64 = 16 * (s / 4) + row64(gg, s % 4), r32 = 16 * (s / 4) + row32(gg, s % 4);
      double v64 = 0.0, v32 = 0.0;
      if (i < P) {
        v64 = (k == 1) ? th_w(th, t, 1, r64, i) : th_skip(th, t, k, r64, i);
        v32 = (k == 1) ? th_w(th, t, 1, r32, i) : th_skip(th, t, k, r32, i);
      }
      ((double*)(prep + l.x_GT))[j] = v64;
      ((float*)(prep + l.y_GT))[j] = (float)v32;
      continue;
    }
    if (j >= nAT + nGT + nG1 + nAm) {  // FP64 [m][ob][s = 4 mb + v][lane]: A_2[16 ob + i][q] W1[q][m]
      j -= nAT + nGT + nG1 + nAm;
      const int ln = (int)(j % 64), s = (int)((j / 64) % l.SH), ob = (int)((j / (64 * l.SH)) % MB);
      const int m = (int)(j / (64 * l.SH * MB));
      const int q = 16 * (s / 4) + row64(ln >> 4, s % 4), r = 16 * ob + (ln & 15);
      ((double*)(prep + l.x_AW))[j] = (L >= 2) ? th_w(th, t, 2, r, q) * th_w(th, t, 1, q, m) : 0.0;
      continue;
    }
    if (j >= nAT + nGT + nG1) {  // row-major A_k for the vector-ALU kernels: [k-1][r][q]
      j -= nAT + nGT + nG1;
      const int k = (int)(j / ((int64_t)H * H)) + 1, r = (int)((j / H) % H), q = (int)(j % H);
      const double v = (k >= 2) ? th_w(th, t, k, r, q) : 0.0;
      ((double*)(prep + l.d_Am))[j] = v;
      ((float*)(prep + l.f_Am))[j] = (float)v;
      continue;
    }
    const int e = (int)(j % 8), lane = (int)((j / 8) % 64), i = lane & 15, g = lane >> 4;
    if (j < nAT) {  // [k-1][mb][tt][lane][e]: A_k[r][16 mb + i]
      const int tt = (int)((j / 512) % SHB), mb = (int)((j / (512 * SHB)) % MB), k = (int)(j / (512 * SHB * MB)) + 1;
      const int r = kperm_row(tt, g, e);
      wAT[j] = (__bf16)(float)((k >= 2 && r < H) ? th_w(th, t, k, r, 16 * mb + i) : 0.0);
      continue;
    }
    j -= nAT;
    if (j < nGT) {  // [k-1][tt][lane][e]: W1[r][i] or B_k[r][i]
      const int tt = (int)((j / 512) % SHB), k = (int)(j / (512 * SHB)) + 1;
      const int r = kperm_row(tt, g, e);
      double v = 0.0;
      if (i < P && r < H) v = (k == 1) ? th_w(th, t, 1, r, i) : th_skip(th, t, k, r, i);
      wGT[j] = (__bf16)(float)v;
      continue;
    }
    j -= nGT;
    {  // [pb][tt][lane][e]: W1[r][m] W1[r][nn], pair 16 pb + i = (m, nn), m <= nn, row-major packed
      const int tt = (int)((j / 512) % SHB), pb = (int)(j / (512 * SHB));
      const int r = kperm_row(tt, g, e), pair = 16 * pb + i;
      double v = 0.0;
      if (pair < P2 && r < H) {
        int h = pair, m = 0;
        while (h >= P - m) { h -= P - m; ++m; }
        v = th_w(th, t, 1, r, m) * th_w(th, t, 1, r, m + h);
      }
      wG1[j] = (__bf16)(float)v;
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

// ---------------------------------------------------------------- dispatch
// Network kernels are instantiated per width in mlp_fwd_h*.hip (forward
// mode) and mlp_adj_h*.hip (adjoint form).
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

int launch_mlp(const PrepLayout& lay, int prec, int algo, const unsigned char* prep, int64_t n,
               const double* K, double* out, int hess, hipStream_t s) {
  if (n == 0) return 0;
  if (algo == 1) {
    if (!mlp_supported(lay.H, lay.L, lay.P)) return -2;
    // widths up to 8 in FP64 and FP32: one point per lane on the vector ALUs
    if (lay.HR <= 8 && (prec == PREC_F64 || prec == PREC_F32)) return launch_mlp_valu(lay, prec, prep, n, K, out, hess, s);
    switch (lay.H) {
      case 16: return launch_mlp_adj_h16(lay, prec, prep, n, K, out, hess, s);
      case 32: return launch_mlp_adj_h32(lay, prec, prep, n, K, out, hess, s);
      case 64: return launch_mlp_adj_h64(lay, prec, prep, n, K, out, hess, s);
      default: return -2;
    }
  }
  if (algo != 0 || !mlp_fwd_supported(lay.H, lay.L, lay.P)) return -2;
  switch (lay.H) {
    case 16: return launch_mlp_fwd_h16(lay, prec, prep, n, K, out, hess, s);
    case 32: return launch_mlp_fwd_h32(lay, prec, prep, n, K, out, hess, s);
    case 64: return launch_mlp_fwd_h64(lay, prec, prep, n, K, out, hess, s);
    default: return -2;
  }
}

int launch_prepare(const PrepLayout& lay, const ThetaLayout& tl, const double* theta,
                   unsigned char* prep, int normalize, int npair, hipStream_t s) {
  k_prep_tables<<<64, 256, 0, s>>>(theta, tl, lay, prep);
  k_prep_frags<<<256, 256, 0, s>>>(theta, tl, lay, prep);
  k_prep_onewave<<<64, 256, 0, s>>>(theta, tl, lay, prep);
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
