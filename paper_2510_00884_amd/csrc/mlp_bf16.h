// Adjoint-form network kernel with every contraction on the BF16 matrix
// cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation) and FP32 activations:
// the value forward, the reverse sweep, the input gradient, the layer-1 Gram
// term and the Jacobian forward of the Hessian
//   d2N/dK dK = sum_k J_k^T diag(gamma_k) J_k,   gamma_k = lambda_k (.) F''(y_k),
// (same outputs as the forward mode of Alg. 4 up to BF16 rounding).
//
// One wave owns a 16-point tile and every neuron, so layers chain register to
// register: a product's result rows (4g + v of each 16-row block, lane
// group g) are packed straight into the next product's B operand, with the K
// dimension of the prepared fragments permuted to that order (K position
// 8g + e of step t is neuron 32t + 4g + e for e < 4 and 32t + 16 + 4g + e - 4
// otherwise).  The gradient and the layer-1 Gram are matrix products whose
// result rows are the inputs and the input pairs.  The Hessian pairs of the
// later layers are sums over neurons of products of two Jacobian columns;
// they run on the packed-BF16 dot instruction (two products per
// instruction) into per-lane FP32 partials that are reduced across lane
// groups once per tile.  The Jacobian of the last layer is formed one row
// block at a time (it feeds nothing else); with three hidden layers the
// layer-2 Jacobian is formed whole, kept only as the packed layer-3 sources
// s_2 (.) J_2, and its Gram term is taken from those sources with the
// weights gamma_2 / s_2^2.
#pragma once
#include <type_traits>
#include <utility>

#include "mma_util.h"
#include "pa_internal.h"

namespace pa {

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f2 __attribute__((ext_vector_type(2)));

__device__ inline bf16x2 pk_bf16(float a, float b) { return __builtin_convertvector((f2){a, b}, bf16x2); }

__device__ inline float dot2(bf16x2 a, bf16x2 b, float c) { return __builtin_amdgcn_fdot2_f32_bf16(a, b, c, false); }

// Eight FP32 values into one BF16 operand (round to nearest even).
__device__ inline bf16x8 pack8(const float (&lo)[4], const float (&hi)[4]) {
  const bf16x2 p0 = pk_bf16(lo[0], lo[1]), p1 = pk_bf16(lo[2], lo[3]);
  const bf16x2 p2 = pk_bf16(hi[0], hi[1]), p3 = pk_bf16(hi[2], hi[3]);
  return (bf16x8){p0[0], p0[1], p1[0], p1[1], p2[0], p2[1], p3[0], p3[1]};
}

// Accumulator-layout rows of every block -> the SHB B operands of a product
// over the neurons (blocks 2t and 2t + 1 in step t; a missing odd block is 0).
template <int MB>
__device__ inline void pack_rows(const float (&x)[MB][4], bf16x8 (&o)[(MB + 1) / 2]) {
  constexpr float zero[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < (MB + 1) / 2; ++t) o[t] = pack8(x[2 * t], (2 * t + 1 < MB) ? x[2 * t + 1] : zero);
}

// Half h (elements 4h .. 4h + 3) of a BF16 operand as two packed pairs.
__device__ inline void half_pairs(const bf16x8& x, int h, bf16x2& a, bf16x2& b) {
  a = h ? (bf16x2){x[4], x[5]} : (bf16x2){x[0], x[1]};
  b = h ? (bf16x2){x[6], x[7]} : (bf16x2){x[2], x[3]};
}

__device__ inline float bf16_to_f32(__bf16 x) { return (float)x; }

// Softplus, F' and F'' from the hardware base-2 exponential and logarithm and
// the reciprocal estimate (about one ulp each): e = e^{-|y|},
// F = max(y, 0) + ln(1 + e), F' = 1/(1 + e) (y >= 0) or e/(1 + e), F'' =
// e/(1 + e)^2.  ln(1 + e) is formed from the rounded 1 + e, an absolute
// error of a few 1e-8, far below the BF16 rounding of every product here.
__device__ inline void softplus3_fast(float y, float& f, float& f1, float& f2) {
  const float e = __builtin_amdgcn_exp2f(-fabsf(y) * 1.44269504088896341f);
  const float d = 1.0f + e;
  const float r = __builtin_amdgcn_rcpf(d);
  f = fmaxf(y, 0.0f) + __builtin_amdgcn_logf(d) * 0.693147180559945309f;
  f1 = (y >= 0.0f) ? r : e * r;
  f2 = e * r * r;
}

// Cross-lane sums in FP32 through lane shuffles.  (The in-place lane-swap
// instructions exchange two registers; the compiler folds such swaps
// wrongly when an operand is a known constant, e.g. the zero partial of a
// missing pair, so they are not used here.)
// Sum over the four lane groups; every lane receives the sum for its column.
__device__ inline float group_sum_f(float x) {
  x += __shfl_xor(x, 16);
  return x + __shfl_xor(x, 32);
}
// Lane group g receives the sum of p_g over the four lane groups: halve the
// set of partials a lane carries at each exchange (three shuffles).
__device__ inline float reduce4f(float p0, float p1, float p2, float p3, int g) {
  const bool lo = g < 2, even = (g & 1) == 0;
  const float a = (lo ? p0 : p2) + __shfl_xor(lo ? p2 : p0, 32);  // p0 (g < 2) or p2 (g >= 2), groups {g, g ^ 2}
  const float b = (lo ? p1 : p3) + __shfl_xor(lo ? p3 : p1, 32);  // p1 or p3 likewise
  return (even ? a : b) + __shfl_xor(even ? b : a, 16);
}

// Waves per SIMD the register budget is sized for: two (256 registers) for
// two hidden layers; one (512) for three, whose Hessian pass keeps the
// packed layer-3 sources of every input column live.
template <int L, bool HESS>
constexpr int bf16_waves() { return (L == 3 && HESS) ? 1 : 2; }

template <int H, int L, int P, bool HESS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(bf16_waves<L, HESS>())))
k_mlp_bf16(const unsigned char* __restrict__ prep, PrepLayout lay, int64_t n, const double* __restrict__ Kin,
           double* __restrict__ out) {
  static_assert(L == 2 || L == 3, "two or three hidden layers");
  static_assert(P <= 16, "inputs fit one K step");
  constexpr int MB = H / 16, SHB = (MB + 1) / 2, P2 = P * (P + 1) / 2, NPB = (P2 + 15) / 16;
  constexpr int WPB = 4;  // waves (one tile each) per workgroup
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, q = lane & 15, g = lane >> 4;

  // matrix-core fragments (one 16-byte entry per lane), staged once
  __shared__ bf16x8 sW1[MB * 64];                    // [mb][lane]: W1
  __shared__ bf16x8 sA[(L - 1) * MB * SHB * 64];     // [k-2][ob][t][lane]: A_k
  __shared__ bf16x8 sB[(L - 1) * MB * 64];           // [k-2][ob][lane]: B_k
  __shared__ bf16x8 sAT[(L - 1) * MB * SHB * 64];    // [k-2][mb][t][lane]: A_k^T
  __shared__ bf16x8 sGT[L * SHB * 64];               // [k-1][t][lane]: W1^T, B_k^T
  __shared__ bf16x8 sG1[HESS ? NPB * SHB * 64 : 1];  // [pb][t][lane]: W1_rm W1_rn
  // FP32 rows (float4 over 4 consecutive neurons)
  __shared__ __align__(16) float sW1t[P * H];        // [m][r] = W1[r][m]
  __shared__ __align__(16) float sBt[(L - 1) * P * H];  // [k-2][m][r] = B_k[r][m]
  __shared__ __align__(16) float sc[L * H];          // [k-1][r]
  __shared__ __align__(16) float sa[H];
  __shared__ double sdb[P];
  __shared__ __align__(16) float kbuf[WPB][16][16];  // per wave: a tile's inputs, [point][input]
  {
    const bf16x8* gW1 = (const bf16x8*)(prep + lay.z_W1);
    const bf16x8* gA = (const bf16x8*)(prep + lay.z_A) + MB * SHB * 64;  // tables start at layer 1
    const bf16x8* gB = (const bf16x8*)(prep + lay.z_B) + MB * 64;
    const bf16x8* gAT = (const bf16x8*)(prep + lay.w_AT) + MB * SHB * 64;
    const bf16x8* gGT = (const bf16x8*)(prep + lay.w_GT);
    const bf16x8* gG1 = (const bf16x8*)(prep + lay.w_G1);
    for (int i = tid; i < MB * 64; i += 64 * WPB) sW1[i] = gW1[i];
    for (int i = tid; i < (L - 1) * MB * SHB * 64; i += 64 * WPB) {
      sA[i] = gA[i];
      sAT[i] = gAT[i];
    }
    for (int i = tid; i < (L - 1) * MB * 64; i += 64 * WPB) sB[i] = gB[i];
    for (int i = tid; i < L * SHB * 64; i += 64 * WPB) sGT[i] = gGT[i];
    if constexpr (HESS)
      for (int i = tid; i < NPB * SHB * 64; i += 64 * WPB) sG1[i] = gG1[i];
    const float* fW1t = (const float*)(prep + lay.f_W1t);
    const float* fBt = (const float*)(prep + lay.f_Bt);
    const float* fc = (const float*)(prep + lay.f_c);
    const float* fa = (const float*)(prep + lay.f_a);
    for (int i = tid; i < P * H; i += 64 * WPB) sW1t[i] = fW1t[i];
    for (int i = tid; i < (L - 1) * P * H; i += 64 * WPB) sBt[i] = fBt[P * H + i];  // layer k >= 2 at k - 1
    for (int i = tid; i < L * H; i += 64 * WPB) sc[i] = fc[i];
    for (int i = tid; i < H; i += 64 * WPB) sa[i] = fa[i];
    for (int i = tid; i < P; i += 64 * WPB) sdb[i] = ((const double*)(prep + lay.d_b))[i];
    for (int i = tid; i < WPB * 16 * 16; i += 64 * WPB) (&kbuf[0][0][0])[i] = 0.f;  // inputs >= P stay 0
  }
  __syncthreads();  // the only barrier: every wave reaches it before any exits

  auto row4 = [&](const float* base, int mb) -> f4 { return *(const f4*)(base + 16 * mb + 4 * g); };
  auto mfma = [](const bf16x8& a, const bf16x8& b, f4 c) -> f4 {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  };
  const int64_t ntiles = (n + 15) / 16;
  // this lane's inputs of a tile: features g + 4j of point q (coalesced over
  // the 16 points of a lane group)
  constexpr int S1 = (P + 3) / 4;
  auto load_k = [&](int64_t tile, double (&kv)[S1]) {
    int64_t qq = tile * 16 + q;
    asm volatile("" : "+v"(qq));  // one opaque index: no per-column address streams across tiles
#pragma unroll
    for (int j = 0; j < S1; ++j) {
      const int m = g + 4 * j;
      kv[j] = (qq < n && m < P) ? Kin[(int64_t)m * n + qq] : 0.0;
    }
  };

  auto tile_body = [&](int64_t tile, const double (&kv)[S1]) {
    int64_t qp = tile * 16 + q;
    // opaque per tile, so the per-lane column addresses of the outputs are
    // formed at each store instead of being held (or spilled) across tiles
    int64_t ns = n;
    asm volatile("" : "+v"(qp), "+s"(ns));
    const bool valid = qp < n;
    // the B operand of the input products wants features 8g .. 8g + 7 of
    // point q in lane (g, q): regroup through this wave's LDS rows (a wave's
    // LDS accesses complete in issue order)
    bf16x8 kb;
    double bK = 0.0;  // this lane's share of b . K, in FP64
#pragma unroll
    for (int j = 0; j < S1; ++j) {
      const int m = g + 4 * j;
      if (m < P) {
        kbuf[w][q][m] = (float)kv[j];
        bK += sdb[m] * kv[j];
      }
    }
    asm volatile("" ::: "memory");
    {
      // inputs 8g .. 8g + 7; lane groups 2 and 3 hold inputs >= 16 (none)
      const f4 zero = {0.f, 0.f, 0.f, 0.f};
      const f4 lo = g < 2 ? *(const f4*)&kbuf[w][q][8 * (g & 1)] : zero;
      const f4 hi = g < 2 ? *(const f4*)&kbuf[w][q][8 * (g & 1) + 4] : zero;
      const float l4[4] = {lo[0], lo[1], lo[2], lo[3]}, h4[4] = {hi[0], hi[1], hi[2], hi[3]};
      kb = pack8(l4, h4);
    }
    asm volatile("" ::: "memory");

    // ---- value forward
    float s1[MB][4], t1[MB][4];
    float sK[L - 1][MB][4], tK[L - 1][MB][4];  // F', F'' of layers 2..L
    bf16x8 zsrc[SHB];
    {
      float z[MB][4];
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        const f4 acc = mfma(sW1[mb * 64 + lane], kb, (f4){0.f, 0.f, 0.f, 0.f});
        const f4 c = row4(sc, mb);
#pragma unroll
        for (int v = 0; v < 4; ++v) softplus3_fast(acc[v] + c[v], z[mb][v], s1[mb][v], t1[mb][v]);
      }
      pack_rows<MB>(z, zsrc);
    }
    float val = 0.f;
    static_for<L - 1>([&](auto KI) {
      constexpr int k = decltype(KI)::value + 2;
      float z[MB][4];
#pragma unroll
      for (int ob = 0; ob < MB; ++ob) {
        f4 acc = mfma(sB[((k - 2) * MB + ob) * 64 + lane], kb, (f4){0.f, 0.f, 0.f, 0.f});
#pragma unroll
        for (int t = 0; t < SHB; ++t) acc = mfma(sA[(((k - 2) * MB + ob) * SHB + t) * 64 + lane], zsrc[t], acc);
        const f4 c = row4(sc + (k - 1) * H, ob);
#pragma unroll
        for (int v = 0; v < 4; ++v) softplus3_fast(acc[v] + c[v], z[ob][v], sK[k - 2][ob][v], tK[k - 2][ob][v]);
      }
      if constexpr (k < L) {
        pack_rows<MB>(z, zsrc);
      } else {
#pragma unroll
        for (int ob = 0; ob < MB; ++ob) {
          const f4 a = row4(sa, ob);
#pragma unroll
          for (int v = 0; v < 4; ++v) val = fmaf(a[v], z[ob][v], val);
        }
      }
    });
    {
      const double v = (double)group_sum_f(val) + group_sum(bK);
      if (g == 0 && valid) out[qp] = v;
    }

    // ---- reverse sweep: mu_k = lambda_k F'(y_k), gamma_k = lambda_k F''(y_k);
    // the gradient W1^T mu_1 + sum_k B_k^T mu_k accumulates on the matrix cores
    float gm[L - 1][MB][4];  // gamma of layers 2..L (kept for the Jacobian pass)
    float g1[MB][4];         // gamma_1
    float lam2[L == 3 ? MB : 1][4];  // lambda_2 (three hidden layers)
    f4 gacc = {0.f, 0.f, 0.f, 0.f};
    {
      float mu[MB][4];
#pragma unroll
      for (int ob = 0; ob < MB; ++ob) {
        const f4 a = row4(sa, ob);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          mu[ob][v] = a[v] * sK[L - 2][ob][v];
          gm[L - 2][ob][v] = a[v] * tK[L - 2][ob][v];
        }
      }
      static_for<L - 1>([&](auto KI) {
        constexpr int k = L - decltype(KI)::value;  // L .. 2: lambda_{k-1} = A_k^T mu_k
        bf16x8 msrc[SHB];
        pack_rows<MB>(mu, msrc);
#pragma unroll
        for (int t = 0; t < SHB; ++t) gacc = mfma(sGT[((k - 1) * SHB + t) * 64 + lane], msrc[t], gacc);
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int t = 0; t < SHB; ++t) acc = mfma(sAT[(((k - 2) * MB + mb) * SHB + t) * 64 + lane], msrc[t], acc);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            if constexpr (k - 1 >= 2) {
              mu[mb][v] = acc[v] * sK[k - 3][mb][v];
              gm[k - 3][mb][v] = acc[v] * tK[k - 3][mb][v];
              if constexpr (L == 3) lam2[mb][v] = acc[v];
            } else {
              mu[mb][v] = acc[v] * s1[mb][v];
              g1[mb][v] = acc[v] * t1[mb][v];
            }
          }
        }
      });
      bf16x8 msrc[SHB];
      pack_rows<MB>(mu, msrc);
#pragma unroll
      for (int t = 0; t < SHB; ++t) gacc = mfma(sGT[t * 64 + lane], msrc[t], gacc);
    }
    // result row 4g + v is input m
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int m = 4 * g + v;
      if (m < P && valid) out[(int64_t)(1 + m) * ns + qp] = (double)gacc[v] + sdb[m];
    }
    if constexpr (!HESS) return;

    // ---- layer-1 Gram: rows are packed input pairs
    f4 hacc[NPB];
    {
      bf16x8 gsrc[SHB];
      pack_rows<MB>(g1, gsrc);
#pragma unroll
      for (int pb = 0; pb < NPB; ++pb) {
        hacc[pb] = (f4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < SHB; ++t) hacc[pb] = mfma(sG1[(pb * SHB + t) * 64 + lane], gsrc[t], hacc[pb]);
      }
    }

    // layer-2 Gram weights gamma_2 / s_2 (three hidden layers)
    float w2[L == 3 ? MB : 1][4];
    if constexpr (L == 3) {
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int v = 0; v < 4; ++v) w2[mb][v] = lam2[mb][v] * (1.0f - sK[0][mb][v]);
    }
    // ---- Jacobian forward of the later layers
    // four packed pairs (16 pb + v + 4 j) per cross-lane reduction, which
    // leaves pair 16 pb + 4 g + v in lane group g: the layout of hacc
    auto reduce_pairs = [&](const float (&pp)[P2]) {
      static_for<NPB * 4>([&](auto GI) {
        constexpr int pb = decltype(GI)::value / 4, v = decltype(GI)::value % 4;
        if constexpr (16 * pb + v < P2) {
          constexpr int h0 = 16 * pb + v;
          hacc[pb][v] += reduce4f(pp[h0], (h0 + 4 < P2) ? pp[h0 + 4 < P2 ? h0 + 4 : 0] : 0.f,
                                  (h0 + 8 < P2) ? pp[h0 + 8 < P2 ? h0 + 8 : 0] : 0.f,
                                  (h0 + 12 < P2) ? pp[h0 + 12 < P2 ? h0 + 12 : 0] : 0.f, g);
        }
      });
    };
    // per-lane pair partials sum_r x_rn y_rm over this lane's four rows
    auto add_pairs = [&](float (&pp)[P2], const bf16x2 (&x)[P][2], const bf16x2 (&y)[P][2]) {
      static_for<P2>([&](auto HI) {
        constexpr int h = decltype(HI)::value;
        constexpr int a = hess_m(h, P), b = hess_n(h, P);  // pair (a, b), a <= b
        pp[h] = dot2(x[a][1], y[b][1], dot2(x[a][0], y[b][0], pp[h]));
      });
    };
    if constexpr (L == 2) {
      // sources of the layer-2 Jacobian columns, s_1 (.) W1[:, m]; the
      // columns are formed one row block at a time
      bf16x8 src[P][SHB];
      static_for<P>([&](auto MI) {
        constexpr int m = decltype(MI)::value;
        float u[MB][4];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          const f4 wv = row4(sW1t + m * H, mb);
#pragma unroll
          for (int v = 0; v < 4; ++v) u[mb][v] = s1[mb][v] * wv[v];
        }
        pack_rows<MB>(u, src[m]);
      });
      float pp[P2];
#pragma unroll
      for (int i = 0; i < P2; ++i) pp[i] = 0.f;
      static_for<MB>([&](auto OB) {
        constexpr int ob = decltype(OB)::value;
        const bf16x8* aL = sA + ob * SHB * 64 + lane;
        bf16x2 jp[P][2], gJ[P][2];  // J_2[ob, m] and gamma_2 J_2[ob, m], packed
        static_for<P>([&](auto MI) {
          constexpr int m = decltype(MI)::value;
          f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int t = 0; t < SHB; ++t) acc = mfma(aL[t * 64], src[m][t], acc);
          const f4 bv = row4(sBt + m * H, ob);
          float J[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) J[v] = acc[v] + bv[v];
          jp[m][0] = pk_bf16(J[0], J[1]);
          jp[m][1] = pk_bf16(J[2], J[3]);
          gJ[m][0] = pk_bf16(gm[0][ob][0] * J[0], gm[0][ob][1] * J[1]);
          gJ[m][1] = pk_bf16(gm[0][ob][2] * J[2], gm[0][ob][3] * J[3]);
        });
        add_pairs(pp, gJ, jp);
      });
      reduce_pairs(pp);
    } else {
      // layer 2 whole: the layer-3 sources src3 = s_2 (.) J_2[:, m] and the
      // layer-2 Gram operands q2 = (gamma_2 / s_2) (.) J_2[:, m], so that
      // sum_r gamma_2 J_rn J_rm = sum_r q2_rn src3_rm (gamma_2 / s_2 =
      // lambda_2 (1 - s_2), no division)
      bf16x8 src3[P][SHB], q2[P][SHB];
      static_for<P>([&](auto MI) {
        constexpr int m = decltype(MI)::value;
        float u[MB][4];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          const f4 wv = row4(sW1t + m * H, mb);
#pragma unroll
          for (int v = 0; v < 4; ++v) u[mb][v] = s1[mb][v] * wv[v];
        }
        asm volatile("" ::: "memory");  // layer-2 fragments are re-read per column, not held
        bf16x8 s2src[SHB];
        pack_rows<MB>(u, s2src);
        float j2s[MB][4], j2q[MB][4];
#pragma unroll
        for (int ob = 0; ob < MB; ++ob) {
          f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int t = 0; t < SHB; ++t) acc = mfma(sA[(ob * SHB + t) * 64 + lane], s2src[t], acc);
          const f4 bv = row4(sBt + m * H, ob);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const float j = acc[v] + bv[v];
            j2s[ob][v] = sK[0][ob][v] * j;
            j2q[ob][v] = w2[ob][v] * j;
          }
        }
        pack_rows<MB>(j2s, src3[m]);
        pack_rows<MB>(j2q, q2[m]);
      });
      float pp[P2];
#pragma unroll
      for (int i = 0; i < P2; ++i) pp[i] = 0.f;
      // layer 3 one row block at a time; row block ob of the packed layer-2
      // operands is half (ob % 2) of K step ob / 2
      static_for<MB>([&](auto OB) {
        constexpr int ob = decltype(OB)::value, tt = ob / 2, hh = ob % 2;
        const bf16x8* aL = sA + (MB + ob) * SHB * 64 + lane;
        bf16x2 jp[P][2], gJ[P][2], xs[P][2], xq[P][2];
        static_for<P>([&](auto MI) {
          constexpr int m = decltype(MI)::value;
          f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int t = 0; t < SHB; ++t) acc = mfma(aL[t * 64], src3[m][t], acc);
          const f4 bv = row4(sBt + P * H + m * H, ob);
          float J[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) J[v] = acc[v] + bv[v];
          jp[m][0] = pk_bf16(J[0], J[1]);
          jp[m][1] = pk_bf16(J[2], J[3]);
          gJ[m][0] = pk_bf16(gm[1][ob][0] * J[0], gm[1][ob][1] * J[1]);
          gJ[m][1] = pk_bf16(gm[1][ob][2] * J[2], gm[1][ob][3] * J[3]);
          half_pairs(src3[m][tt], hh, xs[m][0], xs[m][1]);
          half_pairs(q2[m][tt], hh, xq[m][0], xq[m][1]);
        });
        add_pairs(pp, gJ, jp);
        add_pairs(pp, xq, xs);
      });
      reduce_pairs(pp);
    }
    // lane group g holds pair 16 pb + 4 g + v
#pragma unroll
    for (int pb = 0; pb < NPB; ++pb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int h = 16 * pb + 4 * g + v;
        if (h < P2 && valid) out[(int64_t)(1 + P + h) * ns + qp] = (double)hacc[pb][v];
      }
  };

  // persistent waves: each takes every (gridDim.x * WPB)-th tile, with the
  // next tile's inputs in flight while the current one is computed
  const int64_t stride = (int64_t)gridDim.x * WPB;
  double kn[S1];
  int64_t tile = (int64_t)blockIdx.x * WPB + w;
  if (tile < ntiles) load_k(tile, kn);
  for (; tile < ntiles; tile += stride) {
    asm volatile("" ::: "memory");  // no fragment read is hoisted out of the tile loop
    double kc[S1];
#pragma unroll
    for (int e = 0; e < S1; ++e) kc[e] = kn[e];
    if (tile + stride < ntiles) load_k(tile + stride, kn);
    tile_body(tile, kc);
  }
}

}  // namespace pa
