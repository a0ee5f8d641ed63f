// FP32 adjoint-form network kernel with the Hessian, one wave per 16-point
// tile and every neuron in that wave (two or three hidden layers; the library
// runs it for three, where it replaces the multi-wave kernel): the value
// forward, the reverse sweep and the input gradient as in k_mlp_s1w, the
// layer-1 Gram sum as a matrix product of the pair table W1_rm W1_rn with
// gamma_1, and the Jacobians of the later layers on the 16x16x4 FP32 matrix
// cores, with the Gram sum
//   d2N/dK dK = sum_k J_k^T diag(gamma_k) J_k,  gamma_k = lambda_k (.) F''(y_k),
// accumulated per lane over the lane's rows and reduced across the four lane
// groups once per tile.  With three hidden layers every column of J_2 stays
// in registers (the layer-3 sources s_2 (.) J_2[:, m] are formed from it per
// row block), so a tile needs no LDS exchange and no barrier; the fragment
// tables are staged once per workgroup.  Same outputs as Alg. 4 up to
// rounding; the network contractions in FP32, inputs and outputs FP64.
#pragma once
#include "mlp_bf16.h"
#include "mma_util.h"
#include "pa_internal.h"

namespace pa {

// Waves per SIMD the register budget is sized for: two for two hidden
// layers up to width 32, one for width 64 and for three layers (the columns
// of J_2 are live through layer 3).
template <int H, int L>
constexpr int f32w_waves() { return (L == 3 || H > 32) ? 1 : 2; }

template <int H, int L, int P>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(f32w_waves<H, L>())))
k_mlp_f32w(const unsigned char* __restrict__ prep, PrepLayout lay, int64_t n, const double* __restrict__ Kin,
           double* __restrict__ out) {
  static_assert(L == 2 || L == 3, "two or three hidden layers");
  static_assert(P <= 16, "the gradient rows are one 16-row block");
  using E = EngF32;
  using acc_t = E::acc;
  constexpr int MB = H / 16, SH = H / 4, S1 = (P + 3) / 4, P2 = P * (P + 1) / 2, NPB = (P2 + 15) / 16;
  constexpr int WPB = 4;  // waves (one tile each) per workgroup
  constexpr int NW1 = MB * S1 * 64, NA = MB * SH * 64, NB = MB * S1 * 64, NG = SH * 64, NG1 = NPB * MB * 4 * 64;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, q = lane & 15, g = lane >> 4;

  __shared__ float lW1[NW1], lA[L - 1][NA], lB[L - 1][NB], lAT[L - 1][NA], lG[L][NG], lG1[NG1];
  __shared__ __align__(16) float sW1t[P * H];            // [m][r] = W1[r][m]
  __shared__ __align__(16) float sBt[(L - 1) * P * H];   // [k-2][m][r] = B_k[r][m]
  __shared__ __align__(16) float cs[L * H], sa[H];
  __shared__ double bs[P];
  {
    const float* gW1 = (const float*)(prep + lay.y_W1);
    const float* gA = (const float*)(prep + lay.y_A) + NA;  // per-layer tables start at layer 1
    const float* gB = (const float*)(prep + lay.y_B) + NB;
    const float* gAT = (const float*)(prep + lay.y_ATp) + NA;
    const float* gG = (const float*)(prep + lay.y_GT);
    const float* gG1 = (const float*)(prep + lay.y_G1);
    for (int i = tid; i < NW1; i += 64 * WPB) lW1[i] = gW1[i];
    for (int i = tid; i < (L - 1) * NA; i += 64 * WPB) {
      (&lA[0][0])[i] = gA[i];
      (&lAT[0][0])[i] = gAT[i];
    }
    for (int i = tid; i < (L - 1) * NB; i += 64 * WPB) (&lB[0][0])[i] = gB[i];
    for (int i = tid; i < L * NG; i += 64 * WPB) (&lG[0][0])[i] = gG[i];
    for (int i = tid; i < NG1; i += 64 * WPB) lG1[i] = gG1[i];
    const float* fW1t = (const float*)(prep + lay.f_W1t);
    const float* fBt = (const float*)(prep + lay.f_Bt);
    const float* fc = (const float*)(prep + lay.f_c);
    const float* fa = (const float*)(prep + lay.f_a);
    for (int i = tid; i < P * H; i += 64 * WPB) sW1t[i] = fW1t[i];
    for (int i = tid; i < (L - 1) * P * H; i += 64 * WPB) sBt[i] = fBt[P * H + i];  // layer k >= 2 at k - 1
    for (int i = tid; i < L * H; i += 64 * WPB) cs[i] = fc[i];
    for (int i = tid; i < H; i += 64 * WPB) sa[i] = fa[i];
    for (int i = tid; i < P; i += 64 * WPB) bs[i] = ((const double*)(prep + lay.d_b))[i];
  }
  __syncthreads();  // the only barrier: every wave reaches it before any exits

  // rows 16 mb + 4 g .. + 3 of a length-H row vector (the accumulator rows of block mb)
  auto row4 = [&](const float* base, int mb) -> f4 { return *(const f4*)(base + 16 * mb + 4 * g); };
  const int64_t ntiles = (n + 15) / 16;
  auto load_k = [&](int64_t tile, double (&kv)[S1]) {
    int64_t qq = tile * 16 + q;
    asm volatile("" : "+v"(qq));  // one opaque index: no per-column address streams across tiles
#pragma unroll
    for (int s = 0; s < S1; ++s) {
      const int m = 4 * s + g;
      kv[s] = (qq < n && m < P) ? Kin[(int64_t)m * n + qq] : 0.0;
    }
  };

  auto tile_body = [&](int64_t tile, const double (&kin)[S1]) {
    int64_t qp = tile * 16 + q;
    // opaque per tile: the per-lane output addresses are formed at each store
    int64_t ns = n;
    asm volatile("" : "+v"(qp), "+s"(ns));
    const bool valid = qp < n;
    float kB[S1];
    double bK = 0.0;  // this lane's share of b . K, in FP64
#pragma unroll
    for (int s = 0; s < S1; ++s) {
      const int m = 4 * s + g;
      kB[s] = (float)kin[s];
      if (m < P) bK += bs[m] * kin[s];
    }
    // ---- value forward; F' and F'' of every layer kept
    float s1[MB][4], t1[MB][4], sK[L - 1][MB][4], tK[L - 1][MB][4];
    float val = 0.f;
    {
      float z[MB][4];
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        float a1[S1];
#pragma unroll
        for (int s = 0; s < S1; ++s) a1[s] = lW1[(mb * S1 + s) * 64 + lane];
        const f4 c = row4(cs, mb);
        acc_t acc = {c[0], c[1], c[2], c[3]};  // starts from the bias
        acc = mma_in<E, P>(a1, kB, acc);
#pragma unroll
        for (int v = 0; v < 4; ++v) softplus3(acc[v], z[mb][v], s1[mb][v], t1[mb][v]);
      }
      static_for<L - 1>([&](auto KI) {
        constexpr int k = decltype(KI)::value + 2;
        float zn[MB][4];
#pragma unroll
        for (int ob = 0; ob < MB; ++ob) {
          float AV[SH], BV[S1];
#pragma unroll
          for (int s = 0; s < SH; ++s) AV[s] = lA[k - 2][(ob * SH + s) * 64 + lane];
#pragma unroll
          for (int s = 0; s < S1; ++s) BV[s] = lB[k - 2][(ob * S1 + s) * 64 + lane];
          const f4 c = row4(cs + (k - 1) * H, ob);
          acc_t acc = {c[0], c[1], c[2], c[3]};
          acc = mma_in<E, P>(BV, kB, mma_src<E, MB>(AV, z, acc));
#pragma unroll
          for (int v = 0; v < 4; ++v) softplus3(acc[v], zn[ob][v], sK[k - 2][ob][v], tK[k - 2][ob][v]);
          if constexpr (k == L) {
            const f4 a = row4(sa, ob);
#pragma unroll
            for (int v = 0; v < 4; ++v) val = fmaf(a[v], zn[ob][v], val);
          }
        }
        if constexpr (k < L) {
#pragma unroll
          for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int v = 0; v < 4; ++v) z[mb][v] = zn[mb][v];
        }
      });
    }
    {
      const double v = (double)group_sum_f(val) + group_sum(bK);
      if (g == 0 && valid) out[qp] = v;
    }
    // ---- reverse sweep: mu_k = lambda_k F'(y_k), gamma_k = lambda_k F''(y_k);
    // the input gradient accumulates on the matrix cores (result rows = inputs)
    float gm[L][MB][4];  // gamma_k at k - 1
    acc_t gacc = zero_acc<E>();
    {
      float mu[MB][4];
#pragma unroll
      for (int ob = 0; ob < MB; ++ob) {
        const f4 a = row4(sa, ob);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          mu[ob][v] = a[v] * sK[L - 2][ob][v];
          gm[L - 1][ob][v] = a[v] * tK[L - 2][ob][v];
        }
      }
      static_for<L - 1>([&](auto KI) {
        constexpr int k = L - decltype(KI)::value;  // L .. 2: lambda_{k-1} = A_k^T mu_k
#pragma unroll
        for (int s = 0; s < SH; ++s) gacc = E::mma(lG[k - 1][s * 64 + lane], mu[s / 4][s % 4], gacc);
        float mn[MB][4];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          acc_t acc = zero_acc<E>();
#pragma unroll
          for (int s = 0; s < SH; ++s) acc = E::mma(lAT[k - 2][(mb * SH + s) * 64 + lane], mu[s / 4][s % 4], acc);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const float sp = (k - 1 >= 2) ? sK[(k - 1 >= 2) ? k - 3 : 0][mb][v] : s1[mb][v];
            const float tp = (k - 1 >= 2) ? tK[(k - 1 >= 2) ? k - 3 : 0][mb][v] : t1[mb][v];
            mn[mb][v] = acc[v] * sp;
            gm[k - 2][mb][v] = acc[v] * tp;
          }
        }
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int v = 0; v < 4; ++v) mu[mb][v] = mn[mb][v];
      });
#pragma unroll
      for (int s = 0; s < SH; ++s) gacc = E::mma(lG[0][s * 64 + lane], mu[s / 4][s % 4], gacc);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int c = 4 * g + v;
      if (c < P && valid) out[(int64_t)(1 + c) * ns + qp] = (double)gacc[v] + bs[c];
    }

    // ---- layer-1 Gram: result rows are packed input pairs (pair 16 pb + 4 g + v)
    acc_t hacc[NPB];
#pragma unroll
    for (int pb = 0; pb < NPB; ++pb) {
      hacc[pb] = zero_acc<E>();
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int v = 0; v < 4; ++v) hacc[pb] = E::mma(lG1[((pb * MB + mb) * 4 + v) * 64 + lane], gm[0][mb][v], hacc[pb]);
    }
    // per-lane pair partials over this lane's rows, reduced once per tile
    float pp[P2];
#pragma unroll
    for (int i = 0; i < P2; ++i) pp[i] = 0.f;
    // pp[(a, b)] += sum_v x[a][v] y[b][v] over the packed pairs a <= b
    auto add_pairs = [&](const float (&x)[P][4], const float (&y)[P][4]) {
      static_for<P2>([&](auto HI) {
        constexpr int h = decltype(HI)::value;
        constexpr int a = hess_m(h, P), b = hess_n(h, P);
        float s = pp[h];
#pragma unroll
        for (int v = 0; v < 4; ++v) s = fmaf(x[a][v], y[b][v], s);
        pp[h] = s;
      });
    };
    // column m of J_k for row block ob: A_k src (src over all rows) + B_k[:, m]
    // (the skip column is added after the products, so its LDS read overlaps
    // them instead of holding up the first one)
    auto jac_block = [&](int kk, int ob, int m, const float (&src)[MB][4]) -> acc_t {
      const float* aL = &lA[kk - 2][ob * SH * 64 + lane];
      acc_t acc = zero_acc<E>();
#pragma unroll
      for (int s = 0; s < SH; ++s) acc = E::mma(aL[s * 64], src[s / 4][s % 4], acc);
      const f4 bv = row4(sBt + ((kk - 2) * P + m) * H, ob);
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[v] += bv[v];
      return acc;
    };
    // sources of the layer-2 Jacobian columns: s_1 (.) W1[:, m]
    auto src2 = [&](int m, float (&u)[MB][4]) {
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        const f4 wv = row4(sW1t + m * H, mb);
#pragma unroll
        for (int v = 0; v < 4; ++v) u[mb][v] = s1[mb][v] * wv[v];
      }
    };
    if constexpr (L == 2) {
#pragma unroll 1
      for (int ob = 0; ob < MB; ++ob) {
        asm volatile("" ::: "memory");  // the fragments are read per row block, not held
        float J[P][4], gJ[P][4];
        float g2[4];  // gamma_2 of row block ob, selected without indexing registers at run time
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          g2[v] = gm[1][0][v];
#pragma unroll
          for (int b = 1; b < MB; ++b) g2[v] = (ob == b) ? gm[1][b][v] : g2[v];
        }
        static_for<P>([&](auto MI) {
          constexpr int m = decltype(MI)::value;
          float u[MB][4];
          src2(m, u);
          const acc_t acc = jac_block(2, ob, m, u);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            J[m][v] = acc[v];
            gJ[m][v] = g2[v] * acc[v];
          }
        });
        add_pairs(gJ, J);
      }
    } else {
      // every column of J_2, all rows
      float J2[P][MB][4];
      static_for<P>([&](auto MI) {
        constexpr int m = decltype(MI)::value;
        float u[MB][4];
        src2(m, u);
        asm volatile("" ::: "memory");  // layer-2 fragments are re-read per column, not held
#pragma unroll
        for (int ob = 0; ob < MB; ++ob) {
          const acc_t acc = jac_block(2, ob, m, u);
#pragma unroll
          for (int v = 0; v < 4; ++v) J2[m][ob][v] = acc[v];
        }
      });
      // layer-2 Gram and layer 3, one row block at a time
      static_for<MB>([&](auto OB) {
        constexpr int ob = decltype(OB)::value;
        {
          float x[P][4], y[P][4];
#pragma unroll
          for (int m = 0; m < P; ++m)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              y[m][v] = J2[m][ob][v];
              x[m][v] = gm[1][ob][v] * J2[m][ob][v];
            }
          add_pairs(x, y);
        }
        float J[P][4], gJ[P][4];
        static_for<P>([&](auto MI) {
          constexpr int m = decltype(MI)::value;
          float u[MB][4];  // layer-3 sources s_2 (.) J_2[:, m]
#pragma unroll
          for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int v = 0; v < 4; ++v) u[mb][v] = sK[0][mb][v] * J2[m][mb][v];
          const acc_t acc = jac_block(3, ob, m, u);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            J[m][v] = acc[v];
            gJ[m][v] = gm[2][ob][v] * acc[v];
          }
        });
        add_pairs(gJ, J);
      });
    }
    // four pairs (h0 + 4 j) per cross-lane reduction leave pair 16 pb + 4 g + v
    // in lane group g: the layout of hacc
    static_for<NPB * 4>([&](auto GI) {
      constexpr int pb = decltype(GI)::value / 4, v = decltype(GI)::value % 4;
      if constexpr (16 * pb + v < P2) {
        constexpr int h0 = 16 * pb + v;
        hacc[pb][v] += reduce4f(pp[h0], (h0 + 4 < P2) ? pp[h0 + 4 < P2 ? h0 + 4 : 0] : 0.f,
                                (h0 + 8 < P2) ? pp[h0 + 8 < P2 ? h0 + 8 : 0] : 0.f,
                                (h0 + 12 < P2) ? pp[h0 + 12 < P2 ? h0 + 12 : 0] : 0.f, g);
      }
    });
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
    for (int s = 0; s < S1; ++s) kc[s] = kn[s];
    if (tile + stride < ntiles) load_k(tile + stride, kn);
    tile_body(tile, kc);
  }
}

}  // namespace pa
