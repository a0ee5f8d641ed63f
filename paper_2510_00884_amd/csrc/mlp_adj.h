// Adjoint-form network kernels (value forward, value adjoint, Jacobian
// forward; same outputs as Alg. 4) and their launchers.  Included by the
// per-width translation units mlp_adj_h*.hip.
#pragma once
#include <type_traits>
#include <utility>

#include "mlp_bf16.h"
#include "mlp_f32w.h"
#include "mma_util.h"
#include "pa_internal.h"

namespace pa {

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
  // Jacobian columns per LDS exchange (two barriers each): all of them for
  // the FP64 3 x 64 network, where one workgroup fills a CU anyway; three
  // otherwise
  constexpr int CH = (L >= 3) ? ((L == 3 && H >= 64 && PR == PREC_F64) ? P : 3) : 1;
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
  // PREC_BF16J: the Jacobian pass of layers >= 2 runs on the BF16 matrix
  // cores (these fragments, K permuted to the FP32 accumulator layout);
  // value, reverse sweep, gradient and the layer-1 Gram stay FP32
  constexpr bool JB = PR == PREC_BF16J;
  constexpr int SHB = (H + 31) / 32;
  bf16x8 AZ[JB ? L - 1 : 1][JB ? SHB : 1];
  if constexpr (JB && HESS) {
    const bf16x8* zA = frag_ptr<EngBF16>(prep, lay, 1);
#pragma unroll
    for (int k = 2; k <= L; ++k)
#pragma unroll
      for (int s = 0; s < SHB; ++s) AZ[k - 2][s] = zA[(((k - 1) * MB + w) * SHB + s) * 64 + lane];
  }
  // this wave's layer-1 Gram and reverse-product fragments, the same for
  // every tile, held in registers where the budget allows (no L2 latency in
  // the tile loop)
  constexpr bool HAT = (L - 1) * SH <= 32;
  frag_t g1f[HESS ? NPB : 1][4], atf[HAT ? L - 1 : 1][HAT ? SH : 1];
  if constexpr (HESS) {
#pragma unroll
    for (int pb = 0; pb < NPB; ++pb)
#pragma unroll
      for (int s = 0; s < 4; ++s) g1f[pb][s] = fG1[((pb * MB + w) * 4 + s) * 64 + lane];
  }
  if constexpr (HAT) {
#pragma unroll
    for (int k = 2; k <= L; ++k)
#pragma unroll
      for (int s = 0; s < SH; ++s) atf[k - 2][s] = fAT[(((k - 1) * MB + w) * SH + s) * 64 + lane];
  }
  auto jac_product = [&](int kk, const T (&src)[MB][4]) -> acc_t {
    if constexpr (JB)
      return mma_src<EngBF16, MB>(AZ[kk], src, zero_acc<EngBF16>());
    else
      return mma_src<E, MB>(AV[kk], src, zero_acc<E>());
  };
  for (int i = tid; i < L * H; i += 64 * NW) (&cs[0][0])[i] = t_c[i];
  for (int i = tid; i < H; i += 64 * NW) as_[i] = t_a[i];
  __shared__ SpTab sp[1];
  __shared__ double bs[P];
  for (int i = tid; i < P; i += 64 * NW) bs[i] = d_b[i];
  if constexpr (std::is_same<T, double>::value) softplus_tab_fill(sp[0], tid, 64 * NW);
  __syncthreads();  // W1s, Bs, cs, as_, bs, sp

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
    const int64_t base = tile * 16;
    const int64_t qp = base + q;
    const bool valid = qp < n;
    frag_t kB[S1];
    double bK = 0.0;  // this lane's share of b . K, in FP64 (added by wave 0)
#pragma unroll
    for (int s = 0; s < S1; ++s) {
      const int m = 4 * s + g;
      kB[s] = (T)kin[s];
      if (m < P) bK += bs[m] * kin[s];
    }
    // layer 1: own rows, then z_1 and F'(y_1) of every row through LDS
    T t1w[4], s1w[4], z1[MB][4];
    {
      acc_t acc = mma_in<E, P>(a1, kB, zero_acc<E>());
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        T f, f1, f2;
        const int r = 16 * w + E::row(g, v);
        softplus3((T)(acc[v] + cs[0][r]), f, f1, f2, sp[0]);
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
          softplus3((T)(acc[v] + cs[k - 1][16 * w + E::row(g, v)]), f, f1, f2, sp[0]);
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
          if (w == 0) pl += group_sum(bK);
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
      for (int s = 0; s < SH; ++s) {
        frag_t a;
        if constexpr (HAT) a = atf[k - 2][s];
        else a = at[s * 64];
        acc = E::mma(a, (frag_t)xbuf[0][4 * s + g][q], acc);
      }
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
        for (int s = 0; s < 4; ++s) acc = E::mma(g1f[pb][s], (frag_t)gam[0][s], acc);
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
      // every four pairs into outp at the packed positions of those pairs;
      // gJm = gamma_k (.) J[:, m] of the column m just formed
      auto pair_sum = [&](auto TI, const T (&gJm)[4]) {
        constexpr int t = decltype(TI)::value;
        constexpr int nn = colmaj_n(t);
        T x = (T)0;
#pragma unroll
        for (int v = 0; v < 4; ++v) x += J[nn][v] * gJm[v];
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
            T gJm[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) gJm[v] = gam[1][v] * J[m][v];
            static_for<m + 1>([&](auto NI) {
              pair_sum(std::integral_constant<int, m * (m + 1) / 2 + decltype(NI)::value>{}, gJm);
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
              if constexpr (m < P) {
                T gJm[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) gJm[v] = gam[k - 1][v] * J[m][v];
                static_for<m + 1>([&](auto NI) {
                  pair_sum(std::integral_constant<int, m * (m + 1) / 2 + decltype(NI)::value>{}, gJm);
                });
              }
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
      if (c >= 1 && c <= P) v += bs[c - 1];
      out[(int64_t)c * n + pt] = v;
    }
    __syncthreads();  // outp, l1buf and xbuf free for the next tile
  };
  if constexpr (!PERSIST) {
    double kc[S1];  // one tile per workgroup (see the launcher)
    load_k(blockIdx.x, kc);
    tile_body(blockIdx.x, kc);
  } else {
    // block-uniform tile loop: every wave of a workgroup runs the same
    // tiles, so the barriers inside tile_body match; the next tile's inputs
    // are in flight while the current one is computed
    double kn[S1];
    int64_t tile = blockIdx.x;
    if (tile < ntiles) load_k(tile, kn);
    for (; tile < ntiles; tile += gridDim.x) {
      // with the Hessian, nothing read in the tile body stays live across tiles
      if constexpr (HESS) asm volatile("" ::: "memory");
      double kc[S1];
#pragma unroll
      for (int s = 0; s < S1; ++s) kc[s] = kn[s];
      if (tile + gridDim.x < ntiles) load_k(tile + gridDim.x, kn);
      tile_body(tile, kc);
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
__global__ void __launch_bounds__(PR == PREC_F64 ? 512 : 256) __attribute__((amdgpu_waves_per_eu(2)))
k_mlp_adj2(const unsigned char* __restrict__ prep, PrepLayout lay, int64_t n,
           const double* __restrict__ Kin, double* __restrict__ out) {
  using E = typename std::conditional<PR == PREC_F64, EngF64, EngF32>::type;
  using T = typename E::T;
  using acc_t = typename E::acc;
  using frag_t = typename E::frag;
  constexpr int MB = H / 16, P2 = P * (P + 1) / 2;
  constexpr int SH = H / 4, S1 = (P + 3) / 4, NPB = (P2 + 15) / 16;
  // FP64: the layer-2 and layer-1 matrix-core fragments are staged once per
  // workgroup of eight waves, one tile each (LDS latency instead of L2
  // latency on every tile), with the softplus tables and, for the Hessian,
  // the layer-2 Jacobian column tables A_2 diag(W1[:, m]): a column is then
  // the product of a constant table with F'(y_1), already in registers in
  // K-step order.  FP32 reads the fragments from the prepared tables, four
  // waves per workgroup, which leaves LDS for more resident waves.
  constexpr bool LT = PR == PREC_F64;
  constexpr bool AW = LT && HESS;
  constexpr int WPB = LT ? 8 : 4;  // waves, one tile each, per workgroup
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, q = lane & 15, g = lane >> 4;
  const uint32_t g8 = 8u * (uint32_t)g;

  __shared__ T W1s[P][H], B2s[P][H], c1s[H], c2s[H], as_[H];
  __shared__ double db_s[P];
  __shared__ double hb[HESS ? WPB : 1][HESS ? P2 : 1][16];
  __shared__ SpTab sp[1];
  constexpr int NW1 = MB * S1 * 64, NA2 = MB * SH * 64, NG1 = HESS ? NPB * MB * 4 * 64 : 1;
  __shared__ frag_t lW1[LT ? NW1 : 1], lA[LT ? NA2 : 1], lB[LT ? NW1 : 1], lATp[LT ? NA2 : 1], lG1[LT ? NG1 : 1];
  __shared__ frag_t lAW[AW ? P * NA2 : 1];

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
      softplus_tab_fill(sp[0], tid, 64 * WPB);
    }
    if constexpr (AW) {
      const frag_t* gAW = (const frag_t*)(prep + lay.x_AW);
      for (int i = tid; i < P * NA2; i += 64 * WPB) lAW[i] = gAW[i];
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
    acc_t acc;  // starts from the bias
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = c1s[16 * mb + E::row(g, v)];
    acc = mma_in<E, P>(a1, kB, acc);
#pragma unroll
    for (int v = 0; v < 4; ++v) softplus3((T)acc[v], z1[mb][v], s1[mb][v], t1[mb][v], sp[0]);
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
    acc_t acc;  // starts from the bias
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = c2s[16 * ob + E::row(g, v)];
    acc = mma_in<E, P>(BV, kB, mma_src<E, MB>(AV, z1, acc));
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * ob + E::row(g, v);
      T f, f1, f2;
      softplus3((T)acc[v], f, f1, f2, sp[0]);
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
      // PREC_BF16J: the layer-2 Jacobian contracts over the neurons on the
      // BF16 matrix cores (16x16x32, FP32 accumulation; the K dimension of
      // the prepared BF16 fragments is permuted to the FP32 accumulator
      // layout, so the column sources pack without shuffles); everything
      // else in this kernel is FP32
      constexpr bool JB = PR == PREC_BF16J;
      constexpr int SHB = (H + 31) / 32;
      frag_t AV[(JB || AW) ? 1 : SH];
      bf16x8 AZ[JB ? SHB : 1];
      if constexpr (JB) {
        const bf16x8* zA = frag_ptr<EngBF16>(prep, lay, 1);
#pragma unroll
        for (int s = 0; s < SHB; ++s) AZ[s] = zA[((1 * MB + ob) * SHB + s) * 64 + lane];
      } else if constexpr (!AW) {
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
        acc_t acc;  // starts from the skip column B_2[:, m]
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] = B2s[m][16 * ob + E::row(g, v)];
        if constexpr (AW) {
          // column m = (A_2 diag(W1[:, m])) F'(y_1) + B_2[:, m]
          const frag_t* aw = lAW + (m * MB + ob) * SH * 64 + lane;
#pragma unroll
          for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc = E::mma(aw[(mb * 4 + v) * 64], (frag_t)s1[mb][v], acc);
        } else {
          T src[MB][4];
#pragma unroll
          for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int v = 0; v < 4; ++v) src[mb][v] = s1[mb][v] * W1s[m][16 * mb + E::row(g, v) + zr];
          if constexpr (JB)
            acc = mma_src<EngBF16, MB>(AZ, src, acc);
          else
            acc = mma_src<E, MB>(AV, src, acc);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          Jc[v] = (T)acc[v];
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


// ---------------------------------------------------------------- value and gradient, one wave per tile
// Stress-only form (no Hessian) for any depth: one wave owns a 16-point tile
// and every neuron, so the layers chain register to register (K steps in
// accumulator-row order, as in k_mlp_adj2).  The reverse sweep runs on the
// matrix cores twice over: lambda_{k-1} = A_k^T mu_k with the row-ordered
// transposed weights, and the gradient b + W1^T mu_1 + sum_k B_k^T mu_k as
// one accumulation whose result rows are the inputs (no cross-lane sums).
// Every fragment table is staged once per workgroup of eight persistent
// waves.  The LDS need (s1w_lds_bytes) decides where the launcher may use it.
template <int H, int L, int P, int PR>
__host__ __device__ constexpr int64_t s1w_lds_bytes() {
  constexpr int64_t es = PR == PREC_F64 ? 8 : 4;
  constexpr int64_t MB = H / 16, SH = H / 4, S1 = (P + 3) / 4;
  return es * 64 * (MB * S1 + (L - 1) * MB * (2 * SH + S1) + L * SH) + es * (L + 1) * H + 8 * P +
         (PR == PREC_F64 ? (int64_t)sizeof(SpTab) : 0);
}

template <int H, int L, int P, int PR>
__global__ void __launch_bounds__(512) k_mlp_s1w(const unsigned char* __restrict__ prep, PrepLayout lay, int64_t n,
                                                 const double* __restrict__ Kin, double* __restrict__ out) {
  using E = typename std::conditional<PR == PREC_F64, EngF64, EngF32>::type;
  using T = typename E::T;
  using acc_t = typename E::acc;
  using frag_t = typename E::frag;
  constexpr int MB = H / 16, SH = H / 4, S1 = (P + 3) / 4, WPB = 8;
  constexpr int NW1 = MB * S1 * 64, NA = MB * SH * 64, NB = MB * S1 * 64, NG = SH * 64;
  static_assert(P <= 16, "the gradient rows are one 16-row block");
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, q = lane & 15, g = lane >> 4;
  constexpr bool dbl = PR == PREC_F64;

  __shared__ frag_t lW1[NW1], lA[L - 1][NA], lB[L - 1][NB], lAT[L - 1][NA], lG[L][NG];
  __shared__ T cs[L][H], as_[H];
  __shared__ double bs[P];
  __shared__ SpTab sp[dbl ? 1 : 1];
  {
    const frag_t* gW1 = frag_ptr<E>(prep, lay, 0);
    const frag_t* gA = frag_ptr<E>(prep, lay, 1);
    const frag_t* gB = frag_ptr<E>(prep, lay, 2);
    const frag_t* gAT = (const frag_t*)(prep + (dbl ? lay.x_ATp : lay.y_ATp));
    const frag_t* gG = (const frag_t*)(prep + (dbl ? lay.x_GT : lay.y_GT));
    for (int i = tid; i < NW1; i += 64 * WPB) lW1[i] = gW1[i];
    // layer k >= 2 sits at index k - 1 of the per-layer tables
    for (int i = tid; i < (L - 1) * NA; i += 64 * WPB) {
      (&lA[0][0])[i] = gA[NA + i];
      (&lAT[0][0])[i] = gAT[NA + i];
    }
    for (int i = tid; i < (L - 1) * NB; i += 64 * WPB) (&lB[0][0])[i] = gB[NB + i];
    for (int i = tid; i < L * NG; i += 64 * WPB) (&lG[0][0])[i] = gG[i];
    const T* t_c = (const T*)(prep + (dbl ? lay.d_c : lay.f_c));
    const T* t_a = (const T*)(prep + (dbl ? lay.d_a : lay.f_a));
    for (int i = tid; i < L * H; i += 64 * WPB) (&cs[0][0])[i] = t_c[i];
    for (int i = tid; i < H; i += 64 * WPB) as_[i] = t_a[i];
    for (int i = tid; i < P; i += 64 * WPB) bs[i] = ((const double*)(prep + lay.d_b))[i];
    if constexpr (dbl) softplus_tab_fill(sp[0], tid, 64 * WPB);
  }
  __syncthreads();  // the only barrier: every wave reaches it before any exits

  const int64_t ntiles = (n + 15) / 16;
  auto load_k = [&](int64_t tile, double (&kv)[S1]) {
    const int64_t qq = tile * 16 + q;
#pragma unroll
    for (int s = 0; s < S1; ++s) {
      const int m = 4 * s + g;
      kv[s] = (qq < n && m < P) ? Kin[(int64_t)m * n + qq] : 0.0;
    }
  };
  auto tile_body = [&](int64_t tile, const double (&kin)[S1]) {
    const int64_t qp = tile * 16 + q;
    const bool valid = qp < n;
    frag_t kB[S1];
    double bK = 0.0;  // this lane's share of b . K, in FP64
#pragma unroll
    for (int s = 0; s < S1; ++s) {
      const int m = 4 * s + g;
      kB[s] = (T)kin[s];
      if (m < P) bK += bs[m] * kin[s];
    }
    // ---- value forward; F'(y_k) of every layer kept
    T z[MB][4], sk[L][MB][4];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      frag_t a1[S1];
#pragma unroll
      for (int s = 0; s < S1; ++s) a1[s] = lW1[(mb * S1 + s) * 64 + lane];
      acc_t acc;  // starts from the bias
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[v] = cs[0][16 * mb + E::row(g, v)];
      acc = mma_in<E, P>(a1, kB, acc);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        T f2;
        softplus3((T)acc[v], z[mb][v], sk[0][mb][v], f2, sp[0]);
      }
    }
    double val = 0.0;
    static_for<L - 1>([&](auto KI) {
      constexpr int k = decltype(KI)::value + 2;
      T zn[MB][4];
#pragma unroll
      for (int ob = 0; ob < MB; ++ob) {
        frag_t AV[SH], BV[S1];
#pragma unroll
        for (int s = 0; s < SH; ++s) AV[s] = lA[k - 2][(ob * SH + s) * 64 + lane];
#pragma unroll
        for (int s = 0; s < S1; ++s) BV[s] = lB[k - 2][(ob * S1 + s) * 64 + lane];
        acc_t acc;
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] = cs[k - 1][16 * ob + E::row(g, v)];
        acc = mma_in<E, P>(BV, kB, mma_src<E, MB>(AV, z, acc));
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          T f2;
          softplus3((T)acc[v], zn[ob][v], sk[k - 1][ob][v], f2, sp[0]);
          if constexpr (k == L) val += (double)(as_[16 * ob + E::row(g, v)] * zn[ob][v]);
        }
      }
      if constexpr (k < L) {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int v = 0; v < 4; ++v) z[mb][v] = zn[mb][v];
      }
    });
    val = group_sum(val) + group_sum(bK);
    if (g == 0 && valid) out[qp] = val;
    // ---- reverse: mu_L = a F'(y_L); gradient rows accumulate on the matrix cores
    T mu[MB][4];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int v = 0; v < 4; ++v) mu[mb][v] = as_[16 * mb + E::row(g, v)] * sk[L - 1][mb][v];
    acc_t gacc = zero_acc<E>();
    static_for<L>([&](auto KI) {
      constexpr int k = L - decltype(KI)::value;  // L, L-1, ..., 1
#pragma unroll
      for (int s = 0; s < SH; ++s) gacc = E::mma(lG[k - 1][s * 64 + lane], (frag_t)mu[s / 4][s % 4], gacc);
      if constexpr (k >= 2) {
        T mn[MB][4];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          acc_t acc = zero_acc<E>();
#pragma unroll
          for (int s = 0; s < SH; ++s) acc = E::mma(lAT[k - 2][(mb * SH + s) * 64 + lane], (frag_t)mu[s / 4][s % 4], acc);
#pragma unroll
          for (int v = 0; v < 4; ++v) mn[mb][v] = (T)acc[v] * sk[k - 2][mb][v];
        }
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int v = 0; v < 4; ++v) mu[mb][v] = mn[mb][v];
      }
    });
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int c = E::row(g, v);
      if (c < P && valid) out[(int64_t)(1 + c) * n + qp] = (double)gacc[v] + bs[c];
    }
  };
  // persistent waves: each takes every (gridDim.x * WPB)-th tile, the next
  // tile's inputs in flight while the current one is computed
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
  constexpr int WPB = PR == PREC_F64 ? 8 : 4, block = 64 * WPB;
  const int64_t nblk = ((n + 15) / 16 + WPB - 1) / WPB;
  const unsigned grid = PR == PREC_F64 ? persistent_grid(k_mlp_adj2<H, P, PR, HESS>, block, nblk) : (unsigned)nblk;
  k_mlp_adj2<H, P, PR, HESS><<<grid, block, 0, s>>>(prep, lay, n, K, out);
}

template <int H, int L, int P, int PR>
static void launch_s1w_one(const PrepLayout& lay, const unsigned char* prep, int64_t n, const double* K, double* out,
                           hipStream_t s) {
  const int64_t nblk = ((n + 15) / 16 + 7) / 8;
  k_mlp_s1w<H, L, P, PR><<<persistent_grid(k_mlp_s1w<H, L, P, PR>, 512, nblk), 512, 0, s>>>(prep, lay, n, K, out);
}

template <int H, int L, int P>
static void launch_f32w_one(const PrepLayout& lay, const unsigned char* prep, int64_t n, const double* K,
                            double* out, hipStream_t s) {
  const int64_t nblk = ((n + 15) / 16 + 3) / 4;
  k_mlp_f32w<H, L, P><<<persistent_grid(k_mlp_f32w<H, L, P>, 256, nblk), 256, 0, s>>>(prep, lay, n, K, out);
}

template <int H, int L, int P, bool HESS>
static void launch_bf16_one(const PrepLayout& lay, const unsigned char* prep, int64_t n, const double* K,
                            double* out, hipStream_t s) {
  const int64_t nblk = ((n + 15) / 16 + 3) / 4;
  k_mlp_bf16<H, L, P, HESS><<<persistent_grid(k_mlp_bf16<H, L, P, HESS>, 256, nblk), 256, 0, s>>>(prep, lay, n, K,
                                                                                                   out);
}

template <int H, int L, int P>
static int launch_mlp_adj_t(const PrepLayout& lay, int prec, const unsigned char* prep, int64_t n,
                            const double* K, double* out, int hess, hipStream_t s) {
  // all-BF16 (two and three hidden layers); PREC_BF16C is this pass
  // followed by the FP32 value-and-gradient pass, launched by the caller
  if (prec == PREC_BF16) {
    if constexpr (L <= 3) {
      if (hess) launch_bf16_one<H, L, P, true>(lay, prep, n, K, out, s);
      else launch_bf16_one<H, L, P, false>(lay, prep, n, K, out, s);
      return 0;
    } else {
      return -2;
    }
  }
  // value and gradient only: one wave per tile with LDS-staged tables where
  // they fit (FP64 three-layer width-64 networks keep the multi-wave kernel)
  if (!hess && (prec == PREC_F32 || prec == PREC_BF16J)) {
    launch_s1w_one<H, L, P, PREC_F32>(lay, prep, n, K, out, s);
    return 0;
  }
  // FP32 with the Hessian, three hidden layers: one wave per tile (with two
  // layers the two-layer kernel below, several waves per SIMD, is faster)
  if constexpr (L == 3) {
    if (hess && prec == PREC_F32) {
      launch_f32w_one<H, L, P>(lay, prep, n, K, out, s);
      return 0;
    }
  }
  if constexpr (s1w_lds_bytes<H, L, P, PREC_F64>() <= 160 * 1024) {
    if (!hess && prec == PREC_F64) {
      launch_s1w_one<H, L, P, PREC_F64>(lay, prep, n, K, out, s);
      return 0;
    }
  }
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
      case PREC_BF16J:  // FP32 value and gradient, layer-2 Jacobian in BF16
        if (hess) launch_adj2_one<H, P, PREC_BF16J, true>(lay, prep, n, K, out, s);
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
    case PREC_BF16J:  // FP32 value and gradient, Jacobian pass in BF16
      if (hess) launch_adj_one<H, L, P, PREC_BF16J, true>(lay, prep, n, K, out, s);
      else launch_adj_one<H, L, P, PREC_F32, false>(lay, prep, n, K, out, s);
      break;
    default: return -2;
  }
  return 0;
}


}  // namespace pa
