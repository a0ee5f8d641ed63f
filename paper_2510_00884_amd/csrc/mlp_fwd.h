// Forward-mode network kernel (Alg. 4 of App. B.2) on the matrix cores;
// the layout is described at the top of mlp.hip.  Included by the
// per-width translation units mlp_fwd_h*.hip.
#pragma once
#include <type_traits>
#include <utility>

#include "mma_util.h"
#include "pa_internal.h"

namespace pa {

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

  // ---- layer 1: y1 = W1 K + c1.  With three or more hidden layers each
  // wave evaluates its own rows and the values, F' and F'' of every row come
  // back through the exchange buffer (free until the value column); with two,
  // each wave evaluates all rows (the buffer holds one column)
  T s1[MB][4], t1[MB][4], z1[MB][4];
  if constexpr (CH >= 3) {
    const typename EV::frag* fW1 = frag_ptr<EV>(prep, lay, 0);
    typename EV::frag a1[S1V];
#pragma unroll
    for (int s = 0; s < S1V; ++s) a1[s] = fW1[(w * S1V + s) * 64 + lane];
    typename EV::acc acc = mma_in<EV, P>(a1, kB, zero_acc<EV>());
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * w + EV::row(g, v);
      T f, f1, f2;
      softplus3((T)(acc[v] + t_c[r]), f, f1, f2);
      xbuf[0][r][q] = f;
      xbuf[1][r][q] = f1;
      xbuf[2][r][q] = f2;
    }
    __syncthreads();
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * mb + EV::row(g, v);
        z1[mb][v] = xbuf[0][r][q];
        s1[mb][v] = xbuf[1][r][q];
        t1[mb][v] = xbuf[2][r][q];
      }
    __syncthreads();  // xbuf free for the value column
  } else {
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
    default: return -2;  // PREC_BF16J: adjoint form only
  }
  return 0;
}

}  // namespace pa
