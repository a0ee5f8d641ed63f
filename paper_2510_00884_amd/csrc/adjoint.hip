// Parameter adjoint of the stress (stress calibration):
//   theta_bar = sum_q (dP_q/dtheta)^T P_bar_q,
//   P_q = sum_m dN/dK_m(K_q; theta) g_m(F_q),   g_m = dK_m/dF.
// With lambda_q,m = P_bar_q : g_m (a p-vector per point) this is
//   theta_bar = sum_q d/dtheta [ grad_K N(K_q; theta) . lambda_q ],
// i.e. reverse mode over the network evaluated together with its forward
// tangent along lambda_q (primal z and tangent zdot carried per layer).
// Nothing is stored between forward and backward: every tile of 16 points
// recomputes its activations.
//
// Layout as in the forward network kernel (points on the matrix-core N
// dimension, neurons split across h/16 waves).  The weight gradients are
// sums over points, i.e. products with K = points; the per-point adjoint rows
// are transposed through LDS into the A operand and the activations of the
// previous layer (kept in LDS) supply the B operand.  Workgroups are
// persistent over tiles; each writes one partial theta_bar and a second
// kernel sums the partials in a fixed order (deterministic).
#include <type_traits>
#include <utility>

#include "mma_util.h"
#include "pa_internal.h"

namespace pa {

// K (features) and lambda_m = P_bar : dK_m/dF = 2 (F^T P_bar) : dK_m/dC.
template <int NSV>
__global__ void __launch_bounds__(256) k_adj_inputs(int64_t n, const double* __restrict__ F,
                                                    const double* __restrict__ Pb, ModelConst mc,
                                                    double* __restrict__ K, double* __restrict__ Lam) {
  constexpr int P = Feat<NSV>::P;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  double f[9], pb[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    f[i] = F[i * n + t];
    pb[i] = Pb[i * n + t];
  }
  Kin k;
  kin_compute<NSV>(f, mc, k);
  double kf[P];
  kin_features<NSV>(k, mc, kf);
  // M = F^T P_bar; symmetric-slot weights (off-diagonal slots count twice)
  double Ms[6];
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    int I, J;
    slot_pair(a, I, J);
    double mij = 0.0, mji = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      mij += f[3 * i + I] * pb[3 * i + J];
      mji += f[3 * i + J] * pb[3 * i + I];
    }
    Ms[a] = (I == J) ? mij : mij + mji;
  }
#pragma unroll
  for (int m = 0; m < P; ++m) {
    double d[6];
    kin_dfeature<NSV>(k, mc, m, d);
    double l = 0.0;
#pragma unroll
    for (int a = 0; a < 6; ++a) l += Ms[a] * d[a];
    K[(int64_t)m * n + t] = kf[m];
    Lam[(int64_t)m * n + t] = 2.0 * l;
  }
}

template <int H, int L, int P, int PR>
__global__ void __launch_bounds__(64 * (H / 16)) __attribute__((amdgpu_waves_per_eu(PR == PREC_F32 ? 2 : 1)))
k_param_bwd(const unsigned char* __restrict__ prep, PrepLayout lay, ThetaLayout tl, int64_t n,
            const double* __restrict__ Kin, const double* __restrict__ Lam, double* __restrict__ part) {
  using E = typename std::conditional<PR == PREC_F64, EngF64, EngF32>::type;
  using T = typename E::T;
  using acc_t = typename E::acc;
  constexpr int MB = H / 16, NW = MB, SH = H / 4, S1 = (P + 3) / 4;
  static_assert(P <= 16, "inputs must fit one 16-column block");
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, q = lane & 15, g = lane >> 4;

  __shared__ T zs[L - 1][2][H][16];  // z_k, zdot_k (all rows), k = 1..L-1
  __shared__ T xr[2][H][16];         // reverse exchange: ydot_bar_k, y_bar_k (all rows)
  __shared__ T us[NW][2][16][16];    // per-wave A operand staging: own rows x points
  __shared__ T kl[2][16][16];        // K and lambda [m][point]

  const bool dbl = std::is_same<T, double>::value;
  const T* t_a = (const T*)(prep + (dbl ? lay.d_a : lay.f_a));
  const T* t_c = (const T*)(prep + (dbl ? lay.d_c : lay.f_c));
  const typename E::frag* fW1 = frag_ptr<E>(prep, lay, 0);
  const typename E::frag* fA = frag_ptr<E>(prep, lay, 1);
  const typename E::frag* fB = frag_ptr<E>(prep, lay, 2);
  const typename E::frag* fAT = (const typename E::frag*)(prep + (dbl ? lay.x_AT : lay.y_AT));

  // this wave's forward fragments in registers; the transposed ones and the
  // layer-1 fragments in LDS, shared by the workgroup (in FP64 registers
  // would spill; in FP32 the smaller register budget lets two workgroups
  // share a compute unit)
  constexpr bool ATL = PR == PREC_F32 || L * H <= 3 * 64;
  __shared__ typename E::frag lAT[ATL ? (L - 1) * MB * SH * 64 : 1];
  __shared__ typename E::frag lW1f[MB * S1 * 64];
  __shared__ T cb[L * H];  // hidden biases
  if constexpr (ATL)
    for (int i = tid; i < (L - 1) * MB * SH * 64; i += 64 * NW) lAT[i] = fAT[MB * SH * 64 + i];
  for (int i = tid; i < MB * S1 * 64; i += 64 * NW) lW1f[i] = fW1[i];
  for (int i = tid; i < L * H; i += 64 * NW) cb[i] = t_c[i];
  typename E::frag AV[L - 1][SH], BV[L - 1][S1], AT[ATL ? 1 : L - 1][ATL ? 1 : SH];
#pragma unroll
  for (int k = 2; k <= L; ++k) {
#pragma unroll
    for (int s = 0; s < SH; ++s) {
      AV[k - 2][s] = fA[(((k - 1) * MB + w) * SH + s) * 64 + lane];
      if constexpr (!ATL) AT[k - 2][s] = fAT[(((k - 1) * MB + w) * SH + s) * 64 + lane];
    }
#pragma unroll
    for (int s = 0; s < S1; ++s) BV[k - 2][s] = fB[(((k - 1) * MB + w) * S1 + s) * 64 + lane];
  }
  T a_own[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) a_own[v] = t_a[16 * w + E::row(g, v)];

  // persistent accumulators
  acc_t accA[L - 1][MB], accB[L - 1], accW1 = zero_acc<E>();
#pragma unroll
  for (int k = 0; k < L - 1; ++k) {
    accB[k] = zero_acc<E>();
#pragma unroll
    for (int nb = 0; nb < MB; ++nb) accA[k][nb] = zero_acc<E>();
  }
  T cacc[L][4], aacc[4], bacc[S1];
#pragma unroll
  for (int k = 0; k < L; ++k)
#pragma unroll
    for (int v = 0; v < 4; ++v) cacc[k][v] = (T)0;
#pragma unroll
  for (int v = 0; v < 4; ++v) aacc[v] = (T)0;
#pragma unroll
  for (int s = 0; s < S1; ++s) bacc[s] = (T)0;

  // A operand (own rows x points) from the per-wave staging area, and the
  // outer-product update acc += U_p (16 x 16 points) * V_p^T (16 points x 16 cols).
  auto ufrag = [&](int p, int s) -> typename E::frag { return (typename E::frag)us[w][p][lane & 15][4 * s + g]; };

  __shared__ SpTab sp[1];
  if constexpr (std::is_same<T, double>::value) softplus_tab_fill(sp[0], tid, 64 * NW);
  __syncthreads();  // lAT, cb, sp
  const int64_t ntiles = (n + 15) / 16;
  // this lane's inputs and cotangents of a tile (feature 4 s + g of point q),
  // the next tile's in flight while the current one is computed
  auto load_kl = [&](int64_t tile, double (&kv)[S1], double (&lv)[S1]) {
    const int64_t qq = tile * 16 + q;
#pragma unroll
    for (int s = 0; s < S1; ++s) {
      const int m = 4 * s + g;
      kv[s] = (qq < n && m < P) ? Kin[(int64_t)m * n + qq] : 0.0;
      lv[s] = (qq < n && m < P) ? Lam[(int64_t)m * n + qq] : 0.0;
    }
  };
  double kn[S1], ln[S1];
  if ((int64_t)blockIdx.x < ntiles) load_kl(blockIdx.x, kn, ln);
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t base = tile * 16;
    const int64_t qp = base + q;
    const bool valid = qp < n;
    typename E::frag kB[S1], lB[S1];
#pragma unroll
    for (int s = 0; s < S1; ++s) {
      kB[s] = (T)kn[s];
      lB[s] = (T)ln[s];
      bacc[s] += (T)lB[s];
    }
    if (tile + gridDim.x < ntiles) load_kl(tile + gridDim.x, kn, ln);
    if (w == 0) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        kl[0][4 * s + g][q] = s < S1 ? (T)kB[s < S1 ? s : 0] : (T)0;
        kl[1][4 * s + g][q] = s < S1 ? (T)lB[s < S1 ? s : 0] : (T)0;
      }
    }
    // ---------------- forward: layer 1, this wave's rows (primal and
    // tangent), into LDS for the next layer; the reverse sweep keeps F', F''
    // and the tangent pre-activation
    T s1w[4], t1w[4], yd1w[4];
    {
      typename E::frag a1[S1];
#pragma unroll
      for (int s = 0; s < S1; ++s) a1[s] = lW1f[(w * S1 + s) * 64 + lane];
      acc_t ay = mma_in<E, P>(a1, kB, zero_acc<E>());
      acc_t ad = mma_in<E, P>(a1, lB, zero_acc<E>());
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * w + E::row(g, v);
        T f, f1, f2;
        softplus3((T)(ay[v] + cb[r]), f, f1, f2, sp[0]);
        s1w[v] = f1;
        t1w[v] = f2;
        yd1w[v] = (T)ad[v];
        zs[0][0][r][q] = f;
        zs[0][1][r][q] = f1 * (T)ad[v];
      }
    }
    // ---------------- forward: layers 2..L (own rows)
    T sk[L - 1][4], tk[L - 1][4], ydk[L - 1][4];
    static_for<L - 1>([&](auto KI) {
      constexpr int k = decltype(KI)::value + 2;
      T zsrc[MB][4], zdsrc[MB][4];
      __syncthreads();  // every wave's rows of layer k - 1 are in zs
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          zsrc[mb][v] = zs[k - 2][0][16 * mb + E::row(g, v)][q];
          zdsrc[mb][v] = zs[k - 2][1][16 * mb + E::row(g, v)][q];
        }
      acc_t ay = mma_in<E, P>(BV[k - 2], kB, mma_src<E, MB>(AV[k - 2], zsrc, zero_acc<E>()));
      acc_t ad = mma_in<E, P>(BV[k - 2], lB, mma_src<E, MB>(AV[k - 2], zdsrc, zero_acc<E>()));
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * w + E::row(g, v);
        T f, f1, f2;
        softplus3((T)(ay[v] + cb[(k - 1) * H + r]), f, f1, f2, sp[0]);
        sk[k - 2][v] = f1; tk[k - 2][v] = f2; ydk[k - 2][v] = (T)ad[v];
        const T zd = f1 * (T)ad[v];
        if constexpr (k < L) {
          zs[k - 1][0][r][q] = f;
          zs[k - 1][1][r][q] = zd;
        } else {
          if (valid) aacc[v] += zd;
        }
      }
    });
    __syncthreads();  // zs and kl complete

    // ---------------- reverse
    T zdbar[4], zbar[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) { zdbar[v] = valid ? a_own[v] : (T)0; zbar[v] = (T)0; }
    static_for<L - 1>([&](auto KI) {
      constexpr int k = L - decltype(KI)::value;  // L, L-1, ..., 2
      T ydb[4], yb[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        ydb[v] = zdbar[v] * sk[k - 2][v];
        yb[v] = zbar[v] * sk[k - 2][v] + zdbar[v] * ydk[k - 2][v] * tk[k - 2][v];
        cacc[k - 1][v] += yb[v];
        const int rl = E::row(g, v);
        us[w][0][rl][q] = ydb[v];
        us[w][1][rl][q] = yb[v];
        xr[0][16 * w + rl][q] = ydb[v];
        xr[1][16 * w + rl][q] = yb[v];
      }
      __syncthreads();
      // weight gradients: Abar_k += ydot_bar (x) zdot_{k-1} + y_bar (x) z_{k-1}
#pragma unroll
      for (int nb = 0; nb < MB; ++nb) {
        acc_t c = accA[k - 2][nb];
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
          for (int s = 0; s < 4; ++s)
            c = E::mma(ufrag(p, s), (typename E::frag)zs[k - 2][1 - p][16 * nb + (lane & 15)][4 * s + g], c);
        accA[k - 2][nb] = c;
      }
      // Bbar_k += ydot_bar (x) lambda + y_bar (x) K
      {
        acc_t c = accB[k - 2];
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
          for (int s = 0; s < 4; ++s)
            c = E::mma(ufrag(p, s), (typename E::frag)kl[1 - p][lane & 15][4 * s + g], c);
        accB[k - 2] = c;
      }
      // propagate to layer k-1 (own rows): zdot_bar = A_k^T ydot_bar, z_bar = A_k^T y_bar
      acc_t pd = zero_acc<E>(), pz = zero_acc<E>();
#pragma unroll
      for (int s = 0; s < SH; ++s) {
        typename E::frag at;
        if constexpr (ATL) at = lAT[(((k - 2) * MB + w) * SH + s) * 64 + lane];
        else at = AT[k - 2][s];
        pd = E::mma(at, (typename E::frag)xr[0][4 * s + g][q], pd);
        pz = E::mma(at, (typename E::frag)xr[1][4 * s + g][q], pz);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) { zdbar[v] = (T)pd[v]; zbar[v] = (T)pz[v]; }
      __syncthreads();
    });
    // layer 1 (own rows = block w)
    {
      T ydb[4], yb[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        ydb[v] = zdbar[v] * s1w[v];
        yb[v] = zbar[v] * s1w[v] + zdbar[v] * yd1w[v] * t1w[v];
        cacc[0][v] += yb[v];
        const int rl = E::row(g, v);
        us[w][0][rl][q] = ydb[v];
        us[w][1][rl][q] = yb[v];
      }
      __syncthreads();
      acc_t c = accW1;
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int s = 0; s < 4; ++s)
          c = E::mma(ufrag(p, s), (typename E::frag)kl[1 - p][lane & 15][4 * s + g], c);
      accW1 = c;
      __syncthreads();  // staging areas free for the next tile
    }
  }

  // ---------------- write this workgroup's partial theta_bar (theta layout)
  double* out = part + (int64_t)blockIdx.x * tl.total;
  const int col = lane & 15;
  static_for<L - 1>([&](auto KI) {
    constexpr int k = decltype(KI)::value + 2;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * w + E::row(g, v);
#pragma unroll
      for (int nb = 0; nb < MB; ++nb)
        if (r < tl.H && 16 * nb + col < tl.H) out[tl.A[k] + (int64_t)r * tl.H + 16 * nb + col] = (double)accA[k - 2][nb][v];
      if (col < P && r < tl.H) out[tl.B[k] + (int64_t)r * P + col] = (double)accB[k - 2][v];
    }
  });
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = 16 * w + E::row(g, v);
    if (col < P && r < tl.H) out[tl.W1 + (int64_t)r * P + col] = (double)accW1[v];
  }
  // sums over the 16 points of each lane group
#pragma unroll
  for (int k = 1; k <= L; ++k) {
    const int64_t off = (k == 1) ? tl.c1 : tl.c[k];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double sv = sum16((double)cacc[k - 1][v]);
      if (off >= 0 && q == 0 && 16 * w + E::row(g, v) < tl.H) out[off + 16 * w + E::row(g, v)] = sv;
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const double sv = sum16((double)aacc[v]);
    if (q == 0 && 16 * w + E::row(g, v) < tl.H) out[tl.a + 16 * w + E::row(g, v)] = sv;
  }
#pragma unroll
  for (int s = 0; s < S1; ++s) {
    const double sv = sum16((double)bacc[s]);
    const int m = 4 * s + g;
    if (w == 0 && q == 0 && m < P) out[tl.b + m] = sv;
  }
}

// theta_bar[i] = sum_g part[g][i] in a fixed order.
__global__ void k_sum_partials(int64_t np, int G, const double* __restrict__ part, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  double s = 0.0;
  for (int g = 0; g < G; ++g) s += part[(int64_t)g * np + i];
  out[i] = s;
}

static int grid_of(int64_t n) {
  const int64_t tiles = (n + 15) / 16;
  return (int)(tiles < 1024 ? (tiles > 0 ? tiles : 1) : 1024);
}

int64_t param_backward_ws(int H, int L, int P, int prec, int64_t n) {
  (void)prec;
  const ThetaLayout tl = theta_layout(H, L, P, 1);
  auto al = [](int64_t x) { return (x + 255) & ~int64_t(255); };
  return 2 * al(8 * (int64_t)P * n) + al(8 * (int64_t)grid_of(n) * (tl.total + 64));
}

#define PA_ADJ_CONFIGS(X) \
  X(16, 2, 3) X(16, 2, 5) X(16, 2, 9) X(16, 3, 3) X(16, 3, 5) X(16, 3, 9) \
  X(32, 2, 3) X(32, 2, 5) X(32, 2, 9) X(32, 3, 3) X(32, 3, 5) X(32, 3, 9) \
  X(64, 2, 3) X(64, 2, 5) X(64, 2, 9) X(64, 3, 3) X(64, 3, 5) X(64, 3, 9) \
  X(16, 4, 3) X(16, 4, 5) X(16, 4, 9) X(32, 4, 3) X(32, 4, 5) X(32, 4, 9) X(64, 4, 3) X(64, 4, 5) X(64, 4, 9)

int launch_param_backward(const PrepLayout& lay, const ThetaLayout& tl, int nsv, int prec,
                          const unsigned char* prep, const ModelConst& mc, int64_t n, const double* F,
                          const double* P_bar, double* theta_bar, unsigned char* ws, hipStream_t s) {
  if (prec != PREC_F64 && prec != PREC_F32) return -3;
  auto al = [](int64_t x) { return (x + 255) & ~int64_t(255); };
  double* K = (double*)ws;
  double* Lam = (double*)(ws + al(8 * (int64_t)lay.P * n));
  double* part = (double*)(ws + 2 * al(8 * (int64_t)lay.P * n));
  const int G = grid_of(n);
  if (n > 0) {
    const unsigned nb = (unsigned)((n + 255) / 256);
    switch (nsv) {
      case 0: k_adj_inputs<0><<<nb, 256, 0, s>>>(n, F, P_bar, mc, K, Lam); break;
      case 1: k_adj_inputs<1><<<nb, 256, 0, s>>>(n, F, P_bar, mc, K, Lam); break;
      case 2: k_adj_inputs<2><<<nb, 256, 0, s>>>(n, F, P_bar, mc, K, Lam); break;
      default: return -1;
    }
  }
  const unsigned block = 64 * (lay.H / 16);
  bool done = false;
#define PA_ADJ_DISPATCH(h, l, p)                                                                      \
  if (!done && lay.H == h && lay.L == l && lay.P == p) {                                               \
    if (prec == PREC_F64) k_param_bwd<h, l, p, PREC_F64><<<G, block, 0, s>>>(prep, lay, tl, n, K, Lam, part); \
    else k_param_bwd<h, l, p, PREC_F32><<<G, block, 0, s>>>(prep, lay, tl, n, K, Lam, part);         \
    done = true;                                                                                        \
  }
  PA_ADJ_CONFIGS(PA_ADJ_DISPATCH)
#undef PA_ADJ_DISPATCH
  if (!done) return -2;
  k_sum_partials<<<(unsigned)((tl.total + 255) / 256), 256, 0, s>>>(tl.total, G, part, theta_bar);
  return 0;
}

}  // namespace pa
