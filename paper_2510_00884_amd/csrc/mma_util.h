// Matrix-core helpers shared by the network kernels: fragment access into
// the prepared-parameter buffer, compile-time loops, K-step products with the
// point tile on the N dimension, and cross-lane sums.
#pragma once

#include <type_traits>
#include <utility>

#include "pa_internal.h"

namespace pa {
template <class E>
__device__ inline const typename E::frag* frag_ptr(const unsigned char* prep, const PrepLayout& l, int which);

template <>
__device__ inline const double* frag_ptr<EngF64>(const unsigned char* prep, const PrepLayout& l, int which) {
  return (const double*)(prep + (which == 0 ? l.x_W1 : which == 1 ? l.x_A : l.x_B));
}
template <>
__device__ inline const float* frag_ptr<EngF32>(const unsigned char* prep, const PrepLayout& l, int which) {
  return (const float*)(prep + (which == 0 ? l.y_W1 : which == 1 ? l.y_A : l.y_B));
}
template <>
__device__ inline const bf16x8* frag_ptr<EngBF16>(const unsigned char* prep, const PrepLayout& l, int which) {
  return (const bf16x8*)(prep + (which == 0 ? l.z_W1 : which == 1 ? l.z_A : l.z_B));
}

template <class E, int H>
__device__ constexpr int steps_hidden() { return E::KS == 4 ? H / 4 : (H + 31) / 32; }
template <class E, int P>
__device__ constexpr int steps_input() { return E::KS == 4 ? (P + 3) / 4 : 1; }

// acc += A (16 x H, this wave's rows) * src (H x 16), where src holds, for
// every 16-row block mb, the lane's 4 values at rows 16mb + E::row(g, v).
template <class E, int MB>
__device__ inline typename E::acc mma_src(const typename E::frag* A, const typename E::T (&src)[MB][4],
                                          typename E::acc c) {
  if constexpr (E::KS == 4) {
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int v = 0; v < 4; ++v) c = E::mma(A[mb * 4 + v], (typename E::frag)src[mb][v], c);
  } else {
#pragma unroll
    for (int t = 0; t < (MB + 1) / 2; ++t) {
      bf16x8 b;
      const int t1 = (2 * t + 1 < MB) ? 2 * t + 1 : 2 * t;
#pragma unroll
      for (int e = 0; e < 4; ++e) b[e] = (__bf16)src[2 * t][e];
#pragma unroll
      for (int e = 0; e < 4; ++e) b[4 + e] = (2 * t + 1 < MB) ? (__bf16)src[t1][e] : (__bf16)0.0f;
      c = E::mma(A[t], b, c);
    }
  }
  return c;
}

// acc += Bk (16 x P) * K (P x 16) over the input features.
template <class E, int P>
__device__ inline typename E::acc mma_in(const typename E::frag* A, const typename E::frag* kB,
                                         typename E::acc c) {
#pragma unroll
  for (int s = 0; s < steps_input<E, P>(); ++s) c = E::mma(A[s], kB[s], c);
  return c;
}

// Compile-time loop: f(std::integral_constant<int, I>) for I = 0..N-1, so
// every register-array index inside the body is a constant.
template <class F, int... Is>
__device__ inline void static_for_impl(F&& f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, class F>
__device__ inline void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

__device__ constexpr int hess_m(int h, int P) {
  int c = 0;
  for (int m = 0; m < P; ++m)
    for (int n = m; n < P; ++n) {
      if (c == h) return m;
      ++c;
    }
  return 0;
}
__device__ constexpr int hess_n(int h, int P) {
  int c = 0;
  for (int m = 0; m < P; ++m)
    for (int n = m; n < P; ++n) {
      if (c == h) return n;
      ++c;
    }
  return 0;
}

// Pair t of the column-major upper triangle (m = column, n <= m).
__host__ __device__ constexpr int colmaj_m(int t) {
  int m = 0;
  while (t > m) { t -= m + 1; ++m; }
  return m;
}
__host__ __device__ constexpr int colmaj_n(int t) { return t - colmaj_m(t) * (colmaj_m(t) + 1) / 2; }
// Packed row-major index of pair (n, m), n <= m.
__host__ __device__ constexpr int packed_index(int n, int m, int P) { return n * P - n * (n - 1) / 2 + (m - n); }

template <class E> __device__ inline typename E::acc zero_acc() { return typename E::acc{0, 0, 0, 0}; }

// Exchanges between lane halves on gfx950 (checked on the device):
// swap32(a, b) leaves a = [a lanes 0-31, b lanes 0-31] and
// b = [a lanes 32-63, b lanes 32-63]; swap16(a, b) does the same with the
// 16-lane rows, a = [a.r0, b.r0, a.r2, b.r2], b = [a.r1, b.r1, a.r3, b.r3].
// A double moves as its two dwords.  The operands are pinned to distinct
// registers first: the compiler may otherwise treat a swap of two equal
// values as a no-op and reuse one result for both.
__device__ inline void swap32(double& a, double& b) {
  asm volatile("" : "+v"(a), "+v"(b));
  const unsigned long long ua = __builtin_bit_cast(unsigned long long, a);
  const unsigned long long ub = __builtin_bit_cast(unsigned long long, b);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)ua, (unsigned)ub, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
  a = __builtin_bit_cast(double, (unsigned long long)lo[0] | ((unsigned long long)hi[0] << 32));
  b = __builtin_bit_cast(double, (unsigned long long)lo[1] | ((unsigned long long)hi[1] << 32));
}
__device__ inline void swap16(double& a, double& b) {
  asm volatile("" : "+v"(a), "+v"(b));
  const unsigned long long ua = __builtin_bit_cast(unsigned long long, a);
  const unsigned long long ub = __builtin_bit_cast(unsigned long long, b);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)ua, (unsigned)ub, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
  a = __builtin_bit_cast(double, (unsigned long long)lo[0] | ((unsigned long long)hi[0] << 32));
  b = __builtin_bit_cast(double, (unsigned long long)lo[1] | ((unsigned long long)hi[1] << 32));
}

// Sum a per-lane partial over the four lane groups (rows) of the wave; every
// lane receives the sum for its column.  All 64 lanes must be active.
__device__ inline double group_sum(double x) {
  double y = x;
  swap32(x, y);  // x = [r0, r1, r0, r1], y = [r2, r3, r2, r3]
  double s = x + y, t = s;
  swap16(s, t);  // s = [c01, c01, c23, c23] halves ... summed below
  return s + t;
}

// Sum four per-lane partials p0..p3 (one per column) over the four lane
// groups of a wave.  On return lane group g holds the full sum of column g
// for its point.  All 64 lanes must be active.
__device__ inline double reduce4(double p0, double p1, double p2, double p3, int g) {
  (void)g;
  swap32(p0, p2);  // p0 = [p0.r0, p0.r1, p2.r0, p2.r1], p2 = [p0.r2, p0.r3, p2.r2, p2.r3]
  swap32(p1, p3);
  double k0 = p0 + p2, k1 = p1 + p3;  // rows: [col0 (r0+r2), col0 (r1+r3), col2 .., col2 ..], col1/col3 likewise
  swap16(k0, k1);  // k0 = [k0.r0, k1.r0, k0.r2, k1.r2], k1 = [k0.r1, k1.r1, k0.r3, k1.r3]
  return k0 + k1;
}

// Sum over the 16 lanes that share a lane group (the 16 points of a tile).
__device__ inline double sum16(double x) {
  x += __shfl_xor(x, 1);
  x += __shfl_xor(x, 2);
  x += __shfl_xor(x, 4);
  x += __shfl_xor(x, 8);
  return x;
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

}  // namespace pa
