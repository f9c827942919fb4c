// Shared pieces of the hex kernels: operator kinds, the compile-time 1D tables and
// their even-odd contraction, small device helpers and the XCD-aware block mapping.
#pragma once
#include "mf_internal.h"
#include "hex_tables.inc"

namespace mf {


enum { K_MASS = MF_OP_MASS, K_HELM = MF_OP_HELMHOLTZ, K_LAP = MF_OP_LAPLACIAN, K_POIS = MF_OP_POISSON };

// Compile-time 1D tables (generated from the host table code at build time, see
// gen_hex_tables.cpp): constants are materialised with scalar moves where used.
template <typename T, int N> struct TabT {
  static __device__ __forceinline__ constexpr T B(int a, int i) { return T(HexC<N>::B[a][i]); }
  static __device__ __forceinline__ constexpr T D(int a, int b) { return T(HexC<N>::D[a][b]); }
  static __device__ __forceinline__ constexpr T dB(int a, int i) { return T(HexC<N>::dB[a][i]); }
  static __device__ __forceinline__ constexpr T g(int a) { return T(HexC<N>::g[a]); }
  static __device__ __forceinline__ constexpr T w(int a) { return T(HexC<N>::w[a]); }
};

// The 1D matrices as n x n accessors: B and the collocation derivative D, and their
// transposes (for the test-function side).
template <int N> struct MatB { static constexpr double at(int a, int i) { return HexC<N>::B[a][i]; } };
template <int N> struct MatBt { static constexpr double at(int a, int i) { return HexC<N>::B[i][a]; } };
template <int N> struct MatD { static constexpr double at(int a, int i) { return HexC<N>::D[a][i]; } };
template <int N> struct MatDt { static constexpr double at(int a, int i) { return HexC<N>::D[i][a]; } };

// out[a] = sum_i M(a, i) in[i] for a 1D matrix with the reflection symmetry of the
// tensor bases: M(n-1-a, n-1-i) = SIGN M(a, i). The Gauss points and GLL nodes are
// symmetric about the middle of the interval, so B (and its transpose) has SIGN = +1
// and the derivative D has SIGN = -1. Splitting the input into its even part
// in[i] + in[n-1-i] and odd part in[i] - in[n-1-i] gives each output pair
// (a, n-1-a) from two half-size products: about n^2/2 + n multiply-adds instead of
// n^2, and half as many distinct constants.
template <int N, typename M, int SIGN> constexpr bool reflection_symmetric() {
  for (int a = 0; a < N; a++)
    for (int i = 0; i < N; i++) {
      const double d = M::at(a, i) - SIGN * M::at(N - 1 - a, N - 1 - i);
      const double m = M::at(a, i) < 0 ? -M::at(a, i) : M::at(a, i);
      if ((d < 0 ? -d : d) > 1e-13 * (m > 1 ? m : 1)) return false;
    }
  return true;
}

template <typename T, int N, typename M, int SIGN>
__device__ __forceinline__ void eo_contract(const T (&in)[N], T (&out)[N]) {
  static_assert(reflection_symmetric<N, M, SIGN>(), "1D table lacks the reflection symmetry");
  constexpr int H = N / 2;
  T e[H], o[H];
#pragma unroll
  for (int i = 0; i < H; i++) {
    e[i] = in[i] + in[N - 1 - i];
    o[i] = in[i] - in[N - 1 - i];
  }
#pragma unroll
  for (int a = 0; a < H; a++) {
    T pe = T(0), po = T(0);
#pragma unroll
    for (int i = 0; i < H; i++) {
      pe += T(0.5 * (M::at(a, i) + M::at(a, N - 1 - i))) * e[i];
      po += T(0.5 * (M::at(a, i) - M::at(a, N - 1 - i))) * o[i];
    }
    if constexpr (N % 2 == 1) pe += T(M::at(a, H)) * in[H];
    out[a] = pe + po;
    out[N - 1 - a] = SIGN > 0 ? pe - po : po - pe;
  }
  if constexpr (N % 2 == 1) {
    T m = T(0);
#pragma unroll
    for (int i = 0; i < H; i++) m += T(M::at(H, i)) * (SIGN > 0 ? e[i] : o[i]);
    if constexpr (SIGN > 0) m += T(M::at(H, H)) * in[H];
    out[H] = m;
  }
}

// 1/a from the hardware reciprocal refined by Newton steps e = 1 - a r, r += r e
// (two in FP64, one in FP32): about half the instructions of the IEEE division
// sequence, within an ulp or two of the rounded quotient (a > 0, |det J| here).
__device__ __forceinline__ double recip(double a) {
  double r = __builtin_amdgcn_rcp(a);
  double e = __builtin_fma(-a, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-a, r, 1.0);
  return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float recip(float a) {
  const float r = __builtin_amdgcn_rcpf(a);
  return __builtin_fmaf(r, __builtin_fmaf(-a, r, 1.0f), r);
}

__device__ __forceinline__ void atomic_add_f(double *p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add_f(float *p, float v) { unsafeAtomicAdd(p, v); }

// (xcd_batch / xcd_grid: the XCD-aware workgroup mapping, in mf_internal.h)

}  // namespace mf
