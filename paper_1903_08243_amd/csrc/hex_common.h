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

namespace mf {

// ---------------------------------------------------------------------------------
// FP32 1D contractions on the matrix cores.
//
// v_mfma_f32_4x4x1f32 treats a wavefront as 16 blocks of 4 lanes and adds, per block,
// the outer product of a 4-vector A (one value per lane of the block) and a 4-vector
// B (likewise) to a 4 x 4 accumulator; lane 4b + j receives column j of block b's
// result in its four accumulator registers (row m in register m). With A = column k
// of a 1D table (lane 4b + r holds row r) and B = each lane's own k-th input, the
// lane's column is the table applied to its own pencil: four rows of the product for
// one multiply instruction on the matrix cores (FP32, with FP32 accumulation), and no
// data moves between lanes. Each lane's table values depend only on lane & 3.
//
// n <= 4: the plain n x n product, one instruction per input. n >= 5: the even-odd
// split of eo_contract (even and odd halves of at most 4 rows each, one instruction per
// input e_i, o_i and the middle node), with the splits and recombinations on the VALU.
typedef float mf_f4 __attribute__((ext_vector_type(4)));

// Per-lane table operand of matrix M (n x n, reflection sign SIGN), for lane row r:
// column j of the instruction sequence (j < n). Plain (n <= 4): entry M(r, j).
// Even-odd: j < H + (n odd): the even half's input j (e_j, or the middle node for
// j = H), then j = H + odd + i: the odd half's input o_i.
template <int N, typename M, int SIGN> constexpr float mfma_col(int r, int j) {
  constexpr int H = N / 2, ODD = N % 2;
  if (N <= 4) return (r < N) ? float(M::at(r, j)) : 0.0f;
  if (j < H + ODD) {
    // even half: rows a < H (and for SIGN > 0 the middle row H)
    if (j < H) {
      if (r < H) return float(0.5 * (M::at(r, j) + M::at(r, N - 1 - j)));
      if (ODD && r == H && SIGN > 0) return float(M::at(H, j));
      return 0.0f;
    }
    if (r < H) return float(M::at(r, H));  // middle input
    if (ODD && r == H && SIGN > 0) return float(M::at(H, H));
    return 0.0f;
  }
  const int i = j - H - ODD;
  if (r < H) return float(0.5 * (M::at(r, i) - M::at(r, N - 1 - i)));
  if (ODD && r == H && SIGN < 0) return float(M::at(H, i));
  return 0.0f;
}

// The four tables of the hex kernels (B, D and their transposes) as per-lane columns:
// MfmaCols<N>::v[t][r][j] for t = 0 B, 1 D, 2 B^T, 3 D^T.
template <int N> struct MfmaCols {
  float v[4][4][8];
};
template <int N> constexpr MfmaCols<N> make_mfma_cols() {
  MfmaCols<N> c{};
  for (int r = 0; r < 4; r++)
    for (int j = 0; j < N; j++) {
      c.v[0][r][j] = mfma_col<N, MatB<N>, 1>(r, j);
      c.v[1][r][j] = mfma_col<N, MatD<N>, -1>(r, j);
      c.v[2][r][j] = mfma_col<N, MatBt<N>, 1>(r, j);
      c.v[3][r][j] = mfma_col<N, MatDt<N>, -1>(r, j);
    }
  return c;
}

template <int N, int SIGN>
__device__ __forceinline__ void mfma_contract(const float (&a)[N], const float (&in)[N], float (&out)[N]) {
  constexpr int H = N / 2, ODD = N % 2;
  if constexpr (N <= 4) {
    mf_f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int j = 0; j < N; j++) acc = __builtin_amdgcn_mfma_f32_4x4x1f32(a[j], in[j], acc, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < N; r++) out[r] = acc[r];
  } else {
    mf_f4 pe = {0.0f, 0.0f, 0.0f, 0.0f}, po = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int i = 0; i < H; i++) pe = __builtin_amdgcn_mfma_f32_4x4x1f32(a[i], in[i] + in[N - 1 - i], pe, 0, 0, 0);
    if constexpr (ODD) pe = __builtin_amdgcn_mfma_f32_4x4x1f32(a[H], in[H], pe, 0, 0, 0);
#pragma unroll
    for (int i = 0; i < H; i++)
      po = __builtin_amdgcn_mfma_f32_4x4x1f32(a[H + ODD + i], in[i] - in[N - 1 - i], po, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < H; r++) {
      out[r] = pe[r] + po[r];
      out[N - 1 - r] = SIGN > 0 ? pe[r] - po[r] : po[r] - pe[r];
    }
    if constexpr (ODD) out[H] = SIGN > 0 ? pe[H] : po[H];
  }
}

// The FP32 kernels keep the four tables' per-lane columns in LDS (128 floats per
// workgroup, filled from kMfmaCols) and read the 8 entries of one table into registers
// just before each contraction, so the tables occupy no registers between uses (kept
// resident they cost 4n VGPRs, and occupancy). LaneTabs holds the lane's row pointer;
// it is empty in FP64, whose contractions stay on the VALU with compile-time constants.
template <int N> __constant__ MfmaCols<N> kMfmaCols = make_mfma_cols<N>();
template <typename T, int N> struct LaneTabs {
  __device__ __forceinline__ void bind(const T *) {}
};
template <int N> struct LaneTabs<float, N> {
  const float *row;  // this lane's row (lane & 3) of the LDS copy, [table][row][8]
  __device__ __forceinline__ void bind(const float *lds_tab) { row = lds_tab + (threadIdx.x & 3) * 8; }
};
// workgroup-cooperative copy of the tables into LDS (before a barrier)
template <int N> __device__ __forceinline__ void fill_mfma_tables(float *lds_tab, int t, int nthreads) {
  const float *src = &kMfmaCols<N>.v[0][0][0];
  for (int i = t; i < 128; i += nthreads) lds_tab[i] = src[i];
}

template <int TAB, int N> struct MatOf;
template <int N> struct MatOf<0, N> { using type = MatB<N>; };
template <int N> struct MatOf<1, N> { using type = MatD<N>; };
template <int N> struct MatOf<2, N> { using type = MatBt<N>; };
template <int N> struct MatOf<3, N> { using type = MatDt<N>; };

// out = table TAB (0 B, 1 D, 2 B^T, 3 D^T) applied to the pencil `in`: on the matrix
// cores in FP32, on the VALU (even-odd, compile-time constants) in FP64.
template <typename T, int N, int TAB>
__device__ __forceinline__ void contract(const LaneTabs<T, N> &L, const T (&in)[N], T (&out)[N]) {
  constexpr int SIGN = (TAB & 1) ? -1 : 1;
  if constexpr (__is_same(T, float)) {
    static_assert(reflection_symmetric<N, typename MatOf<TAB, N>::type, SIGN>(), "table symmetry");
    typedef float f4v __attribute__((ext_vector_type(4)));
    const f4v lo = *reinterpret_cast<const f4v *>(L.row + TAB * 32);
    const f4v hi = *reinterpret_cast<const f4v *>(L.row + TAB * 32 + 4);
    float a[N];
#pragma unroll
    for (int j = 0; j < N; j++) a[j] = j < 4 ? lo[j] : hi[j - 4];
    mfma_contract<N, SIGN>(a, in, out);
  } else {
    eo_contract<T, N, typename MatOf<TAB, N>::type, SIGN>(in, out);
  }
}

}  // namespace mf
