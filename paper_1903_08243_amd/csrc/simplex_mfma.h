// One-component simplex operators (MASS with a vertex coefficient, HELMHOLTZ,
// LAPLACIAN, POISSON) with both contractions on the matrix cores, for tetrahedra
// (DIM = 3) and triangles (DIM = 2). Simplices are not sum-factorised (Section 4): the
// local kernel contracts dense tabulations of the reference basis at the quadrature
// points (Section 2.1), and over a batch of cells both contractions are GEMMs with the
// tabulation shared by every cell:
//   forward  U[(q,a)][cell] = sum_i tab[q][i][a] x[i][cell]
//   backward y[i][cell]     = sum_(q,a) tab[q][i][a] P[(q,a)][cell]
// where the rows a = 0..DIM-1 are the reference gradient and a = DIM the basis value.
// Computed with v_mfma_{f32,f64}_16x16x4 (operands: A[m][k] from lane m + 16 k, B[k][n]
// from lane n + 16 k; result C[m][n] in lane n + 16 (m / 4), element m % 4 for FP32 and
// in lane n + 16 (m % 4), element m / 4 for FP64, as measured on gfx950). A wavefront
// owns 16 cells (n = cell) and one accumulator. The forward rows are ordered so that
// the row of (q = 4 r + g, a) lands in lane group g, element a, so one K-step chain
// leaves lane (cell, g) with the reference gradient and the value of u at point q (for
// DIM = 2 the element a = 3 is padding); the lane forms the pointwise fluxes there,
// which are exactly the B operands of the backward K-steps (r, a), a = 0..DIM. The
// per-lane A operands are host-built (simplex_mfma_scalar_tables).
#pragma once
#include "mf_internal.h"

namespace mf {

typedef float mf_floatx4 __attribute__((ext_vector_type(4)));
typedef double mf_doublex4 __attribute__((ext_vector_type(4)));
template <typename T> struct Mfma16;
template <> struct Mfma16<float> {
  typedef mf_floatx4 V;
  static __device__ __forceinline__ V fma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma16<double> {
  typedef mf_doublex4 V;
  static __device__ __forceinline__ V fma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

template <int DIM, int K> constexpr int simplex_nodes() {
  return DIM == 3 ? (K + 1) * (K + 2) * (K + 3) / 6 : (K + 1) * (K + 2) / 2;
}

// The action of one wavefront's 16 cells. gp: the cell's geometry (d xi_b / d x_a at
// b DIM + a, then |det J|), cp: its DIM + 1 vertex coefficients (null: 1), entries 64
// apart; mp: its map entries, 64 apart. Tables (A.tab): phi [nq][D], reference
// gradients [nq][D][DIM], weights [nq], vertex basis [nq][DIM+1], then fwd[r][s][64]
// and bwd[t][r][DIM+1][64]. yacc[t][v]: the local result at node 16 t + 4 g + v (FP32)
// or 16 t + g + 4 v (FP64), g = lane / 16.
template <typename T, int DIM, int K, int NQ, int KIND>
__device__ __forceinline__ void simplex_scalar_cells16(
    const TetArgs<T> &A, const int32_t *mp, const T *gp, const T *cp, const bool valid, const int lane,
    typename Mfma16<T>::V (&yacc)[(simplex_nodes<DIM, K>() + 15) / 16]) {
  using MF = Mfma16<T>;
  using V4 = typename MF::V;
  constexpr int D = simplex_nodes<DIM, K>(), NV = DIM + 1, NB = DIM + 1;
  constexpr int NR = (NQ + 3) / 4, NS = (D + 3) / 4, NT = (D + 15) / 16;
  constexpr bool VAL = KIND == MF_OP_MASS || KIND == MF_OP_HELMHOLTZ;
  constexpr bool GRAD = KIND != MF_OP_MASS;
  constexpr bool COEF = KIND == MF_OP_MASS || KIND == MF_OP_POISSON;
  const int g = lane >> 4;
  T Ki[DIM * DIM];
#pragma unroll
  for (int m = 0; m < DIM * DIM; m++) Ki[m] = gp[m * 64];
  const T adet = gp[DIM * DIM * 64];
  T cv[NV];
#pragma unroll
  for (int v = 0; v < NV; v++) cv[v] = (COEF && cp) ? cp[v * 64] : T(1);
  const T *qw = A.tab + NQ * D * (1 + DIM);
  const T *vb = qw + NQ;
  const T *fwd = vb + NQ * NV;
  const T *bwd = fwd + NR * NS * 64;
  T xv[NS];
#pragma unroll
  for (int s = 0; s < NS; s++) {
    const int i = 4 * s + g;
    const int idx = (valid && i < D) ? mp[i * 64] : -1;
    xv[s] = idx >= 0 ? A.x[idx] : T(0);
  }
#pragma unroll
  for (int t = 0; t < NT; t++) yacc[t] = V4{T(0), T(0), T(0), T(0)};
  constexpr int RU = NR <= 4 ? NR : 1;
#pragma unroll RU
  for (int r = 0; r < NR; r++) {
    V4 acc = V4{T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int s = 0; s < NS; s++) acc = MF::fma(fwd[(r * NS + s) * 64 + lane], xv[s], acc);
    const int q = 4 * r + g, qq = q < NQ ? q : 0;
    const T wd = q < NQ ? qw[qq] * adet : T(0);
    T cq = T(1);
    if constexpr (COEF) {
      cq = T(0);
#pragma unroll
      for (int v = 0; v < NV; v++) cq += vb[NV * qq + v] * cv[v];
    }
    T P[DIM + 1];
#pragma unroll
    for (int d = 0; d <= DIM; d++) P[d] = T(0);
    if constexpr (GRAD) {
      // physical gradient G_a = sum_b g_b d xi_b / d x_a scaled by w |det| (kappa), and
      // its reference-direction form P_d = sum_a d xi_d / d x_a G_a
      const T sc = wd * (KIND == MF_OP_POISSON ? cq : T(1));
      T G[DIM];
#pragma unroll
      for (int a = 0; a < DIM; a++) {
        T v = T(0);
#pragma unroll
        for (int b = 0; b < DIM; b++) v += acc[b] * Ki[b * DIM + a];
        G[a] = sc * v;
      }
#pragma unroll
      for (int d = 0; d < DIM; d++) {
        T v = T(0);
#pragma unroll
        for (int a = 0; a < DIM; a++) v += G[a] * Ki[d * DIM + a];
        P[d] = v;
      }
    }
    if constexpr (VAL) P[DIM] = wd * (KIND == MF_OP_MASS ? cq : T(1)) * acc[DIM];
#pragma unroll
    for (int t = 0; t < NT; t++) {
      const T *bt = bwd + (t * NR + r) * NB * 64 + lane;
      if constexpr (GRAD)
#pragma unroll
        for (int d = 0; d < DIM; d++) yacc[t] = MF::fma(bt[d * 64], P[d], yacc[t]);
      if constexpr (VAL) yacc[t] = MF::fma(bt[DIM * 64], P[DIM], yacc[t]);
    }
  }
}

// Atomic or coloured scatter: one wavefront per 16 cells of the AoSoA layout
// ([cell/64][entry][64] map, geometry, coefficients), contiguous ranges of quarters
// per XCD.
template <typename T, int DIM, int K, int NQ, int KIND, bool ATOMIC>
__global__ void __launch_bounds__(64) simplex_scalar_mfma_kernel(const TetArgs<T> A) {
  using V4 = typename Mfma16<T>::V;
  constexpr int D = simplex_nodes<DIM, K>(), NT = (D + 15) / 16, G = DIM * DIM + 1, NV = DIM + 1;
  const int lane = threadIdx.x;
  const int j = lane & 15, g = lane >> 4;
  const int64_t nqb = 4 * ((A.c1 + 63) / 64 - A.c0 / 64), per = (nqb + 7) / 8;
  const int64_t qb = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (qb >= nqb) return;
  const int64_t batch = A.c0 / 64 + qb / 4;
  const int cl = 16 * (int)(qb % 4) + j;
  const int64_t cell = batch * 64 + cl;
  bool valid = cell >= A.c0 && cell < A.c1;
  if (valid && A.cell_user) {
    const int64_t u = A.cell_user[cell];
    valid = u >= A.ulo && u < A.uhi;
  }
  const int32_t *mp = A.map + batch * (D * 64) + cl;
  V4 yacc[NT];
  simplex_scalar_cells16<T, DIM, K, NQ, KIND>(A, mp, A.geo + batch * (G * 64) + cl,
                                              A.coef ? A.coef + batch * (NV * 64) + cl : nullptr, valid, lane, yacc);
  constexpr bool F64 = sizeof(T) == 8;
#pragma unroll
  for (int t = 0; t < NT; t++)
#pragma unroll
    for (int v = 0; v < 4; v++) {
      const int i = F64 ? 16 * t + g + 4 * v : 16 * t + 4 * g + v;
      const int idx = (valid && i < D) ? mp[i * 64] : -1;
      if (idx >= 0) {
        if constexpr (ATOMIC) unsafeAtomicAdd(&A.y[idx], yacc[t][v]);
        else A.y[idx] += yacc[t][v];  // cells of one launch share no node
      }
    }
}

// Patch scatter (SimplexPatchArgs): one workgroup of four wavefronts per patch; each
// round the wavefronts take the patch's next 64 slots, the local results are summed
// into the patch's nodes in LDS (FP64 sums for both precisions: LDS FP32 atomic adds
// measured several times slower), and after the last round every node of the patch is
// written once: into y if no other patch touches it, else into its slot of sbuf. The
// slot geometry holds d xi / d x, |det J| and, for MASS and POISSON, the vertex
// coefficients.
template <typename T, int DIM, int K, int NQ, int KIND>
__global__ void __launch_bounds__(256) simplex_scalar_patch_kernel(const TetArgs<T> A, const SimplexPatchArgs<T> P) {
  using V4 = typename Mfma16<T>::V;
  constexpr int D = simplex_nodes<DIM, K>(), NT = (D + 15) / 16;
  constexpr bool F64 = sizeof(T) == 8;
  constexpr bool COEF = KIND == MF_OP_MASS || KIND == MF_OP_POISSON;
  constexpr int G0 = DIM * DIM + 1, G = COEF ? G0 + DIM + 1 : G0;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double *acc = reinterpret_cast<double *>(smem_raw);
  const int64_t p = xcd_batch(blockIdx.x, P.npatch);
  if (p >= P.npatch) return;  // whole workgroup: no barrier skipped
  const int n0 = P.nptr[p], nn = P.nptr[p + 1] - n0;
  for (int e = threadIdx.x; e < nn; e += blockDim.x) acc[e] = 0.0;
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j = lane & 15, g = lane >> 4, cl = 16 * w + j;
  const int nblk = P.cap / 64;
  for (int r = 0; r < nblk; r++) {
    const int64_t blk = p * nblk + r;
    const T *gp = P.geo + blk * (G * 64) + cl;
    V4 yacc[NT];
    simplex_scalar_cells16<T, DIM, K, NQ, KIND>(A, P.map + blk * (D * 64) + cl, gp, COEF ? gp + G0 * 64 : nullptr,
                                                true, lane, yacc);
    const uint16_t *lp = P.lmap + blk * (D * 64) + cl;
#pragma unroll
    for (int t = 0; t < NT; t++)
#pragma unroll
      for (int v = 0; v < 4; v++) {
        const int i = F64 ? 16 * t + g + 4 * v : 16 * t + 4 * g + v;
        if (i < D) {
          const int l = lp[i * 64];
          if (l != kSlotSkip) atomicAdd(&acc[l], (double)yacc[t][v]);
        }
      }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nn; e += blockDim.x) {
    const int32_t o = P.out[n0 + e];
    if (o & kSharedOut) P.sbuf[o & (kSharedOut - 1)] = (T)acc[e];
    else A.y[o] = P.accumulate ? A.y[o] + (T)acc[e] : (T)acc[e];
  }
}

template <typename T, int DIM, int K, int NQ, int KIND>
static int launch_simplex_scalar_kq(const TetArgs<T> &a, const SimplexPatchArgs<T> *p, bool atomic, hipStream_t s) {
  if (p) {
    if (p->npatch <= 0) return MF_OK;
    const size_t lds = (size_t)p->nmax * sizeof(double);
    if (lds > 64 * 1024) return fail(MF_EUNSUPPORTED, "simplex patch scatter: patch node list too long for LDS");
    simplex_scalar_patch_kernel<T, DIM, K, NQ, KIND>
        <<<dim3((unsigned)xcd_grid(p->npatch)), dim3(256), lds, s>>>(a, *p);
  } else {
    const int64_t nqb = 4 * ((a.c1 + 63) / 64 - a.c0 / 64);
    if (a.c1 <= a.c0) return MF_OK;
    const dim3 g((unsigned)(((nqb + 7) / 8) * 8)), b(64);
    if (atomic) simplex_scalar_mfma_kernel<T, DIM, K, NQ, KIND, true><<<g, b, 0, s>>>(a);
    else simplex_scalar_mfma_kernel<T, DIM, K, NQ, KIND, false><<<g, b, 0, s>>>(a);
  }
  MF_HIP(hipGetLastError());
  return MF_OK;
}

// kind dispatch for one (DIM, K, NQ): patch scatter when p is set, else atomic or
// coloured
template <typename T, int DIM, int K, int NQ>
static int launch_simplex_scalar_k(int kind, const TetArgs<T> &a, const SimplexPatchArgs<T> *p, bool atomic,
                                   hipStream_t s) {
  switch (kind) {
    case MF_OP_MASS: return launch_simplex_scalar_kq<T, DIM, K, NQ, MF_OP_MASS>(a, p, atomic, s);
    case MF_OP_HELMHOLTZ: return launch_simplex_scalar_kq<T, DIM, K, NQ, MF_OP_HELMHOLTZ>(a, p, atomic, s);
    case MF_OP_LAPLACIAN: return launch_simplex_scalar_kq<T, DIM, K, NQ, MF_OP_LAPLACIAN>(a, p, atomic, s);
    case MF_OP_POISSON: return launch_simplex_scalar_kq<T, DIM, K, NQ, MF_OP_POISSON>(a, p, atomic, s);
  }
  return fail(MF_EUNSUPPORTED, "simplex one-component operator: kind");
}

}  // namespace mf
