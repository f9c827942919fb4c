// Triangle operators of degree 1-6 on the matrix cores: the one-component forms (MASS
// with a vertex coefficient, HELMHOLTZ, LAPLACIAN, POISSON) from simplex_mfma.h with
// DIM = 2, and 2D linear elasticity below
// (geometry [cell/64][5][64]: d xi_b / d x_a at 2 b + a, |det J|; coefficients
// [cell/64][3][64]), on the rules the triangle setup takes for these integrands: the
// collapsed Gauss product rules of n^2 points, n = 1..8.
#include "simplex_mfma.h"

namespace mf {

// 2D linear elasticity (two node-interleaved components; stress lambda tr(grad u) I +
// mu (grad u + grad u^T)) in the same GEMM form: one accumulator per component, its
// rows a = 0, 1 the reference gradient (the value row a = 2 of the shared tables is
// not used); backward K-steps (r, 0) and (r, 1).
// The action of one wavefront's 16 cells (mp, gp: the cell's map and geometry entries,
// 64 apart): yacc[t][c][v] is component c at node 16 t + 4 g + v (FP32) or 16 t + g + 4 v
// (FP64), g = lane / 16.
template <typename T, int K, int NQ>
__device__ __forceinline__ void tri_elas_cells16(const TetArgs<T> &A, const int32_t *mp, const T *gp, const bool valid,
                                                 const int lane,
                                                 typename Mfma16<T>::V (&yacc)[(simplex_nodes<2, K>() + 15) / 16][2]) {
  using MF = Mfma16<T>;
  using V4 = typename MF::V;
  constexpr int D = simplex_nodes<2, K>(), NR = (NQ + 3) / 4, NS = (D + 3) / 4, NT = (D + 15) / 16;
  const int g = lane >> 4;
  T Ki[4];
#pragma unroll
  for (int m = 0; m < 4; m++) Ki[m] = gp[m * 64];
  const T adet = gp[4 * 64];
  const T *qw = A.tab + NQ * D * 3;
  const T *fwd = qw + NQ + NQ * 3;
  const T *bwd = fwd + NR * NS * 64;
  T xv[NS][2];
#pragma unroll
  for (int s = 0; s < NS; s++) {
    const int i = 4 * s + g;
    const int idx = (valid && i < D) ? mp[i * 64] : -1;
#pragma unroll
    for (int c = 0; c < 2; c++) xv[s][c] = idx >= 0 ? A.x[2 * (int64_t)idx + c] : T(0);
  }
#pragma unroll
  for (int t = 0; t < NT; t++)
#pragma unroll
    for (int c = 0; c < 2; c++) yacc[t][c] = V4{T(0), T(0), T(0), T(0)};
  constexpr int RU = NR <= 4 ? NR : 1;
#pragma unroll RU
  for (int r = 0; r < NR; r++) {
    V4 acc[2];
#pragma unroll
    for (int c = 0; c < 2; c++) acc[c] = V4{T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int s = 0; s < NS; s++) {
      const T av = fwd[(r * NS + s) * 64 + lane];
#pragma unroll
      for (int c = 0; c < 2; c++) acc[c] = MF::fma(av, xv[s][c], acc[c]);
    }
    const int q = 4 * r + g;
    const T wd = q < NQ ? qw[q] * adet : T(0);
    // physical gradients G[c][a] = sum_b g_cb d xi_b / d x_a, stress S, and the pulled
    // back flux w |det| sum_a S[c][a] d xi_d / d x_a
    T G[2][2];
#pragma unroll
    for (int c = 0; c < 2; c++)
#pragma unroll
      for (int a = 0; a < 2; a++) G[c][a] = acc[c][0] * Ki[a] + acc[c][1] * Ki[2 + a];
    const T tr = A.lam * (G[0][0] + G[1][1]), od = A.mu * (G[0][1] + G[1][0]);
    const T S[2][2] = {{tr + T(2) * A.mu * G[0][0], od}, {od, tr + T(2) * A.mu * G[1][1]}};
#pragma unroll
    for (int t = 0; t < NT; t++) {
      const T *bt = bwd + (t * NR + r) * 3 * 64 + lane;
#pragma unroll
      for (int d = 0; d < 2; d++) {
        const T av = bt[d * 64];
#pragma unroll
        for (int c = 0; c < 2; c++)
          yacc[t][c] = MF::fma(av, wd * (S[c][0] * Ki[2 * d] + S[c][1] * Ki[2 * d + 1]), yacc[t][c]);
      }
    }
  }
}

template <typename T, int K, int NQ, bool ATOMIC>
__global__ void __launch_bounds__(64) tri_elasticity_mfma_kernel(const TetArgs<T> A) {
  using V4 = typename Mfma16<T>::V;
  constexpr int D = simplex_nodes<2, K>(), NT = (D + 15) / 16;
  constexpr bool F64 = sizeof(T) == 8;
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
  V4 yacc[NT][2];
  tri_elas_cells16<T, K, NQ>(A, mp, A.geo + batch * (5 * 64) + cl, valid, lane, yacc);
#pragma unroll
  for (int t = 0; t < NT; t++)
#pragma unroll
    for (int v = 0; v < 4; v++) {
      const int i = F64 ? 16 * t + g + 4 * v : 16 * t + 4 * g + v;
      const int idx = (valid && i < D) ? mp[i * 64] : -1;
      if (idx >= 0) {
#pragma unroll
        for (int c = 0; c < 2; c++) {
          if constexpr (ATOMIC) unsafeAtomicAdd(&A.y[2 * (int64_t)idx + c], yacc[t][c][v]);
          else A.y[2 * (int64_t)idx + c] += yacc[t][c][v];  // cells of one launch share no node
        }
      }
    }
}

// Patch scatter of 2D elasticity (as simplex_scalar_patch_kernel, two components per
// node in the LDS sums; slot geometry d xi / d x and |det J|, 5 entries).
template <typename T, int K, int NQ>
__global__ void __launch_bounds__(256) tri_elasticity_patch_kernel(const TetArgs<T> A, const SimplexPatchArgs<T> P) {
  using V4 = typename Mfma16<T>::V;
  constexpr int D = simplex_nodes<2, K>(), NT = (D + 15) / 16;
  constexpr bool F64 = sizeof(T) == 8;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double *acc = reinterpret_cast<double *>(smem_raw);
  const int64_t p = xcd_batch(blockIdx.x, P.npatch);
  if (p >= P.npatch) return;  // whole workgroup: no barrier skipped
  const int n0 = P.nptr[p], nn = P.nptr[p + 1] - n0;
  for (int e = threadIdx.x; e < 2 * nn; e += blockDim.x) acc[e] = 0.0;
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j = lane & 15, g = lane >> 4, cl = 16 * w + j;
  const int nblk = P.cap / 64;
  for (int r = 0; r < nblk; r++) {
    const int64_t blk = p * nblk + r;
    V4 yacc[NT][2];
    tri_elas_cells16<T, K, NQ>(A, P.map + blk * (D * 64) + cl, P.geo + blk * (5 * 64) + cl, true, lane, yacc);
    const uint16_t *lp = P.lmap + blk * (D * 64) + cl;
#pragma unroll
    for (int t = 0; t < NT; t++)
#pragma unroll
      for (int v = 0; v < 4; v++) {
        const int i = F64 ? 16 * t + g + 4 * v : 16 * t + 4 * g + v;
        if (i < D) {
          const int l = lp[i * 64];
          if (l != kSlotSkip)
#pragma unroll
            for (int c = 0; c < 2; c++) atomicAdd(&acc[2 * l + c], (double)yacc[t][c][v]);
        }
      }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nn; e += blockDim.x) {
    const int32_t o = P.out[n0 + e];
    if (o & kSharedOut) {
      T *d = P.sbuf + 2 * (int64_t)(o & (kSharedOut - 1));
      d[0] = (T)acc[2 * e];
      d[1] = (T)acc[2 * e + 1];
    } else {
      T *d = A.y + 2 * (int64_t)o;
      d[0] = P.accumulate ? d[0] + (T)acc[2 * e] : (T)acc[2 * e];
      d[1] = P.accumulate ? d[1] + (T)acc[2 * e + 1] : (T)acc[2 * e + 1];
    }
  }
}

template <typename T, int K, int NQ>
static int launch_tri_elasticity_kq(const TetArgs<T> &a, const SimplexPatchArgs<T> *p, bool atomic, hipStream_t s) {
  if (p) {
    if (p->npatch <= 0) return MF_OK;
    const size_t lds = (size_t)p->nmax * 2 * sizeof(double);
    if (lds > 64 * 1024) return fail(MF_EUNSUPPORTED, "triangle patch scatter: patch node list too long for LDS");
    tri_elasticity_patch_kernel<T, K, NQ><<<dim3((unsigned)xcd_grid(p->npatch)), dim3(256), lds, s>>>(a, *p);
  } else {
    const int64_t nqb = 4 * ((a.c1 + 63) / 64 - a.c0 / 64);
    if (a.c1 <= a.c0) return MF_OK;
    const dim3 g((unsigned)(((nqb + 7) / 8) * 8)), b(64);
    if (atomic) tri_elasticity_mfma_kernel<T, K, NQ, true><<<g, b, 0, s>>>(a);
    else tri_elasticity_mfma_kernel<T, K, NQ, false><<<g, b, 0, s>>>(a);
  }
  MF_HIP(hipGetLastError());
  return MF_OK;
}

// rules of degree 2k - 2 (collapsed Gauss, n^2 points, n = k)
template <typename T>
static int launch_tri_elasticity_t(int k, int nq, const TetArgs<T> &a, const SimplexPatchArgs<T> *p, bool atomic,
                                   hipStream_t s) {
#define MF_TRI_EL(K, NQ) \
  if (k == K && nq == NQ) return launch_tri_elasticity_kq<T, K, NQ>(a, p, atomic, s);
  MF_TRI_EL(1, 1) MF_TRI_EL(2, 4) MF_TRI_EL(3, 9) MF_TRI_EL(4, 16) MF_TRI_EL(5, 25) MF_TRI_EL(6, 36)
#undef MF_TRI_EL
  return fail(MF_EUNSUPPORTED, "triangle elasticity on MFMA: degree / rule");
}
template <typename T>
int launch_tri_elasticity_mfma(int k, int nq, const TetArgs<T> &a, bool atomic, hipStream_t s) {
  return launch_tri_elasticity_t<T>(k, nq, a, nullptr, atomic, s);
}
template <typename T>
int launch_tri_elasticity_patches(int k, int nq, const TetArgs<T> &a, const SimplexPatchArgs<T> &p, hipStream_t s) {
  return launch_tri_elasticity_t<T>(k, nq, a, &p, false, s);
}
template int launch_tri_elasticity_mfma<double>(int, int, const TetArgs<double> &, bool, hipStream_t);
template int launch_tri_elasticity_mfma<float>(int, int, const TetArgs<float> &, bool, hipStream_t);
template int launch_tri_elasticity_patches<double>(int, int, const TetArgs<double> &,
                                                   const SimplexPatchArgs<double> &, hipStream_t);
template int launch_tri_elasticity_patches<float>(int, int, const TetArgs<float> &, const SimplexPatchArgs<float> &,
                                                  hipStream_t);

template <typename T>
static int launch_tri_scalar_mfma_t(int k, int nq, int kind, const TetArgs<T> &a, const SimplexPatchArgs<T> *p,
                                    bool atomic, hipStream_t s) {
#define MF_TRI_KQ(K, NQ) \
  if (k == K && nq == NQ) return launch_simplex_scalar_k<T, 2, K, NQ>(kind, a, p, atomic, s);
  MF_TRI_KQ(1, 1) MF_TRI_KQ(1, 4) MF_TRI_KQ(1, 9)
  MF_TRI_KQ(2, 4) MF_TRI_KQ(2, 9) MF_TRI_KQ(2, 16)
  MF_TRI_KQ(3, 9) MF_TRI_KQ(3, 16) MF_TRI_KQ(3, 25)
  MF_TRI_KQ(4, 16) MF_TRI_KQ(4, 25) MF_TRI_KQ(4, 36)
  MF_TRI_KQ(5, 25) MF_TRI_KQ(5, 36) MF_TRI_KQ(5, 49)
  MF_TRI_KQ(6, 36) MF_TRI_KQ(6, 49) MF_TRI_KQ(6, 64)
#undef MF_TRI_KQ
  return fail(MF_EUNSUPPORTED, "triangle scalar operator on MFMA: degree / rule");
}

template <typename T>
int launch_tri_scalar_mfma(int k, int nq, int kind, const TetArgs<T> &a, bool atomic, hipStream_t s) {
  return launch_tri_scalar_mfma_t<T>(k, nq, kind, a, nullptr, atomic, s);
}
template <typename T>
int launch_tri_scalar_patches(int k, int nq, int kind, const TetArgs<T> &a, const SimplexPatchArgs<T> &p,
                              hipStream_t s) {
  return launch_tri_scalar_mfma_t<T>(k, nq, kind, a, &p, false, s);
}
template int launch_tri_scalar_mfma<double>(int, int, int, const TetArgs<double> &, bool, hipStream_t);
template int launch_tri_scalar_mfma<float>(int, int, int, const TetArgs<float> &, bool, hipStream_t);
template int launch_tri_scalar_patches<double>(int, int, int, const TetArgs<double> &,
                                               const SimplexPatchArgs<double> &, hipStream_t);
template int launch_tri_scalar_patches<float>(int, int, int, const TetArgs<float> &,
                                              const SimplexPatchArgs<float> &, hipStream_t);

}  // namespace mf
