// Operator action on affine simplices.
//
// Affine cells have one Jacobian per cell (Section 2.1: the Jacobian is
// constant on each triangle when the coordinate map is affine; Section 4.1:
// tri and tet meshes use an affine map), so the FP64 setup precomputes
// J^{-1} and |det J| per cell once. Simplices are not sum-factorised
// (Section 4.2.3): the kernels contract dense tabulations of the reference
// basis gradients at quadrature points, the paper's constant tables.
//
// Layouts follow the paper's cross-element idea (Section 3.1: element index
// fastest in every temporary): AoSoA [cell/64][entry][cell%64] maps, geometry and
// coefficients, so a wavefront's loads of one entry are unit-stride. Over a batch
// of cells both contractions are GEMMs with the tabulation shared by every cell,
// so the tet kernels of degree >= 2 (and every one-component form) run them on the
// matrix cores, 16 cells per wavefront (simplex_mfma.h); P1 elasticity keeps one
// lane per cell. Here: tet elasticity and the hyperelastic tangent, the scalar tet
// dispatch, the closed-form P1 triangle mass, the patch scatter's shared-node sum.
#include <type_traits>

#include "simplex_mfma.h"

namespace mf {

__device__ __forceinline__ void atomic_add_s(double *p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add_s(float *p, float v) { unsafeAtomicAdd(p, v); }

// ----------------------------------------------------------------- tet linear elasticity
// a(u, v) = int sigma(u) : grad v, sigma = lambda tr(grad u) I + mu (grad u + grad u^T)
// (supplementary material, "elasticity", with Lame parameters).
// Block = 3 wavefronts; wavefront c carries displacement component c of the same 64
// cells, so each lane keeps only that component's D nodal values (and D outputs) in
// registers. The three components meet once per quadrature point through LDS to form
// the stress.
template <typename T, int K, int NQ, bool ATOMIC>
__global__ void __launch_bounds__(192) tet_elasticity_kernel(const TetArgs<T> A) {
  constexpr int D = (K + 1) * (K + 2) * (K + 3) / 6;
  __shared__ T sG[2][9][64];
  const int lane = threadIdx.x & 63, c = threadIdx.x >> 6;
  // XCD-aware: workgroup w runs on XCD w % 8; each XCD takes a contiguous range of batches
  const int64_t nbt = (A.c1 + 63) / 64 - A.c0 / 64, per = (nbt + 7) / 8;
  const int64_t bl = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (bl >= nbt) return;
  const int64_t batch = A.c0 / 64 + bl;
  const int64_t cell = batch * 64 + lane;
  bool valid = cell >= A.c0 && cell < A.c1;
  if (valid && A.cell_user) {
    const int64_t u = A.cell_user[cell];
    valid = u >= A.ulo && u < A.uhi;
  }
  const int32_t *mp = A.map + batch * (D * 64) + lane;
  const T *gp = A.geo + batch * (10 * 64) + lane;
  T Ki[9];
#pragma unroll
  for (int m = 0; m < 9; m++) Ki[m] = gp[m * 64];
  const T adet = gp[9 * 64];
  T xe[D], ye[D];
#pragma unroll
  for (int i = 0; i < D; i++) {
    const int idx = valid ? mp[i * 64] : -1;
    xe[i] = idx >= 0 ? A.x[3 * (int64_t)idx + c] : T(0);
    ye[i] = T(0);
  }
  const T *__restrict__ dphi = A.tab;
  const T *__restrict__ qw = A.tab + NQ * D * 3;
  for (int q = 0; q < NQ; q++) {
    const T *tq = dphi + q * D * 3;
    T g0 = T(0), g1 = T(0), g2 = T(0);
#pragma unroll
    for (int i = 0; i < D; i++) {
      g0 += xe[i] * tq[3 * i + 0];
      g1 += xe[i] * tq[3 * i + 1];
      g2 += xe[i] * tq[3 * i + 2];
    }
    const int buf = q & 1;
#pragma unroll
    for (int a = 0; a < 3; a++) sG[buf][3 * c + a][lane] = g0 * Ki[a] + g1 * Ki[3 + a] + g2 * Ki[6 + a];
    __syncthreads();
    // row c and column c of the displacement gradient (c is uniform per wavefront)
    const T tr = sG[buf][0][lane] + sG[buf][4][lane] + sG[buf][8][lane];
    T sig[3];
#pragma unroll
    for (int a = 0; a < 3; a++)
      sig[a] = A.mu * (sG[buf][3 * c + a][lane] + sG[buf][3 * a + c][lane]) + (a == c ? A.lam * tr : T(0));
    const T wd = qw[q] * adet;
    T P[3];
#pragma unroll
    for (int d = 0; d < 3; d++) P[d] = wd * (sig[0] * Ki[3 * d + 0] + sig[1] * Ki[3 * d + 1] + sig[2] * Ki[3 * d + 2]);
#pragma unroll
    for (int i = 0; i < D; i++) ye[i] += P[0] * tq[3 * i + 0] + P[1] * tq[3 * i + 1] + P[2] * tq[3 * i + 2];
  }
#pragma unroll
  for (int i = 0; i < D; i++) {
    const int idx = valid ? mp[i * 64] : -1;
    if (idx >= 0) {
      if constexpr (ATOMIC) atomic_add_s(&A.y[3 * (int64_t)idx + c], ye[i]);
      else A.y[3 * (int64_t)idx + c] += ye[i];  // cells of one launch share no node
    }
  }
}

// ----------------------------------------------------------------- scalar tet operators
// MASS int c u v, HELMHOLTZ int grad u . grad v + u v, LAPLACIAN int grad u . grad v,
// POISSON int kappa grad u . grad v on affine tets (supplementary operator list), with
// the vertex coefficient interpolated by the vertex basis; dense tabulation (simplices
// are not sum-factorised), both contractions on MFMA (tet_scalar_cells16 below).
template <typename T>
static int launch_tet_scalar_mfma(int k, int nq, int kind, const TetArgs<T> &a, const SimplexPatchArgs<T> *p,
                                  bool atomic, hipStream_t s);

// every degree runs on MFMA (the tables carry the per-lane operands after the vertex
// basis)
template <typename T>
int launch_tet_scalar(int k, int nq, int kind, const TetArgs<T> &a, bool atomic, hipStream_t s) {
  return launch_tet_scalar_mfma<T>(k, nq, kind, a, nullptr, atomic, s);
}
template int launch_tet_scalar<double>(int, int, int, const TetArgs<double> &, bool, hipStream_t);
template int launch_tet_scalar<float>(int, int, int, const TetArgs<float> &, bool, hipStream_t);

// ----------------------------------------------------------------- tet elasticity on MFMA
// Both contractions of the action are GEMMs over a batch of cells (the
// tabulation of the reference gradients is shared by all cells):
//   forward  G[(q,a)][(cell,c)] = sum_i dphi[q][i][a] x[i][(cell,c)]
//   backward y[i][(cell,c)]     = sum_(q,a) dphi[q][i][a] P[(q,a)][(cell,c)]
// computed with v_mfma_f32_16x16x4f32 / v_mfma_f64_16x16x4f64 (degree >= 2;
// operands: A[m][k] from lane m + 16 k, B[k][n] from lane n + 16 k; result
// C[m][n] in lane n + 16 (m / 4), element m % 4 for FP32, and in lane
// n + 16 (m % 4), element m / 4 for FP64 -- measured on gfx950).
// A wavefront owns 16 cells (n = cell) and one accumulator per displacement
// component. The forward rows are ordered so that the row of (q = 4 r + g, a)
// lands in lane group g, element a (a = 3 is padding), so lane (cell, g) ends up
// with the full reference gradient of all three components at one point, forms
// the stress there, and its P values are exactly the B operand of the backward
// K-steps (r, a) whose 4 entries are the points q = 4 r + 0..3. The per-lane
// operands of the tabulation are precomputed on the host (mfma_tab layout:
// fwd[r][s][64], bwd[t][r][a][64]).
// (Mfma16: the MFMA wrappers of simplex_mfma.h)

// One wavefront per 16 cells (a quarter of a 64-cell layout block); a workgroup holds
// blockDim.x / 64 consecutive quarters (1 or 4; the wavefronts share nothing but cache
// lines). A colour of the 48^3 x 6 workload holds about 21,000 cells: 4-wavefront groups
// give about 335 workgroups for 256 CUs, one-wavefront groups about 1,300, which spread
// more evenly (P2: 362 -> 327 us in FP64); P3 in FP64 (two wavefronts per SIMD) runs
// faster with the four quarters of a layout block on one CU (737 against 832 us).
// HYPER: the St-Venant-Kirchhoff tangent at A.u0 instead of linear elasticity: the
// gradient of u0 at each point comes from the same forward contraction, and the flux
// is dF S + F dS (F = I + grad u0, E = (F^T F - I)/2, S = lambda tr(E) I + 2 mu E,
// dF = grad u, dE = (dF^T F + F^T dF)/2, dS = lambda tr(dE) I + 2 mu dE).
// The action of one wavefront's 16 cells (cell j = lane % 16 of quarter w of a 64-cell
// layout block whose map and geometry entries start at mp and gp, already offset to
// the lane's cell): yacc[t][c][v] is the local result of component c at node
// i = 16 t + 4 g + v (FP32) or 16 t + g + 4 v (FP64), g = lane / 16.
template <typename T, int K, int NQ, bool HYPER>
__device__ __forceinline__ void tet_elas_cells16(
    const TetArgs<T> &A, const int32_t *mp, const T *gp, const bool valid, const int lane,
    typename Mfma16<T>::V (&yacc)[((K + 1) * (K + 2) * (K + 3) / 6 + 15) / 16][3]) {
  using MF = Mfma16<T>;
  using V4 = typename MF::V;
  constexpr int D = (K + 1) * (K + 2) * (K + 3) / 6;
  constexpr int NR = (NQ + 3) / 4, NS = (D + 3) / 4, NT = (D + 15) / 16;
  const int g = lane >> 4;
  T Ki[9];
#pragma unroll
  for (int m = 0; m < 9; m++) Ki[m] = gp[m * 64];
  const T adet = gp[9 * 64];
  const T *qw = A.tab + NQ * D * 3;
  const T *fwd = qw + NQ;
  const T *bwd = fwd + NR * NS * 64;
  // nodal values: lane (cell, g) holds the nodes i = 4 s + g, all three components
  T xv[NS][3];
#pragma unroll
  for (int s = 0; s < NS; s++) {
    const int i = 4 * s + g;
    const int idx = (valid && i < D) ? mp[i * 64] : -1;
#pragma unroll
    for (int c = 0; c < 3; c++) xv[s][c] = idx >= 0 ? A.x[3 * (int64_t)idx + c] : T(0);
  }
  // the linearisation point at the same nodes (through the unflagged map if constrained)
  T u0v[HYPER ? NS : 1][3];
  if constexpr (HYPER) {
    const int32_t *mq = A.u0map ? A.u0map + (mp - A.map) : mp;
#pragma unroll
    for (int s = 0; s < NS; s++) {
      const int i = 4 * s + g;
      const int idx = (valid && i < D) ? mq[i * 64] : -1;
#pragma unroll
      for (int c = 0; c < 3; c++) u0v[s][c] = idx >= 0 ? A.u0[3 * (int64_t)idx + c] : T(0);
    }
  }
#pragma unroll
  for (int t = 0; t < NT; t++)
#pragma unroll
    for (int c = 0; c < 3; c++) yacc[t][c] = V4{T(0), T(0), T(0), T(0)};
  // point groups: unrolled up to the 14-point rule; the 125-point rule keeps the loop
  constexpr int RU = NR <= 4 ? NR : 1;
#pragma unroll RU
  for (int r = 0; r < NR; r++) {
    V4 gacc[3], g0acc[HYPER ? 3 : 1];
#pragma unroll
    for (int c = 0; c < 3; c++) gacc[c] = V4{T(0), T(0), T(0), T(0)};
    if constexpr (HYPER)
#pragma unroll
      for (int c = 0; c < 3; c++) g0acc[c] = V4{T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int s = 0; s < NS; s++) {
      const T av = fwd[(r * NS + s) * 64 + lane];
#pragma unroll
      for (int c = 0; c < 3; c++) gacc[c] = MF::fma(av, xv[s][c], gacc[c]);
      if constexpr (HYPER)
#pragma unroll
        for (int c = 0; c < 3; c++) g0acc[c] = MF::fma(av, u0v[s][c], g0acc[c]);
    }
    // point q = 4 r + g of this lane's cell: reference gradients gacc[c][a]
    const int q = 4 * r + g;
    const T wd = q < NQ ? qw[q] * adet : T(0);
    T gr[3][3];
#pragma unroll
    for (int c = 0; c < 3; c++)
#pragma unroll
      for (int a = 0; a < 3; a++) gr[c][a] = gacc[c][0] * Ki[a] + gacc[c][1] * Ki[3 + a] + gacc[c][2] * Ki[6 + a];
    // flux f[c][a] against d v_c / d x_a
    T f[3][3];
    if constexpr (HYPER) {
      T F[3][3], S[3][3], M[3][3];
#pragma unroll
      for (int c = 0; c < 3; c++)
#pragma unroll
        for (int a = 0; a < 3; a++)
          F[c][a] = (c == a ? T(1) : T(0)) + g0acc[c][0] * Ki[a] + g0acc[c][1] * Ki[3 + a] + g0acc[c][2] * Ki[6 + a];
      // S from E = (F^T F - I)/2; M = F^T dF, so dE = (M + M^T)/2
      T trE = T(0);
#pragma unroll
      for (int i = 0; i < 3; i++)
#pragma unroll
        for (int jj = 0; jj < 3; jj++) {
          T cc = T(0), mm = T(0);
#pragma unroll
          for (int k = 0; k < 3; k++) {
            cc += F[k][i] * F[k][jj];
            mm += F[k][i] * gr[k][jj];
          }
          const T e = T(0.5) * (cc - (i == jj ? T(1) : T(0)));
          if (i == jj) trE += e;
          S[i][jj] = T(2) * A.mu * e;
          M[i][jj] = mm;
        }
      const T trM = M[0][0] + M[1][1] + M[2][2];
#pragma unroll
      for (int i = 0; i < 3; i++) S[i][i] += A.lam * trE;
#pragma unroll
      for (int i = 0; i < 3; i++)
#pragma unroll
        for (int a = 0; a < 3; a++) {
          T v = T(0);
#pragma unroll
          for (int k = 0; k < 3; k++) {
            const T dS = A.mu * (M[k][a] + M[a][k]) + (k == a ? A.lam * trM : T(0));
            v += gr[i][k] * S[k][a] + F[i][k] * dS;
          }
          f[i][a] = v;
        }
    } else {
      const T tr = gr[0][0] + gr[1][1] + gr[2][2];
#pragma unroll
      for (int c = 0; c < 3; c++)
#pragma unroll
        for (int a = 0; a < 3; a++) f[c][a] = A.mu * (gr[c][a] + gr[a][c]) + (a == c ? A.lam * tr : T(0));
    }
    T P[3][3];
#pragma unroll
    for (int c = 0; c < 3; c++)
#pragma unroll
      for (int d = 0; d < 3; d++) P[c][d] = wd * (f[c][0] * Ki[3 * d + 0] + f[c][1] * Ki[3 * d + 1] + f[c][2] * Ki[3 * d + 2]);
#pragma unroll
    for (int t = 0; t < NT; t++)
#pragma unroll
      for (int d = 0; d < 3; d++) {
        const T av = bwd[((t * NR + r) * 3 + d) * 64 + lane];
#pragma unroll
        for (int c = 0; c < 3; c++) yacc[t][c] = MF::fma(av, P[c][d], yacc[t][c]);
      }
  }
}

template <typename T, int K, int NQ, bool ATOMIC, bool HYPER = false>
__global__ void __launch_bounds__(256) tet_elasticity_mfma_kernel(const TetArgs<T> A) {
  using V4 = typename Mfma16<T>::V;
  constexpr int D = (K + 1) * (K + 2) * (K + 3) / 6;
  constexpr int NT = (D + 15) / 16;
  const int lane = threadIdx.x & 63, wpg = blockDim.x >> 6;
  const int j = lane & 15, g = lane >> 4;
  // workgroup units of wpg quarters; contiguous ranges of units per XCD
  const int64_t nqb = 4 * ((A.c1 + 63) / 64 - A.c0 / 64), nbu = (nqb + wpg - 1) / wpg, per = (nbu + 7) / 8;
  const int64_t bu = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  const int64_t qb = bu * wpg + (threadIdx.x >> 6);
  if (bu >= nbu || qb >= nqb) return;  // no barriers: wavefronts may leave on their own
  const int64_t batch = A.c0 / 64 + qb / 4;
  const int w = (int)(qb % 4);
  const int cl = 16 * w + j;
  const int64_t cell = batch * 64 + cl;
  bool valid = cell >= A.c0 && cell < A.c1;
  if (valid && A.cell_user) {
    const int64_t u = A.cell_user[cell];
    valid = u >= A.ulo && u < A.uhi;
  }
  const int32_t *mp = A.map + batch * (D * 64) + cl;
  const T *gp = A.geo + batch * (10 * 64) + cl;
  V4 yacc[NT][3];
  tet_elas_cells16<T, K, NQ, HYPER>(A, mp, gp, valid, lane, yacc);
  // lane (cell, g) holds y for the nodes i = 16 t + 4 g + v (FP32), 16 t + g + 4 v (FP64)
  constexpr bool F64 = sizeof(T) == 8;
#pragma unroll
  for (int t = 0; t < NT; t++)
#pragma unroll
    for (int v = 0; v < 4; v++) {
      const int i = F64 ? 16 * t + g + 4 * v : 16 * t + 4 * g + v;
      const int idx = (valid && i < D) ? mp[i * 64] : -1;
      if (idx >= 0) {
#pragma unroll
        for (int c = 0; c < 3; c++) {
          if constexpr (ATOMIC) atomic_add_s(&A.y[3 * (int64_t)idx + c], yacc[t][c][v]);
          else A.y[3 * (int64_t)idx + c] += yacc[t][c][v];  // cells of one launch share no node
        }
      }
    }
}

// Patch scatter (SimplexPatchArgs): one workgroup of four wavefronts per patch; each
// round the wavefronts take the patch's next 64 slots (16 cells each, as above), and
// the local results are summed into the patch's nodes in LDS with LDS atomics. After
// the last round every node of the patch is written once: into y if no other patch
// touches it, else into its slot of sbuf.
template <typename T, int K, int NQ>
__global__ void __launch_bounds__(256) tet_elasticity_patch_kernel(const TetArgs<T> A, const SimplexPatchArgs<T> P) {
  using V4 = typename Mfma16<T>::V;
  constexpr int D = (K + 1) * (K + 2) * (K + 3) / 6;
  constexpr int NT = (D + 15) / 16;
  constexpr bool F64 = sizeof(T) == 8;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // sums in FP64 for both precisions: LDS FP32 atomic adds measured several times
  // slower than FP64 ones here (the FP32 P2 kernel waited on LDS 70x longer)
  double *acc = reinterpret_cast<double *>(smem_raw);
  const int64_t p = xcd_batch(blockIdx.x, P.npatch);  // contiguous patch ranges per XCD
  if (p >= P.npatch) return;                           // whole workgroup: no barrier skipped
  const int n0 = P.nptr[p], nn = P.nptr[p + 1] - n0;
  for (int e = threadIdx.x; e < 3 * nn; e += blockDim.x) acc[e] = 0.0;
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j = lane & 15, g = lane >> 4, cl = 16 * w + j;
  const int nblk = P.cap / 64;
  for (int r = 0; r < nblk; r++) {
    const int64_t blk = p * nblk + r;
    V4 yacc[NT][3];
    tet_elas_cells16<T, K, NQ, false>(A, P.map + blk * (D * 64) + cl, P.geo + blk * (10 * 64) + cl, true, lane,
                                      yacc);
    const uint16_t *lp = P.lmap + blk * (D * 64) + cl;
#pragma unroll
    for (int t = 0; t < NT; t++)
#pragma unroll
      for (int v = 0; v < 4; v++) {
        const int i = F64 ? 16 * t + g + 4 * v : 16 * t + 4 * g + v;
        if (i < D) {
          const int l = lp[i * 64];
          if (l != kSlotSkip) {
#pragma unroll
            for (int c = 0; c < 3; c++) atomicAdd(&acc[3 * l + c], (double)yacc[t][c][v]);
          }
        }
      }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nn; e += blockDim.x) {
    const int32_t o = P.out[n0 + e];
    if (o & kSharedOut) {
      T *d = P.sbuf + 3 * (int64_t)(o & (kSharedOut - 1));
#pragma unroll
      for (int c = 0; c < 3; c++) d[c] = (T)acc[3 * e + c];
    } else {
      T *d = A.y + 3 * (int64_t)o;
#pragma unroll
      for (int c = 0; c < 3; c++) d[c] = P.accumulate ? d[c] + (T)acc[3 * e + c] : (T)acc[3 * e + c];
    }
  }
}

// ----------------------------------------------------------------- scalar tet operators on MFMA
// simplex_scalar_* of simplex_mfma.h with DIM = 3, on the rules of the tet quadrature
// table the scalar kinds take: 1 point (degree 1), 4 (degree 2), 14 (degree 5), and the
// conical Gauss-Jacobi products of n^3 points, exact to degree 2n - 1 (64, 125, 216,
// 343)
template <typename T>
static int launch_tet_scalar_mfma(int k, int nq, int kind, const TetArgs<T> &a, const SimplexPatchArgs<T> *p,
                                  bool atomic, hipStream_t s) {
#define MF_TET_KQ(K, NQ) \
  if (k == K && nq == NQ) return launch_simplex_scalar_k<T, 3, K, NQ>(kind, a, p, atomic, s);
  MF_TET_KQ(1, 1) MF_TET_KQ(1, 4) MF_TET_KQ(1, 14)
  MF_TET_KQ(2, 4) MF_TET_KQ(2, 14)
  MF_TET_KQ(3, 14) MF_TET_KQ(3, 64)
  MF_TET_KQ(4, 64) MF_TET_KQ(4, 125)
  MF_TET_KQ(5, 125) MF_TET_KQ(5, 216)
  MF_TET_KQ(6, 216) MF_TET_KQ(6, 343)
#undef MF_TET_KQ
  return fail(MF_EUNSUPPORTED, "tet scalar operator on MFMA: degree / rule");
}

template <typename T>
int launch_tet_scalar_patches(int k, int nq, int kind, const TetArgs<T> &a, const SimplexPatchArgs<T> &p,
                              hipStream_t s) {
  return launch_tet_scalar_mfma<T>(k, nq, kind, a, &p, false, s);
}
template int launch_tet_scalar_patches<double>(int, int, int, const TetArgs<double> &,
                                               const SimplexPatchArgs<double> &, hipStream_t);
template int launch_tet_scalar_patches<float>(int, int, int, const TetArgs<float> &,
                                              const SimplexPatchArgs<float> &, hipStream_t);

// Per-lane MFMA operands of the one-component forms (simplex_mfma.h): forward rows
// (q, a) with the reference gradient for a < dim and the basis value phi[q][i] for
// a = dim (a = 3 is padding on triangles), and backward K-steps for a = 0..dim.
int simplex_mfma_scalar_table_floats(int dim, int D, int nq) {
  const int NR = (nq + 3) / 4, NS = (D + 3) / 4, NT = (D + 15) / 16;
  return NR * NS * 64 + NT * NR * (dim + 1) * 64;
}

void simplex_mfma_scalar_tables(int dim, int D, int nq, const double *phi, const double *dphi, double *out,
                                bool f64) {
  const int NR = (nq + 3) / 4, NS = (D + 3) / 4, NT = (D + 15) / 16, NB = dim + 1;
  double *fwd = out, *bwd = out + NR * NS * 64;
  auto entry = [&](int q, int i, int a) {
    if (q >= nq || i >= D || a > dim) return 0.0;
    return a < dim ? dphi[(q * D + i) * dim + a] : phi[q * D + i];
  };
  for (int r = 0; r < NR; r++)
    for (int s = 0; s < NS; s++)
      for (int l = 0; l < 64; l++) {
        const int m = l % 16, kk = l / 16;
        const int q = 4 * r + (f64 ? m % 4 : m / 4), a = f64 ? m / 4 : m % 4;
        fwd[(r * NS + s) * 64 + l] = entry(q, 4 * s + kk, a);
      }
  for (int t = 0; t < NT; t++)
    for (int r = 0; r < NR; r++)
      for (int d = 0; d < NB; d++)
        for (int l = 0; l < 64; l++)
          bwd[((t * NR + r) * NB + d) * 64 + l] = entry(4 * r + l / 16, 16 * t + l % 16, d);
}

template <typename T>
__global__ void __launch_bounds__(256) simplex_shared_reduce_kernel(const int32_t *sptr, const int32_t *snode,
                                                                     const T *sbuf, T *y, int64_t n, int nc,
                                                                     int accumulate) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * nc) return;
  const int64_t i = t / nc;
  const int c = (int)(t - i * nc);
  T v = T(0);
  for (int32_t q = sptr[i]; q < sptr[i + 1]; q++) v += sbuf[(int64_t)q * nc + c];
  T *d = y + (int64_t)snode[i] * nc + c;
  *d = accumulate ? *d + v : v;
}

template <typename T>
int launch_simplex_shared_reduce(const int32_t *sptr, const int32_t *snode, const T *sbuf, T *y, int64_t nshared,
                                 int ncomp, bool accumulate, hipStream_t s) {
  if (nshared <= 0) return MF_OK;
  const int64_t n = nshared * ncomp;
  simplex_shared_reduce_kernel<T><<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(
      sptr, snode, sbuf, y, nshared, ncomp, accumulate ? 1 : 0);
  MF_HIP(hipGetLastError());
  return MF_OK;
}
template int launch_simplex_shared_reduce<double>(const int32_t *, const int32_t *, const double *, double *,
                                                  int64_t, int, bool, hipStream_t);
template int launch_simplex_shared_reduce<float>(const int32_t *, const int32_t *, const float *, float *, int64_t,
                                                 int, bool, hipStream_t);

template <typename T, int K, int NQ>
static int launch_tet_patch_kq(const TetArgs<T> &a, const SimplexPatchArgs<T> &p, hipStream_t s) {
  if (p.npatch <= 0) return MF_OK;
  const size_t lds = (size_t)p.nmax * 3 * sizeof(double);
  if (lds > 64 * 1024) return fail(MF_EUNSUPPORTED, "tet patch scatter: patch node list too long for LDS");
  tet_elasticity_patch_kernel<T, K, NQ><<<dim3((unsigned)xcd_grid(p.npatch)), dim3(256), lds, s>>>(a, p);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

template <typename T>
int launch_tet_elasticity_patches(int k, int nq, const TetArgs<T> &a, const SimplexPatchArgs<T> &p,
                                  hipStream_t s) {
  if (k == 2 && nq == 4) return launch_tet_patch_kq<T, 2, 4>(a, p, s);
  if (k == 3 && nq == 14) return launch_tet_patch_kq<T, 3, 14>(a, p, s);
  return fail(MF_EUNSUPPORTED, "tet patch scatter: degree / rule");
}
template int launch_tet_elasticity_patches<double>(int, int, const TetArgs<double> &,
                                                   const SimplexPatchArgs<double> &, hipStream_t);
template int launch_tet_elasticity_patches<float>(int, int, const TetArgs<float> &,
                                                  const SimplexPatchArgs<float> &, hipStream_t);

// Per-lane MFMA operands of the tabulation dphi[q][i][a] (host, for the kernel above).
int tet_mfma_table_floats(int k, int nq) {
  const int D = (k + 1) * (k + 2) * (k + 3) / 6;
  const int NR = (nq + 3) / 4, NS = (D + 3) / 4, NT = (D + 15) / 16;
  return NR * NS * 64 + NT * NR * 3 * 64;
}

void tet_mfma_tables(int k, int nq, const double *dphi, double *out, bool f64) {
  const int D = (k + 1) * (k + 2) * (k + 3) / 6;
  const int NR = (nq + 3) / 4, NS = (D + 3) / 4, NT = (D + 15) / 16;
  double *fwd = out, *bwd = out + NR * NS * 64;
  for (int r = 0; r < NR; r++)
    for (int s = 0; s < NS; s++)
      for (int l = 0; l < 64; l++) {
        const int m = l % 16, kk = l / 16, i = 4 * s + kk;
        const int q = 4 * r + (f64 ? m % 4 : m / 4), a = f64 ? m / 4 : m % 4;
        fwd[(r * NS + s) * 64 + l] = (a < 3 && q < nq && i < D) ? dphi[(q * D + i) * 3 + a] : 0.0;
      }
  for (int t = 0; t < NT; t++)
    for (int r = 0; r < NR; r++)
      for (int d = 0; d < 3; d++)
        for (int l = 0; l < 64; l++) {
          const int i = 16 * t + l % 16, q = 4 * r + l / 16;
          bwd[((t * NR + r) * 3 + d) * 64 + l] = (i < D && q < nq) ? dphi[(q * D + i) * 3 + d] : 0.0;
        }
}

// diag[(i,c)] = sum_q w |det| [ lambda (d_c phi_i)^2 + mu (|grad phi_i|^2 + (d_c phi_i)^2) ]
template <typename T, int K, int NQ>
__global__ void __launch_bounds__(192) tet_elasticity_diag_kernel(const TetArgs<T> A) {
  constexpr int D = (K + 1) * (K + 2) * (K + 3) / 6;
  const int lane = threadIdx.x & 63, c = threadIdx.x >> 6;
  const int64_t batch = A.c0 / 64 + blockIdx.x;
  const int64_t cell = batch * 64 + lane;
  const bool valid = cell >= A.c0 && cell < A.c1;
  const int32_t *mp = A.map + batch * (D * 64) + lane;
  const T *gp = A.geo + batch * (10 * 64) + lane;
  T Ki[9];
  for (int m = 0; m < 9; m++) Ki[m] = gp[m * 64];
  const T adet = gp[9 * 64];
  const T *dphi = A.tab;
  const T *qw = A.tab + NQ * D * 3;
  for (int i = 0; i < D; i++) {
    T acc = T(0);
    for (int q = 0; q < NQ; q++) {
      const T *tq = dphi + (q * D + i) * 3;
      T gr[3];
      for (int a = 0; a < 3; a++) gr[a] = tq[0] * Ki[a] + tq[1] * Ki[3 + a] + tq[2] * Ki[6 + a];
      const T n2 = gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2];
      const T gc = c == 0 ? gr[0] : (c == 1 ? gr[1] : gr[2]);
      acc += qw[q] * adet * (A.lam * gc * gc + A.mu * (n2 + gc * gc));
    }
    const int idx = valid ? mp[i * 64] : -1;
    if (idx >= 0) atomic_add_s(&A.y[3 * (int64_t)idx + c], acc);
  }
}

template <typename T, int K, int NQ>
static int launch_tet_kq(const TetArgs<T> &a, hipStream_t s, bool diag, bool atomic) {
  const int64_t b0 = a.c0 / 64, b1 = (a.c1 + 63) / 64;
  if (a.c1 <= a.c0) return MF_OK;
  dim3 grid((unsigned)(diag ? b1 - b0 : ((b1 - b0 + 7) / 8) * 8)), block(192);
  if constexpr (K >= 2) {
    if (!diag) {
      const int wpg = (K == 3 && sizeof(T) == 8) ? 4 : 1;  // wavefronts (16 cells each) per group
      const int64_t nbu = (4 * (b1 - b0) + wpg - 1) / wpg;
      const dim3 gq((unsigned)(((nbu + 7) / 8) * 8)), bq(64 * wpg);
      if (atomic) tet_elasticity_mfma_kernel<T, K, NQ, true><<<gq, bq, 0, s>>>(a);
      else tet_elasticity_mfma_kernel<T, K, NQ, false><<<gq, bq, 0, s>>>(a);
      MF_HIP(hipGetLastError());
      return MF_OK;
    }
  }
  if constexpr (K <= 3) {
    if (diag) tet_elasticity_diag_kernel<T, K, NQ><<<grid, block, 0, s>>>(a);
    else if (atomic) tet_elasticity_kernel<T, K, NQ, true><<<grid, block, 0, s>>>(a);
    else tet_elasticity_kernel<T, K, NQ, false><<<grid, block, 0, s>>>(a);
    MF_HIP(hipGetLastError());
    return MF_OK;
  }
  return fail(MF_EUNSUPPORTED, "tet elasticity: fused diagonal for degrees 1-3 only");
}

template <typename T>
static int launch_tet(int k, int nq, const TetArgs<T> &a, hipStream_t s, bool diag, bool atomic) {
  if (k == 1 && nq == 1) return launch_tet_kq<T, 1, 1>(a, s, diag, atomic);
  if (k == 2 && nq == 4) return launch_tet_kq<T, 2, 4>(a, s, diag, atomic);
  if (k == 3 && nq == 14) return launch_tet_kq<T, 3, 14>(a, s, diag, atomic);
  if (!diag) {  // degrees 4-6 (rules of degree 2k - 2): the MFMA kernel; their diagonal is element-wise
    if (k == 4 && nq == 64) return launch_tet_kq<T, 4, 64>(a, s, false, atomic);
    if (k == 5 && nq == 125) return launch_tet_kq<T, 5, 125>(a, s, false, atomic);
    if (k == 6 && nq == 216) return launch_tet_kq<T, 6, 216>(a, s, false, atomic);
  }
  return fail(MF_EUNSUPPORTED, "tet elasticity: degree / rule");
}

// St-Venant-Kirchhoff tangent: the MFMA kernel with HYPER for P1 (one point), P2
// (14 points, exact for the degree 4 integrand) and P3 (the 125-point conical rule,
// exact to degree 9, for the degree 8 integrand); one wavefront per workgroup.
template <typename T, int K, int NQ>
static int launch_tet_hyper_kq(const TetArgs<T> &a, bool atomic, hipStream_t s) {
  const int64_t b0 = a.c0 / 64, b1 = (a.c1 + 63) / 64;
  if (a.c1 <= a.c0) return MF_OK;
  const dim3 gq((unsigned)(((4 * (b1 - b0) + 7) / 8) * 8)), bq(64);
  if (atomic) tet_elasticity_mfma_kernel<T, K, NQ, true, true><<<gq, bq, 0, s>>>(a);
  else tet_elasticity_mfma_kernel<T, K, NQ, false, true><<<gq, bq, 0, s>>>(a);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

template <typename T> int launch_tet_elasticity(int k, int nq, const TetArgs<T> &a, bool atomic, hipStream_t s) {
  if (a.u0) {
    if (k == 1 && nq == 1) return launch_tet_hyper_kq<T, 1, 1>(a, atomic, s);
    if (k == 2 && nq == 14) return launch_tet_hyper_kq<T, 2, 14>(a, atomic, s);
    if (k == 3 && nq == 125) return launch_tet_hyper_kq<T, 3, 125>(a, atomic, s);
    if (k == 4 && nq == 343) return launch_tet_hyper_kq<T, 4, 343>(a, atomic, s);
    if (k == 5 && nq == 729) return launch_tet_hyper_kq<T, 5, 729>(a, atomic, s);
    if (k == 6 && nq == 1331) return launch_tet_hyper_kq<T, 6, 1331>(a, atomic, s);
    return fail(MF_EUNSUPPORTED, "tet hyperelasticity: degree / rule");
  }
  return launch_tet<T>(k, nq, a, s, false, atomic);
}
template <typename T> int launch_tet_elasticity_diag(int k, int nq, const TetArgs<T> &a, hipStream_t s) {
  return launch_tet<T>(k, nq, a, s, true, true);
}
template int launch_tet_elasticity<double>(int, int, const TetArgs<double> &, bool, hipStream_t);
template int launch_tet_elasticity<float>(int, int, const TetArgs<float> &, bool, hipStream_t);
template int launch_tet_elasticity_diag<double>(int, int, const TetArgs<double> &, hipStream_t);
template int launch_tet_elasticity_diag<float>(int, int, const TetArgs<float> &, hipStream_t);

// ----------------------------------------------------------------- tri P1 mass with P1 coefficient
// Exact element matrix: int_T lam_a lam_i lam_j = |T| (1 + d_ai + d_aj + d_ij + 2 d_ai d_aj) / 60,
// so with s_a = |T| c_a, S = sum s_a, X = sum x_j:
//   y_i = [ (S + s_i) X + <s, x> + (S + 2 s_i) x_i ] / 60.
template <typename T>
__global__ void __launch_bounds__(256) tri_mass_kernel(const TriArgs<T> A, bool diag, bool atomic) {
  const int64_t cell = A.c0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= A.c1) return;
  if (A.cell_user) {
    const int64_t u = A.cell_user[cell];
    if (u < A.ulo || u >= A.uhi) return;
  }
  int idx[3];
  T s[3], x[3];
#pragma unroll
  for (int i = 0; i < 3; i++) {
    idx[i] = A.map[cell * 3 + i];
    s[i] = A.geo[cell * 4 + i];
    x[i] = (!diag && idx[i] >= 0) ? A.x[idx[i]] : T(0);
  }
  const T S = s[0] + s[1] + s[2];
  const T X = x[0] + x[1] + x[2];
  const T sx = s[0] * x[0] + s[1] * x[1] + s[2] * x[2];
  const T k60 = T(1) / T(60);
#pragma unroll
  for (int i = 0; i < 3; i++) {
    const T v = diag ? (T(2) * S + T(4) * s[i]) * k60 : ((S + s[i]) * X + sx + (S + T(2) * s[i]) * x[i]) * k60;
    if (idx[i] >= 0) {
      if (atomic) atomic_add_s(&A.y[idx[i]], v);
      else A.y[idx[i]] += v;  // cells of one launch share no node
    }
  }
}

// Patch scatter of the P1 mass (SimplexPatchArgs, geometry s_a = |T| c_a per slot):
// a workgroup of 256 threads per patch, a thread per slot in turn, node sums in LDS.
template <typename T>
__global__ void __launch_bounds__(256) tri_mass_patch_kernel(const T *__restrict__ x, T *__restrict__ y,
                                                             const SimplexPatchArgs<T> P) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double *acc = reinterpret_cast<double *>(smem_raw);  // FP64 sums, as in the tet patch kernel
  const int64_t p = xcd_batch(blockIdx.x, P.npatch);
  if (p >= P.npatch) return;
  const int n0 = P.nptr[p], nn = P.nptr[p + 1] - n0;
  for (int e = threadIdx.x; e < nn; e += blockDim.x) acc[e] = 0.0;
  __syncthreads();
  const T k60 = T(1) / T(60);
  for (int sl = threadIdx.x; sl < P.cap; sl += blockDim.x) {
    const int64_t q = p * P.cap + sl, b = q / 64, l = q % 64;
    int idx[3], li[3];
    T sa[3], xv[3];
#pragma unroll
    for (int i = 0; i < 3; i++) {
      idx[i] = P.map[(b * 3 + i) * 64 + l];
      li[i] = P.lmap[(b * 3 + i) * 64 + l];
      sa[i] = P.geo[(b * 3 + i) * 64 + l];
      xv[i] = idx[i] >= 0 ? x[idx[i]] : T(0);
    }
    const T S = sa[0] + sa[1] + sa[2];
    const T X = xv[0] + xv[1] + xv[2];
    const T sx = sa[0] * xv[0] + sa[1] * xv[1] + sa[2] * xv[2];
#pragma unroll
    for (int i = 0; i < 3; i++)
      if (li[i] != kSlotSkip) atomicAdd(&acc[li[i]], (double)(((S + sa[i]) * X + sx + (S + T(2) * sa[i]) * xv[i]) * k60));
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nn; e += blockDim.x) {
    const int32_t o = P.out[n0 + e];
    if (o & kSharedOut) P.sbuf[o & (kSharedOut - 1)] = (T)acc[e];
    else y[o] = P.accumulate ? y[o] + (T)acc[e] : (T)acc[e];
  }
}

template <typename T> int launch_tri_mass_patches(const T *x, T *y, const SimplexPatchArgs<T> &p, hipStream_t s) {
  if (p.npatch <= 0) return MF_OK;
  const size_t lds = (size_t)p.nmax * sizeof(double);
  if (lds > 64 * 1024) return fail(MF_EUNSUPPORTED, "triangle patch scatter: patch node list too long for LDS");
  tri_mass_patch_kernel<T><<<dim3((unsigned)xcd_grid(p.npatch)), dim3(256), lds, s>>>(x, y, p);
  MF_HIP(hipGetLastError());
  return MF_OK;
}
template int launch_tri_mass_patches<double>(const double *, double *, const SimplexPatchArgs<double> &, hipStream_t);
template int launch_tri_mass_patches<float>(const float *, float *, const SimplexPatchArgs<float> &, hipStream_t);

template <typename T> static int launch_tri(const TriArgs<T> &a, hipStream_t s, bool diag, bool atomic) {
  const int64_t n = a.c1 - a.c0;
  if (n <= 0) return MF_OK;
  tri_mass_kernel<T><<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(a, diag, atomic);
  MF_HIP(hipGetLastError());
  return MF_OK;
}
template <typename T> int launch_tri_mass(const TriArgs<T> &a, bool atomic, hipStream_t s) {
  return launch_tri<T>(a, s, false, atomic);
}
template <typename T> int launch_tri_mass_diag(const TriArgs<T> &a, hipStream_t s) { return launch_tri<T>(a, s, true, true); }
template int launch_tri_mass<double>(const TriArgs<double> &, bool, hipStream_t);
template int launch_tri_mass<float>(const TriArgs<float> &, bool, hipStream_t);
template int launch_tri_mass_diag<double>(const TriArgs<double> &, hipStream_t);
template int launch_tri_mass_diag<float>(const TriArgs<float> &, hipStream_t);

}  // namespace mf
