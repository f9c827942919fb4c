// Operators on simplices of degree 4-6 (triangles and tetrahedra; mass with a vertex
// coefficient, Helmholtz, Laplacian with one or dim components, Poisson, elasticity):
// the paper's local kernel by dense tabulation (Section 2.1: the basis and its
// reference gradients tabulated at the quadrature points, the affine Jacobian per
// cell; simplices are not sum-factorised, Section 4), for element sizes where a lane
// per cell would need more registers than a lane has.
//
// A workgroup takes CB consecutive cells. (0) A thread per (cell, node, component)
// gathers x into LDS. (A) A thread per (cell, quadrature point) contracts the cell's
// values with the tabulated basis (tables transposed, [node][point], so neighbouring
// threads read neighbouring entries), forms the physical gradient with the cell's
// J^{-1}, applies the pointwise operator and stores the value flux and the reference
// flux of each component in LDS. (B) A thread per (cell, node) contracts the fluxes with
// the tabulated test functions ([point][node]) and scatters (atomic or, within a colour,
// plain read-modify-write).
#include "mf_internal.h"

namespace mf {

namespace {
__device__ __forceinline__ void sd_atomic_add(double *p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void sd_atomic_add(float *p, float v) { unsafeAtomicAdd(p, v); }
}  // namespace

template <typename T, int DIM>
__global__ void __launch_bounds__(256) simplex_dense_kernel(const SimplexDenseArgs<T> A, const bool atomic) {
  constexpr int G = DIM * DIM + 1, NV = DIM + 1, NF = 1 + DIM;
  const int D = A.D, NQ = A.nq, nc = A.ncomp, CB = A.cb;
  extern __shared__ __align__(16) unsigned char sd_lds[];
  T *xs = reinterpret_cast<T *>(sd_lds);  // [CB][D][nc]
  T *fq = xs + CB * D * nc;               // [CB][NQ][nc][1 + DIM]
  // tables: vT [D][NQ], gT [DIM][D][NQ], v [NQ][D], g [NQ][DIM][D], w [NQ], vb [NQ][NV]
  const T *vT = A.tab, *gT = vT + D * NQ, *v = gT + DIM * D * NQ, *g = v + NQ * D, *w = g + NQ * DIM * D,
          *vb = w + NQ;
  const int64_t first = A.c0 + (int64_t)blockIdx.x * CB;
  auto cell_ok = [&](int s) -> bool {
    const int64_t K = first + s;
    if (K >= A.c1) return false;
    if (!A.cell_user) return true;
    const int64_t u = A.cell_user[K];
    return u >= A.ulo && u < A.uhi;
  };
  auto node_of = [&](int64_t K, int i) { return A.map[((K / 64) * D + i) * 64 + K % 64]; };
  // (0) gather
  for (int e = threadIdx.x; e < CB * D * nc; e += blockDim.x) {
    const int s = e / (D * nc), r = e - s * D * nc, i = r / nc, c = r - i * nc;
    T val = T(0);
    if (cell_ok(s)) {
      const int32_t n = node_of(first + s, i);
      if (n >= 0) val = A.x[(int64_t)n * nc + c];
    }
    xs[e] = val;
  }
  __syncthreads();
  // (A) points
  for (int e = threadIdx.x; e < CB * NQ; e += blockDim.x) {
    const int s = e / NQ, q = e - s * NQ;
    T *f = fq + (size_t)e * nc * NF;
    if (!cell_ok(s)) {
      for (int m = 0; m < nc * NF; m++) f[m] = T(0);
      continue;
    }
    const int64_t K = first + s, b = K / 64, l = K % 64;
    T Ki[DIM * DIM];
#pragma unroll
    for (int m = 0; m < DIM * DIM; m++) Ki[m] = A.geo[(b * G + m) * 64 + l];
    const T wd = w[q] * A.geo[(b * G + DIM * DIM) * 64 + l];
    T cq = T(1);
    if (A.coef) {
      cq = T(0);
#pragma unroll
      for (int a = 0; a < NV; a++) cq += vb[q * NV + a] * A.coef[(b * NV + a) * 64 + l];
    }
    // (the component loops run to 3 with a guard, so that the register arrays are
    // indexed by constants)
    T u[3] = {T(0), T(0), T(0)}, gr[3][DIM];
#pragma unroll
    for (int c = 0; c < 3; c++)
#pragma unroll
      for (int d = 0; d < DIM; d++) gr[c][d] = T(0);
    const T *xc = xs + s * D * nc;
    for (int i = 0; i < D; i++) {
      const T vi = vT[i * NQ + q];
      T gi[DIM];
#pragma unroll
      for (int d = 0; d < DIM; d++) gi[d] = gT[(d * D + i) * NQ + q];
#pragma unroll
      for (int c = 0; c < 3; c++)
        if (c < nc) {
          const T xv = xc[i * nc + c];
          u[c] += vi * xv;
#pragma unroll
          for (int d = 0; d < DIM; d++) gr[c][d] += gi[d] * xv;
        }
    }
    // physical gradients G[c][a] = sum_d K[d][a] gr[c][d]
    T Gp[3][3];
#pragma unroll
    for (int c = 0; c < 3; c++)
#pragma unroll
      for (int a = 0; a < 3; a++) {
        T t = T(0);
        if (a < DIM)
#pragma unroll
          for (int d = 0; d < DIM; d++) t += Ki[d * DIM + a] * gr[c][d];
        Gp[c][a] = t;
      }
    // physical flux (against grad v) and value flux, then the reference flux
    // fr[d] = sum_a K[d][a] f[a]
    T tr = T(0);
    if (A.kind == MF_OP_ELASTICITY)
#pragma unroll
      for (int a = 0; a < DIM; a++) tr += Gp[a][a];
#pragma unroll
    for (int c = 0; c < 3; c++) {
      if (c >= nc) break;
      T f1[DIM], f0 = T(0);
#pragma unroll
      for (int a = 0; a < DIM; a++) {
        T val = Gp[c][a];  // HELMHOLTZ, LAPLACIAN
        if (A.kind == MF_OP_POISSON) val = cq * Gp[c][a];
        else if (A.kind == MF_OP_MASS) val = T(0);
        else if (A.kind == MF_OP_ELASTICITY) val = A.mu * (Gp[c][a] + Gp[a][c]) + (a == c ? A.lam * tr : T(0));
        f1[a] = wd * val;
      }
      if (A.kind == MF_OP_MASS) f0 = wd * cq * u[c];
      else if (A.kind == MF_OP_HELMHOLTZ) f0 = wd * u[c];
      f[c * NF] = f0;
#pragma unroll
      for (int d = 0; d < DIM; d++) {
        T t = T(0);
#pragma unroll
        for (int a = 0; a < DIM; a++) t += Ki[d * DIM + a] * f1[a];
        f[c * NF + 1 + d] = t;
      }
    }
  }
  __syncthreads();
  // (B) nodes and the scatter
  for (int e = threadIdx.x; e < CB * D; e += blockDim.x) {
    const int s = e / D, i = e - s * D;
    if (!cell_ok(s)) continue;
    const int32_t n = node_of(first + s, i);
    if (n < 0) continue;  // constrained: never scattered
    const T *fs = fq + (size_t)s * NQ * nc * NF;
    T acc[3] = {T(0), T(0), T(0)};
    for (int q = 0; q < NQ; q++) {
      const T vi = v[q * D + i];
      T gi[DIM];
#pragma unroll
      for (int d = 0; d < DIM; d++) gi[d] = g[(q * DIM + d) * D + i];
#pragma unroll
      for (int c = 0; c < 3; c++)
        if (c < nc) {
          const T *f = fs + (q * nc + c) * NF;
          T t = vi * f[0];
#pragma unroll
          for (int d = 0; d < DIM; d++) t += gi[d] * f[1 + d];
          acc[c] += t;
        }
    }
#pragma unroll
    for (int c = 0; c < 3; c++) {
      if (c >= nc) break;
      T *yp = A.y + (int64_t)n * nc + c;
      if (atomic) sd_atomic_add(yp, acc[c]);
      else *yp += acc[c];
    }
  }
}

// cells per workgroup: as many as about 48 KB of LDS holds, at most 16
template <typename T> int simplex_dense_cells_per_block(int D, int nq, int ncomp, int dim) {
  const size_t per = ((size_t)D * ncomp + (size_t)nq * ncomp * (1 + dim)) * sizeof(T);
  int cb = (int)((48 * 1024) / per);
  return cb < 1 ? 1 : (cb > 16 ? 16 : cb);
}

template <typename T> int launch_simplex_dense(int dim, const SimplexDenseArgs<T> &a, bool atomic, hipStream_t s) {
  if (a.c1 <= a.c0) return MF_OK;
  if (a.ncomp < 1 || a.ncomp > 3) return fail(MF_EINVAL, "simplex dense kernel: ncomp");
  const size_t lds = ((size_t)a.cb * a.D * a.ncomp + (size_t)a.cb * a.nq * a.ncomp * (1 + dim)) * sizeof(T);
  if (lds > 64 * 1024) return fail(MF_EUNSUPPORTED, "simplex dense kernel: element too large for LDS");
  const int64_t nb = (a.c1 - a.c0 + a.cb - 1) / a.cb;
  if (dim == 3)
    simplex_dense_kernel<T, 3><<<dim3((unsigned)nb), dim3(256), lds, s>>>(a, atomic);
  else
    simplex_dense_kernel<T, 2><<<dim3((unsigned)nb), dim3(256), lds, s>>>(a, atomic);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

template int simplex_dense_cells_per_block<double>(int, int, int, int);
template int simplex_dense_cells_per_block<float>(int, int, int, int);
template int launch_simplex_dense<double>(int, const SimplexDenseArgs<double> &, bool, hipStream_t);
template int launch_simplex_dense<float>(int, const SimplexDenseArgs<float> &, bool, hipStream_t);

}  // namespace mf
