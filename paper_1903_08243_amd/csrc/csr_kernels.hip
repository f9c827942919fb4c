// Element matrices added into a global CSR matrix: the paper's assembly of a bilinear
// form into a sparse matrix (Section 5: the same local kernel with a matrix scatter,
// the batched local results unpacked into the global structure). A thread per (cell,
// row node); it forms the cell's element-matrix row blocks from the tabulated basis at
// the quadrature points and adds each entry at its CSR position (binary search of the
// column in the row), with device atomics, since rows are shared between cells.
#include "mf_internal.h"

namespace mf {

namespace {
__device__ __forceinline__ void csr_add(double *p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void csr_add(float *p, float v) { unsafeAtomicAdd(p, (float)v); }

__device__ __forceinline__ int64_t csr_find(const int64_t *rowptr, const int32_t *col, int64_t r, int32_t c) {
  int64_t lo = rowptr[r], hi = rowptr[r + 1] - 1;
  while (lo <= hi) {
    const int64_t m = (lo + hi) >> 1;
    const int32_t v = col[m];
    if (v == c) return m;
    if (v < c) lo = m + 1;
    else hi = m - 1;
  }
  return -1;  // not in the pattern (cannot happen for entries of one cell)
}
}  // namespace

constexpr int kMaxD = 20;  // P3 tets

// a(u, v) entries in FP64: MASS c u v, HELMHOLTZ grad u . grad v + u v, LAPLACIAN
// grad u . grad v (per component), POISSON kappa grad u . grad v, ELASTICITY
// lambda d_c v_i d_d u_j + mu (delta_cd grad u_j . grad v_i + d_d v_i d_c u_j) for
// component c of the test and d of the trial function.
template <typename T>
__global__ void __launch_bounds__(256) tet_element_csr_kernel(const int32_t *__restrict__ fmap,
                                                              const int32_t *__restrict__ unode,
                                                              const T *__restrict__ geo, const T *__restrict__ coef,
                                                              const double *__restrict__ tab, int64_t ncells, int D,
                                                              int NQ, int kind, int nc, double lam, double mu,
                                                              const int64_t *__restrict__ rowptr,
                                                              const int32_t *__restrict__ col, T *__restrict__ vals) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ncells * D) return;
  const int64_t K = t / D;
  const int i = (int)(t - K * D);
  const int64_t b = K / 64, l = K % 64;
  if (fmap[(b * D + i) * 64 + l] < 0) return;  // constrained row: set separately
  double Ki[9];
  for (int m = 0; m < 9; m++) Ki[m] = (double)geo[(b * 10 + m) * 64 + l];
  const double adet = (double)geo[(b * 10 + 9) * 64 + l];
  double cv[4] = {1.0, 1.0, 1.0, 1.0};
  if (coef)
    for (int v = 0; v < 4; v++) cv[v] = (double)coef[(b * 4 + v) * 64 + l];
  const double *phi = tab, *dphi = tab + NQ * D, *w = dphi + NQ * D * 3, *vb = w + NQ;
  const int32_t ui = unode[K * D + i];
  for (int j = 0; j < D; j++) {
    if (fmap[(b * D + j) * 64 + l] < 0) continue;  // constrained column: zero
    double e[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int q = 0; q < NQ; q++) {
      double gi[3], gj[3];
      for (int a = 0; a < 3; a++) {
        const double *ti = dphi + (q * D + i) * 3, *tj = dphi + (q * D + j) * 3;
        gi[a] = ti[0] * Ki[a] + ti[1] * Ki[3 + a] + ti[2] * Ki[6 + a];
        gj[a] = tj[0] * Ki[a] + tj[1] * Ki[3 + a] + tj[2] * Ki[6 + a];
      }
      const double wd = w[q] * adet, gg = gi[0] * gj[0] + gi[1] * gj[1] + gi[2] * gj[2];
      if (kind == MF_OP_ELASTICITY) {
        for (int c = 0; c < 3; c++)
          for (int d = 0; d < 3; d++)
            e[c][d] += wd * (lam * gi[c] * gj[d] + mu * ((c == d ? gg : 0.0) + gi[d] * gj[c]));
      } else {
        const double cq = vb[q * 4] * cv[0] + vb[q * 4 + 1] * cv[1] + vb[q * 4 + 2] * cv[2] + vb[q * 4 + 3] * cv[3];
        const double pp = phi[q * D + i] * phi[q * D + j];
        double v = 0.0;
        if (kind == MF_OP_MASS) v = cq * pp;
        else if (kind == MF_OP_HELMHOLTZ) v = gg + pp;
        else if (kind == MF_OP_LAPLACIAN) v = gg;
        else v = cq * gg;  // POISSON
        for (int c = 0; c < 3; c++) e[c][c] += wd * v;
      }
    }
    const int32_t uj = unode[K * D + j];
    for (int c = 0; c < nc; c++)
      for (int d = 0; d < nc; d++) {
        if (kind != MF_OP_ELASTICITY && c != d) continue;
        const int64_t pos = csr_find(rowptr, col, (int64_t)ui * nc + c, uj * nc + d);
        if (pos >= 0) csr_add(&vals[pos], (T)e[c][d]);
      }
  }
}

// P1 triangle mass with a vertex coefficient: int_T c phi_i phi_j for c = sum_a c_a
// lambda_a, i.e. sum_a s_a (1 + [a=i] + [a=j] + [i=j] + 2 [a=i][a=j]) / 60 with
// s_a = |T| c_a (the closed form of the action kernel)
template <typename T>
__global__ void __launch_bounds__(256) tri_mass_element_csr_kernel(const int32_t *__restrict__ fmap,
                                                                   const int32_t *__restrict__ unode,
                                                                   const T *__restrict__ geo, int64_t ncells,
                                                                   const int64_t *__restrict__ rowptr,
                                                                   const int32_t *__restrict__ col,
                                                                   T *__restrict__ vals) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ncells * 3) return;
  const int64_t K = t / 3;
  const int i = (int)(t - K * 3);
  if (fmap[K * 3 + i] < 0) return;
  double sa[3];
  for (int a = 0; a < 3; a++) sa[a] = (double)geo[K * 4 + a];
  for (int j = 0; j < 3; j++) {
    if (fmap[K * 3 + j] < 0) continue;
    double v = 0.0;
    for (int a = 0; a < 3; a++)
      v += sa[a] * (1.0 + (a == i) + (a == j) + (i == j) + 2.0 * (a == i) * (a == j));
    const int64_t pos = csr_find(rowptr, col, unode[K * 3 + i], unode[K * 3 + j]);
    if (pos >= 0) csr_add(&vals[pos], (T)(v / 60.0));
  }
}

template <typename T> __global__ void set_at_kernel(const int64_t *pos, int64_t n, T v, T *vals) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) vals[pos[t]] = v;
}

template <typename T>
int launch_tet_element_csr(const int32_t *fmap, const int32_t *unode, const T *geo, const T *coef,
                           const double *tab, int64_t ncells, int D, int nq, int kind, int ncomp, double lam,
                           double mu, const int64_t *rowptr, const int32_t *col, T *vals, hipStream_t s) {
  if (D > kMaxD) return fail(MF_EUNSUPPORTED, "assembly: tets up to P3");
  const int64_t n = ncells * D;
  if (n == 0) return MF_OK;
  tet_element_csr_kernel<T><<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(
      fmap, unode, geo, coef, tab, ncells, D, nq, kind, ncomp, lam, mu, rowptr, col, vals);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

template <typename T>
int launch_tri_mass_element_csr(const int32_t *fmap, const int32_t *unode, const T *geo, int64_t ncells,
                                const int64_t *rowptr, const int32_t *col, T *vals, hipStream_t s) {
  const int64_t n = ncells * 3;
  if (n == 0) return MF_OK;
  tri_mass_element_csr_kernel<T><<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(fmap, unode, geo, ncells,
                                                                                          rowptr, col, vals);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

template <typename T> int launch_set_at(const int64_t *pos, int64_t n, T v, T *vals, hipStream_t s) {
  if (n <= 0) return MF_OK;
  set_at_kernel<T><<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(pos, n, v, vals);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

template int launch_tet_element_csr<double>(const int32_t *, const int32_t *, const double *, const double *,
                                            const double *, int64_t, int, int, int, int, double, double,
                                            const int64_t *, const int32_t *, double *, hipStream_t);
template int launch_tet_element_csr<float>(const int32_t *, const int32_t *, const float *, const float *,
                                           const double *, int64_t, int, int, int, int, double, double,
                                           const int64_t *, const int32_t *, float *, hipStream_t);
template int launch_tri_mass_element_csr<double>(const int32_t *, const int32_t *, const double *, int64_t,
                                                 const int64_t *, const int32_t *, double *, hipStream_t);
template int launch_tri_mass_element_csr<float>(const int32_t *, const int32_t *, const float *, int64_t,
                                                const int64_t *, const int32_t *, float *, hipStream_t);
template int launch_set_at<double>(const int64_t *, int64_t, double, double *, hipStream_t);
template int launch_set_at<float>(const int64_t *, int64_t, float, float *, hipStream_t);

}  // namespace mf
