// Element matrices added into a global CSR matrix: the paper's assembly of a bilinear
// form into a sparse matrix (Section 5: the same local kernel with a matrix scatter,
// the batched local results unpacked into the global structure). The entries are
// formed from the tabulated basis at the operator's quadrature points in FP64 and
// each is added at its CSR position (binary search of the column in the row) with a
// device atomic, since rows are shared between cells. Simplices: a thread per (cell,
// row node); tensor-product cells (more nodes per cell): a thread per (cell, row node,
// column node).
#include "mf_internal.h"

namespace mf {

namespace {
__device__ __forceinline__ void csr_add(double *p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void csr_add(float *p, double v) { unsafeAtomicAdd(p, (float)v); }

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

// the element-matrix entry, or DIM x DIM block for ELASTICITY, of the form at one
// point: gradients gi, gj and values pi, pj of the two basis functions, coefficient cq
// (1 where the kind has none), weight wd = w |det J|. MASS c u v, HELMHOLTZ
// grad u . grad v + u v, LAPLACIAN grad u . grad v (per component), POISSON
// kappa grad u . grad v, ELASTICITY lambda d_c v_i d_d u_j + mu (delta_cd grad u_j .
// grad v_i + d_d v_i d_c u_j) for component c of the test and d of the trial function.
template <int DIM>
__device__ __forceinline__ void form_at_point(int kind, const double *gi, const double *gj, double pi, double pj,
                                              double cq, double wd, double lam, double mu, double (&e)[3][3]) {
  double gg = 0.0;
  for (int a = 0; a < DIM; a++) gg += gi[a] * gj[a];
  if (kind == MF_OP_ELASTICITY) {
    for (int c = 0; c < DIM; c++)
      for (int d = 0; d < DIM; d++)
        e[c][d] += wd * (lam * gi[c] * gj[d] + mu * ((c == d ? gg : 0.0) + gi[d] * gj[c]));
  } else {
    double v = gg;  // LAPLACIAN
    if (kind == MF_OP_MASS) v = cq * pi * pj;
    else if (kind == MF_OP_HELMHOLTZ) v = gg + pi * pj;
    else if (kind == MF_OP_POISSON) v = cq * gg;
    for (int c = 0; c < 3; c++) e[c][c] += wd * v;
  }
}

template <typename T>
__device__ __forceinline__ void add_block(int kind, int nc, int64_t ui, int64_t uj, const double (&e)[3][3],
                                          const int64_t *rowptr, const int32_t *col, T *vals) {
  for (int c = 0; c < nc; c++)
    for (int d = 0; d < nc; d++) {
      if (kind != MF_OP_ELASTICITY && c != d) continue;
      const int64_t pos = csr_find(rowptr, col, ui * nc + c, (int32_t)(uj * nc + d));
      if (pos >= 0) csr_add(&vals[pos], e[c][d]);
    }
}
}  // namespace

constexpr int kMaxD = 84;  // P6 tets

// Simplices: AoSoA map [cell/64][D][64], geometry [cell/64][DIM*DIM + 1][64] (d xi_b /
// d x_a at b*DIM + a, then |det J|), vertex coefficients [cell/64][DIM+1][64]; tab
// (FP64): phi [nq][D], reference gradients [nq][D][DIM], weights [nq], vertex basis
// [nq][DIM+1].
template <typename T, int DIM>
__global__ void __launch_bounds__(256) simplex_element_csr_kernel(
    const int32_t *__restrict__ fmap, const int32_t *__restrict__ unode, const T *__restrict__ geo,
    const T *__restrict__ coef, const double *__restrict__ tab, int64_t ncells, int D, int NQ, int kind, int nc,
    double lam, double mu, const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
    T *__restrict__ vals) {
  constexpr int G = DIM * DIM + 1, NV = DIM + 1;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ncells * D) return;
  const int64_t K = t / D;
  const int i = (int)(t - K * D);
  const int64_t b = K / 64, l = K % 64;
  if (fmap[(b * D + i) * 64 + l] < 0) return;  // constrained row: set separately
  double Ki[DIM * DIM];
  for (int m = 0; m < DIM * DIM; m++) Ki[m] = (double)geo[(b * G + m) * 64 + l];
  const double adet = (double)geo[(b * G + DIM * DIM) * 64 + l];
  double cv[NV];
  for (int v = 0; v < NV; v++) cv[v] = coef ? (double)coef[(b * NV + v) * 64 + l] : 1.0;
  const double *phi = tab, *dphi = tab + NQ * D, *w = dphi + NQ * D * DIM, *vb = w + NQ;
  const int64_t ui = unode[K * D + i];
  for (int j = 0; j < D; j++) {
    if (fmap[(b * D + j) * 64 + l] < 0) continue;  // constrained column: zero
    double e[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int q = 0; q < NQ; q++) {
      double gi[DIM], gj[DIM];
      for (int a = 0; a < DIM; a++) {
        double si = 0.0, sj = 0.0;
        for (int bb = 0; bb < DIM; bb++) {
          si += dphi[(q * D + i) * DIM + bb] * Ki[bb * DIM + a];
          sj += dphi[(q * D + j) * DIM + bb] * Ki[bb * DIM + a];
        }
        gi[a] = si;
        gj[a] = sj;
      }
      double cq = 0.0;
      for (int v = 0; v < NV; v++) cq += vb[q * NV + v] * cv[v];
      form_at_point<DIM>(kind, gi, gj, phi[q * D + i], phi[q * D + j], cq, w[q] * adet, lam, mu, e);
    }
    add_block(kind, nc, ui, unode[K * D + j], e, rowptr, col, vals);
  }
}

// Hexahedra: map [cell][n^3] (node i1 + n i2 + n^2 i3), trilinear monomial
// coefficients [cell][24] (c1..c7 of each coordinate at 3 (m-1) + r), coefficient
// polynomial [cell][8] (c0..c7). Quadrilaterals: map [cell][n^2] (i1 + n i2), bilinear
// coefficients [cell][6] (c1, c2, c3 of each coordinate at 2 (m-1) + r), vertex
// coefficients [cell][4]. tab (FP64): B [q][n], B' [q][n], weights [q], points [q].
template <typename T, int DIM>
__global__ void __launch_bounds__(256) tensor_element_csr_kernel(
    const int32_t *__restrict__ map, const int32_t *__restrict__ unode, const T *__restrict__ geo,
    const T *__restrict__ coef, const double *__restrict__ tab, int64_t ncells, int n, int nq, int kind, int nc,
    double lam, double mu, const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
    T *__restrict__ vals) {
  const int D = DIM == 3 ? n * n * n : n * n;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ncells * D * D) return;
  const int64_t K = t / ((int64_t)D * D);
  const int ij = (int)(t - K * D * D), i = ij / D, j = ij - (ij / D) * D;
  if (map[K * D + i] < 0 || map[K * D + j] < 0) return;  // constrained row / column
  int ia[3] = {i % n, (i / n) % n, DIM == 3 ? i / (n * n) : 0};
  int ja[3] = {j % n, (j / n) % n, DIM == 3 ? j / (n * n) : 0};
  const double *B = tab, *Bd = tab + nq * n, *w = Bd + nq * n, *g = w + nq;
  constexpr int NG = DIM == 3 ? 24 : 6, NK = DIM == 3 ? 8 : 4;
  double c[NG];
  for (int m = 0; m < NG; m++) c[m] = (double)geo[K * NG + m];
  double kc[NK];
  // no coefficient: the constant 1 (monomial form on hexes, vertex values on quads)
  for (int m = 0; m < NK; m++) kc[m] = coef ? (double)coef[K * NK + m] : (DIM == 2 || m == 0 ? 1.0 : 0.0);
  double e[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  const int nq3 = DIM == 3 ? nq : 1;
  for (int q3 = 0; q3 < nq3; q3++)
    for (int q2 = 0; q2 < nq; q2++)
      for (int q1 = 0; q1 < nq; q1++) {
        const int qa[3] = {q1, q2, q3};
        const double x[3] = {g[q1], g[q2], DIM == 3 ? g[q3] : 0.0};
        double J[DIM][DIM], Cf[DIM][DIM], det, cq;
        if constexpr (DIM == 3) {
          for (int r = 0; r < 3; r++) {
            J[r][0] = c[r] + c[9 + r] * x[1] + c[12 + r] * x[2] + c[18 + r] * x[1] * x[2];
            J[r][1] = c[3 + r] + c[9 + r] * x[0] + c[15 + r] * x[2] + c[18 + r] * x[0] * x[2];
            J[r][2] = c[6 + r] + c[12 + r] * x[0] + c[15 + r] * x[1] + c[18 + r] * x[0] * x[1];
          }
          Cf[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
          Cf[0][1] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
          Cf[0][2] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
          Cf[1][0] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
          Cf[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
          Cf[1][2] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
          Cf[2][0] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
          Cf[2][1] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
          Cf[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
          det = J[0][0] * Cf[0][0] + J[0][1] * Cf[0][1] + J[0][2] * Cf[0][2];
          cq = kc[0] + kc[1] * x[0] + kc[2] * x[1] + kc[3] * x[2] + kc[4] * x[0] * x[1] + kc[5] * x[0] * x[2] +
               kc[6] * x[1] * x[2] + kc[7] * x[0] * x[1] * x[2];
        } else {
          for (int r = 0; r < 2; r++) {
            J[r][0] = c[r] + c[4 + r] * x[1];
            J[r][1] = c[2 + r] + c[4 + r] * x[0];
          }
          Cf[0][0] = J[1][1];
          Cf[0][1] = -J[1][0];
          Cf[1][0] = -J[0][1];
          Cf[1][1] = J[0][0];
          det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
          cq = (1 - x[0]) * (1 - x[1]) * kc[0] + x[0] * (1 - x[1]) * kc[1] + (1 - x[0]) * x[1] * kc[2] +
               x[0] * x[1] * kc[3];
        }
        double pi = 1.0, pj = 1.0, ri[DIM], rj[DIM];
        for (int a = 0; a < DIM; a++) {
          pi *= B[qa[a] * n + ia[a]];
          pj *= B[qa[a] * n + ja[a]];
        }
        for (int a = 0; a < DIM; a++) {
          double si = 1.0, sj = 1.0;
          for (int bb = 0; bb < DIM; bb++) {
            si *= bb == a ? Bd[qa[bb] * n + ia[bb]] : B[qa[bb] * n + ia[bb]];
            sj *= bb == a ? Bd[qa[bb] * n + ja[bb]] : B[qa[bb] * n + ja[bb]];
          }
          ri[a] = si;
          rj[a] = sj;
        }
        // physical gradient: J^{-T} ref, (J^{-1})_{e r} = Cf[r][e] / det
        double gi[DIM], gj[DIM];
        for (int r = 0; r < DIM; r++) {
          double si = 0.0, sj = 0.0;
          for (int a = 0; a < DIM; a++) {
            si += Cf[r][a] * ri[a];
            sj += Cf[r][a] * rj[a];
          }
          gi[r] = si / det;
          gj[r] = sj / det;
        }
        double wd = (det < 0.0 ? -det : det) * w[q1] * w[q2];
        if (DIM == 3) wd *= w[q3];
        form_at_point<DIM>(kind, gi, gj, pi, pj, cq, wd, lam, mu, e);
      }
  add_block(kind, nc, unode[K * D + i], unode[K * D + j], e, rowptr, col, vals);
}

// P1 triangle mass with a vertex coefficient: int_T c phi_i phi_j for c = sum_a c_a
// lambda_a, i.e. sum_a s_a (1 + [a=i] + [a=j] + [i=j] + 2 [a=i][a=j]) / 60 with
// s_a = |T| c_a (the closed form of the action kernel); map [cell][3]
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
    if (pos >= 0) csr_add(&vals[pos], v / 60.0);
  }
}

template <typename T> __global__ void set_at_kernel(const int64_t *pos, int64_t n, T v, T *vals) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) vals[pos[t]] = v;
}

template <typename T>
int launch_simplex_element_csr(int dim, const int32_t *fmap, const int32_t *unode, const T *geo, const T *coef,
                               const double *tab, int64_t ncells, int D, int nq, int kind, int ncomp, double lam,
                               double mu, const int64_t *rowptr, const int32_t *col, T *vals, hipStream_t s) {
  if (D > kMaxD) return fail(MF_EUNSUPPORTED, "assembly: simplices up to P6");
  const int64_t n = ncells * D;
  if (n == 0) return MF_OK;
  const dim3 g((unsigned)((n + 255) / 256)), b(256);
  if (dim == 3)
    simplex_element_csr_kernel<T, 3><<<g, b, 0, s>>>(fmap, unode, geo, coef, tab, ncells, D, nq, kind, ncomp, lam,
                                                     mu, rowptr, col, vals);
  else
    simplex_element_csr_kernel<T, 2><<<g, b, 0, s>>>(fmap, unode, geo, coef, tab, ncells, D, nq, kind, ncomp, lam,
                                                     mu, rowptr, col, vals);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

template <typename T>
int launch_tensor_element_csr(int dim, const int32_t *map, const int32_t *unode, const T *geo, const T *coef,
                              const double *tab, int64_t ncells, int n, int nq, int kind, int ncomp, double lam,
                              double mu, const int64_t *rowptr, const int32_t *col, T *vals, hipStream_t s) {
  const int64_t D = dim == 3 ? (int64_t)n * n * n : (int64_t)n * n, tot = ncells * D * D;
  if (tot == 0) return MF_OK;
  if ((tot + 255) / 256 > INT32_MAX) return fail(MF_EUNSUPPORTED, "assembly: too many element-matrix entries");
  const dim3 g((unsigned)((tot + 255) / 256)), b(256);
  if (dim == 3)
    tensor_element_csr_kernel<T, 3><<<g, b, 0, s>>>(map, unode, geo, coef, tab, ncells, n, nq, kind, ncomp, lam, mu,
                                                    rowptr, col, vals);
  else
    tensor_element_csr_kernel<T, 2><<<g, b, 0, s>>>(map, unode, geo, coef, tab, ncells, n, nq, kind, ncomp, lam, mu,
                                                    rowptr, col, vals);
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

#define MF_CSR_INST(T)                                                                                             \
  template int launch_simplex_element_csr<T>(int, const int32_t *, const int32_t *, const T *, const T *,          \
                                             const double *, int64_t, int, int, int, int, double, double,          \
                                             const int64_t *, const int32_t *, T *, hipStream_t);                  \
  template int launch_tensor_element_csr<T>(int, const int32_t *, const int32_t *, const T *, const T *,           \
                                            const double *, int64_t, int, int, int, int, double, double,           \
                                            const int64_t *, const int32_t *, T *, hipStream_t);                   \
  template int launch_tri_mass_element_csr<T>(const int32_t *, const int32_t *, const T *, int64_t,                \
                                              const int64_t *, const int32_t *, T *, hipStream_t);                 \
  template int launch_set_at<T>(const int64_t *, int64_t, T, T *, hipStream_t);
MF_CSR_INST(double)
MF_CSR_INST(float)
#undef MF_CSR_INST

}  // namespace mf
