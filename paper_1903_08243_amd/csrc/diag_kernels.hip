// Diagonal of the operator (for the Jacobi preconditioner) computed entry by entry from
// the element matrices' diagonals, for the operators whose action kernels have no
// fused diagonal pass: the one-component tet operators, the triangle operators of
// degree 1-3 other than the closed-form P1 mass, hex elasticity and the hex scalar
// operators with k+2 points. A thread per (cell, node) evaluates the node's basis
// function and its gradient at every quadrature point (Section 2.1: the local kernel's
// tabulation and geometry) in FP64 and adds the diagonal entries of its element
// matrix into d with device atomics. Off the hot path: once per operator.
#include "mf_internal.h"

namespace mf {

namespace {
__device__ __forceinline__ void diag_add(double *p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void diag_add(float *p, double v) { unsafeAtomicAdd(p, (float)v); }
}  // namespace

// Simplices (DIM = 2, 3): AoSoA map [cell/64][D][64], geometry [cell/64][DIM*DIM + 1][64]
// (d xi_b / d x_a at b*DIM + a, then |det J|), vertex coefficients [cell/64][DIM+1][64].
// tab (FP64): phi [nq][D], reference gradients [nq][D][DIM], weights [nq], vertex
// basis [nq][DIM+1].
template <typename T, int DIM>
__global__ void __launch_bounds__(256) simplex_element_diag_kernel(const int32_t *__restrict__ fmap,
                                                                   const T *__restrict__ geo,
                                                                   const T *__restrict__ coef,
                                                                   const double *__restrict__ tab, int64_t ncells,
                                                                   int D, int NQ, int kind, int nc, double lam,
                                                                   double mu, T *__restrict__ d) {
  constexpr int G = DIM * DIM + 1, NV = DIM + 1;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ncells * D) return;
  const int64_t K = t / D;
  const int i = (int)(t - K * D);
  const int64_t b = K / 64, l = K % 64;
  const int32_t node = fmap[(b * D + i) * 64 + l];
  if (node < 0) return;  // constrained: set to 1 afterwards
  double Ki[DIM * DIM];
  for (int m = 0; m < DIM * DIM; m++) Ki[m] = (double)geo[(b * G + m) * 64 + l];
  const double adet = (double)geo[(b * G + DIM * DIM) * 64 + l];
  double cv[NV];
  for (int v = 0; v < NV; v++) cv[v] = coef ? (double)coef[(b * NV + v) * 64 + l] : 1.0;
  const double *phi = tab, *dphi = tab + NQ * D, *w = dphi + NQ * D * DIM, *vb = w + NQ;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int q = 0; q < NQ; q++) {
    double gi[DIM];
    for (int a = 0; a < DIM; a++) {
      double s = 0.0;
      for (int bb = 0; bb < DIM; bb++) s += dphi[(q * D + i) * DIM + bb] * Ki[bb * DIM + a];
      gi[a] = s;
    }
    double gg = 0.0;
    for (int a = 0; a < DIM; a++) gg += gi[a] * gi[a];
    const double wd = w[q] * adet, p = phi[q * D + i];
    if (kind == MF_OP_ELASTICITY) {
      for (int c = 0; c < DIM; c++) acc[c] += wd * (lam * gi[c] * gi[c] + mu * (gg + gi[c] * gi[c]));
    } else {
      double cq = 0.0;
      for (int v = 0; v < NV; v++) cq += vb[q * NV + v] * cv[v];
      double val = gg;                                    // LAPLACIAN
      if (kind == MF_OP_MASS) val = cq * p * p;
      else if (kind == MF_OP_HELMHOLTZ) val = gg + p * p;
      else if (kind == MF_OP_POISSON) val = cq * gg;
      acc[0] += wd * val;
    }
  }
  for (int c = 0; c < nc; c++) diag_add(&d[(int64_t)node * nc + c], kind == MF_OP_ELASTICITY ? acc[c] : acc[0]);
}

// Hexahedra: map [cell][n^3] (node i1 + n i2 + n^2 i3), trilinear coefficients
// [cell][24] (c1..c7 of each coordinate, entry 3 (m-1) + r), vertex coefficient
// polynomial [cell][8] (c0..c7). tab (FP64): B [q][n] (basis at the Gauss points),
// B' [q][n], weights [q], points [q].
template <typename T>
__global__ void __launch_bounds__(256) hex_element_diag_kernel(const int32_t *__restrict__ map,
                                                               const T *__restrict__ geo,
                                                               const T *__restrict__ coef,
                                                               const double *__restrict__ tab, int64_t ncells, int n,
                                                               int nq, int kind, int nc, double lam, double mu,
                                                               T *__restrict__ d) {
  const int D = n * n * n;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ncells * D) return;
  const int64_t K = t / D;
  const int i = (int)(t - K * D);
  const int32_t node = map[K * D + i];
  if (node < 0) return;
  const int i1 = i % n, i2 = (i / n) % n, i3 = i / (n * n);
  double c[7][3];
  for (int m = 0; m < 7; m++)
    for (int r = 0; r < 3; r++) c[m][r] = (double)geo[K * 24 + 3 * m + r];
  double kc[8] = {1, 0, 0, 0, 0, 0, 0, 0};
  if (coef)
    for (int m = 0; m < 8; m++) kc[m] = (double)coef[K * 8 + m];
  const double *B = tab, *Bd = tab + nq * n, *w = Bd + nq * n, *g = w + nq;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int qc = 0; qc < nq; qc++)
    for (int qb = 0; qb < nq; qb++)
      for (int qa = 0; qa < nq; qa++) {
        const double x1 = g[qa], x2 = g[qb], x3 = g[qc];
        double J[3][3];
        for (int r = 0; r < 3; r++) {
          J[r][0] = c[0][r] + c[3][r] * x2 + c[4][r] * x3 + c[6][r] * x2 * x3;
          J[r][1] = c[1][r] + c[3][r] * x1 + c[5][r] * x3 + c[6][r] * x1 * x3;
          J[r][2] = c[2][r] + c[4][r] * x1 + c[5][r] * x2 + c[6][r] * x1 * x2;
        }
        // cofactors C[r][e] of J: J^{-1}[e][r] = C[r][e] / det
        double C[3][3];
        C[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        C[0][1] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        C[0][2] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        C[1][0] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
        C[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
        C[1][2] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
        C[2][0] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
        C[2][1] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
        C[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        const double det = J[0][0] * C[0][0] + J[0][1] * C[0][1] + J[0][2] * C[0][2];
        const double ba = B[qa * n + i1], bb = B[qb * n + i2], bc = B[qc * n + i3];
        const double ref[3] = {Bd[qa * n + i1] * bb * bc, ba * Bd[qb * n + i2] * bc, ba * bb * Bd[qc * n + i3]};
        double gp[3];  // physical gradient
        for (int r = 0; r < 3; r++) gp[r] = (C[r][0] * ref[0] + C[r][1] * ref[1] + C[r][2] * ref[2]) / det;
        const double gg = gp[0] * gp[0] + gp[1] * gp[1] + gp[2] * gp[2];
        const double wd = w[qa] * w[qb] * w[qc] * (det < 0.0 ? -det : det), p = ba * bb * bc;
        if (kind == MF_OP_ELASTICITY) {
          for (int e = 0; e < 3; e++) acc[e] += wd * (lam * gp[e] * gp[e] + mu * (gg + gp[e] * gp[e]));
        } else {
          const double kq = kc[0] + kc[1] * x1 + kc[2] * x2 + kc[3] * x3 + kc[4] * x1 * x2 + kc[5] * x1 * x3 +
                            kc[6] * x2 * x3 + kc[7] * x1 * x2 * x3;
          double val = gg;  // LAPLACIAN
          if (kind == MF_OP_MASS) val = kq * p * p;
          else if (kind == MF_OP_HELMHOLTZ) val = gg + p * p;
          else if (kind == MF_OP_POISSON) val = kq * gg;
          acc[0] += wd * val;
        }
      }
  for (int e = 0; e < nc; e++) diag_add(&d[(int64_t)node * nc + e], kind == MF_OP_ELASTICITY ? acc[e] : acc[0]);
}

template <typename T>
int launch_simplex_element_diag(int dim, const int32_t *fmap, const T *geo, const T *coef, const double *tab,
                                int64_t ncells, int D, int nq, int kind, int nc, double lam, double mu, T *d,
                                hipStream_t s) {
  const int64_t n = ncells * D;
  if (n == 0) return MF_OK;
  const dim3 g((unsigned)((n + 255) / 256)), b(256);
  if (dim == 3)
    simplex_element_diag_kernel<T, 3><<<g, b, 0, s>>>(fmap, geo, coef, tab, ncells, D, nq, kind, nc, lam, mu, d);
  else
    simplex_element_diag_kernel<T, 2><<<g, b, 0, s>>>(fmap, geo, coef, tab, ncells, D, nq, kind, nc, lam, mu, d);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

template <typename T>
int launch_hex_element_diag(const int32_t *map, const T *geo, const T *coef, const double *tab, int64_t ncells,
                            int n, int nq, int kind, int nc, double lam, double mu, T *d, hipStream_t s) {
  const int64_t tot = ncells * n * n * n;
  if (tot == 0) return MF_OK;
  hex_element_diag_kernel<T><<<dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s>>>(map, geo, coef, tab, ncells,
                                                                                       n, nq, kind, nc, lam, mu, d);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

template int launch_simplex_element_diag<double>(int, const int32_t *, const double *, const double *,
                                                 const double *, int64_t, int, int, int, int, double, double,
                                                 double *, hipStream_t);
template int launch_simplex_element_diag<float>(int, const int32_t *, const float *, const float *, const double *,
                                                int64_t, int, int, int, int, double, double, float *, hipStream_t);
template int launch_hex_element_diag<double>(const int32_t *, const double *, const double *, const double *,
                                             int64_t, int, int, int, int, double, double, double *, hipStream_t);
template int launch_hex_element_diag<float>(const int32_t *, const float *, const float *, const double *, int64_t,
                                            int, int, int, int, double, double, float *, hipStream_t);

}  // namespace mf
