// Operators on simplices of degree 4-6 (mass with a vertex coefficient, Helmholtz,
// Laplacian with one or dim components, Poisson, elasticity; the library runs
// triangles here, tetrahedra on the matrix-core kernels):
// the paper's local kernel by dense tabulation (Section 2.1: the basis and its
// reference gradients tabulated at the quadrature points, the affine Jacobian per
// cell; simplices are not sum-factorised, Section 4), for element sizes where a lane
// per cell would need more registers than a lane has.
//
// A workgroup takes CB consecutive cells. (0) A thread per (cell, node, component)
// gathers x into LDS. Then for each chunk of QC quadrature points: (A) a thread per
// (cell, point) contracts the cell's values with the tabulated basis (tables
// transposed, [node][point], so neighbouring threads read neighbouring entries), forms
// the physical gradient with the cell's J^{-1}, applies the pointwise operator and
// stores the value flux and the reference flux of each component in LDS; (B) the
// thread of each (cell, node) adds the chunk's fluxes contracted with the tabulated
// test functions ([point][node]). Last it scatters (atomic or, within a colour, plain
// read-modify-write). With HYPER the St-Venant-Kirchhoff tangent at u0 (vector tets):
// u0 is gathered beside x and its gradient formed at every point.
#include "mf_internal.h"

namespace mf {

namespace {
__device__ __forceinline__ void sd_atomic_add(double *p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void sd_atomic_add(float *p, float v) { unsafeAtomicAdd(p, v); }
}  // namespace

template <typename T, int DIM, bool HYPER>
__global__ void __launch_bounds__(256) simplex_dense_kernel(const SimplexDenseArgs<T> A, const bool atomic) {
  constexpr int G = DIM * DIM + 1, NV = DIM + 1, NF = 1 + DIM;
  const int D = A.D, NQ = A.nq, nc = A.ncomp, CB = A.cb, QC = A.qc;
  extern __shared__ __align__(16) unsigned char sd_lds[];
  T *xs = reinterpret_cast<T *>(sd_lds);      // [CB][D][nc]
  T *x0 = xs + CB * D * nc;                   // [CB][D][3] u0 (HYPER)
  T *fq = x0 + (HYPER ? CB * D * 3 : 0);      // [CB][QC][nc][1 + DIM]
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
  auto aosoa = [&](int64_t K, int i) { return ((K / 64) * D + i) * 64 + K % 64; };
  // (0) gather x (and u0, through the unflagged map when nodes are constrained)
  for (int e = threadIdx.x; e < CB * D * nc; e += blockDim.x) {
    const int s = e / (D * nc), r = e - s * D * nc, i = r / nc, c = r - i * nc;
    T val = T(0), val0 = T(0);
    if (cell_ok(s)) {
      const int64_t at = aosoa(first + s, i);
      const int32_t n = A.map[at];
      if (n >= 0) val = A.x[(int64_t)n * nc + c];
      if constexpr (HYPER) {
        const int32_t n0 = A.u0map ? A.u0map[at] : n;
        if (n0 >= 0) val0 = A.u0[(int64_t)n0 * 3 + c];
      }
    }
    xs[e] = val;
    if constexpr (HYPER) x0[e] = val0;
  }
  // the thread of (cell, node) for the test side: the host keeps CB * D <= blockDim
  const int sB = threadIdx.x / D, iB = threadIdx.x - sB * D;
  const bool ownB = sB < CB && cell_ok(sB);
  const int32_t nB = ownB ? A.map[aosoa(first + sB, iB)] : -1;
  T acc[3] = {T(0), T(0), T(0)};
  for (int q0 = 0; q0 < NQ; q0 += QC) {
    const int nqc = NQ - q0 < QC ? NQ - q0 : QC;
    __syncthreads();  // xs written (first chunk) / fq read by the previous chunk
    // (A) points q0 .. q0 + nqc of every cell
    for (int e = threadIdx.x; e < CB * nqc; e += blockDim.x) {
      const int s = e / nqc, qq = e - s * nqc, q = q0 + qq;
      T *f = fq + ((size_t)s * QC + qq) * nc * NF;
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
      T u[3] = {T(0), T(0), T(0)}, gr[3][DIM], gr0[3][DIM];
#pragma unroll
      for (int c = 0; c < 3; c++)
#pragma unroll
        for (int d = 0; d < DIM; d++) gr[c][d] = gr0[c][d] = T(0);
      const T *xc = xs + s * D * nc, *x0c = x0 + s * D * 3;
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
            if constexpr (HYPER) {
              const T xv0 = x0c[i * 3 + c];
#pragma unroll
              for (int d = 0; d < DIM; d++) gr0[c][d] += gi[d] * xv0;
            }
          }
      }
      // physical gradients G[c][a] = sum_d K[d][a] gr[c][d]
      T Gp[3][3], G0[3][3];
#pragma unroll
      for (int c = 0; c < 3; c++)
#pragma unroll
        for (int a = 0; a < 3; a++) {
          T t = T(0), t0 = T(0);
          if (a < DIM)
#pragma unroll
            for (int d = 0; d < DIM; d++) {
              t += Ki[d * DIM + a] * gr[c][d];
              t0 += Ki[d * DIM + a] * gr0[c][d];
            }
          Gp[c][a] = t;
          G0[c][a] = t0;
        }
      // physical flux Sg[c][a] (against d v_c / d x_a) and value flux f0[c]
      T Sg[3][3], f0[3] = {T(0), T(0), T(0)};
      if constexpr (HYPER) {
        // St-Venant-Kirchhoff tangent at u0: F = I + grad u0, E = (F^T F - I)/2,
        // S = lam tr(E) I + 2 mu E, dE = (grad u^T F + F^T grad u)/2, flux grad u S + F dS
        T F[3][3], S[3][3], dS[3][3], trE = T(0), trdE = T(0);
#pragma unroll
        for (int c = 0; c < 3; c++)
#pragma unroll
          for (int a = 0; a < 3; a++) F[c][a] = (c == a ? T(1) : T(0)) + G0[c][a];
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
          for (int j = 0; j < 3; j++) {
            T ff = T(0), gf = T(0);
#pragma unroll
            for (int k = 0; k < 3; k++) {
              ff += F[k][i] * F[k][j];
              gf += Gp[k][i] * F[k][j] + F[k][i] * Gp[k][j];
            }
            const T E = T(0.5) * (ff - (i == j ? T(1) : T(0))), dE = T(0.5) * gf;
            if (i == j) {
              trE += E;
              trdE += dE;
            }
            S[i][j] = T(2) * A.mu * E;
            dS[i][j] = T(2) * A.mu * dE;
          }
#pragma unroll
        for (int i = 0; i < 3; i++) {
          S[i][i] += A.lam * trE;
          dS[i][i] += A.lam * trdE;
        }
#pragma unroll
        for (int c = 0; c < 3; c++)
#pragma unroll
          for (int a = 0; a < 3; a++) {
            T t = T(0);
#pragma unroll
            for (int k = 0; k < 3; k++) t += Gp[c][k] * S[k][a] + F[c][k] * dS[k][a];
            Sg[c][a] = wd * t;
          }
      } else {
        T tr = T(0);
        if (A.kind == MF_OP_ELASTICITY)
#pragma unroll
          for (int a = 0; a < DIM; a++) tr += Gp[a][a];
#pragma unroll
        for (int c = 0; c < 3; c++)
#pragma unroll
          for (int a = 0; a < 3; a++) {
            T val = Gp[c][a];  // HELMHOLTZ, LAPLACIAN
            if (A.kind == MF_OP_POISSON) val = cq * Gp[c][a];
            else if (A.kind == MF_OP_MASS) val = T(0);
            else if (A.kind == MF_OP_ELASTICITY) val = A.mu * (Gp[c][a] + Gp[a][c]) + (a == c ? A.lam * tr : T(0));
            Sg[c][a] = wd * val;
          }
#pragma unroll
        for (int c = 0; c < 3; c++) {
          if (A.kind == MF_OP_MASS) f0[c] = wd * cq * u[c];
          else if (A.kind == MF_OP_HELMHOLTZ) f0[c] = wd * u[c];
        }
      }
      // reference flux fr[d] = sum_a K[d][a] Sg[c][a]
#pragma unroll
      for (int c = 0; c < 3; c++) {
        if (c >= nc) break;
        f[c * NF] = f0[c];
#pragma unroll
        for (int d = 0; d < DIM; d++) {
          T t = T(0);
#pragma unroll
          for (int a = 0; a < DIM; a++) t += Ki[d * DIM + a] * Sg[c][a];
          f[c * NF + 1 + d] = t;
        }
      }
    }
    __syncthreads();
    // (B) this chunk's contribution to the test function of (cell sB, node iB)
    if (nB >= 0) {
      const T *fs = fq + (size_t)sB * QC * nc * NF;
      for (int qq = 0; qq < nqc; qq++) {
        const int q = q0 + qq;
        const T vi = v[q * D + iB];
        T gi[DIM];
#pragma unroll
        for (int d = 0; d < DIM; d++) gi[d] = g[(q * DIM + d) * D + iB];
#pragma unroll
        for (int c = 0; c < 3; c++)
          if (c < nc) {
            const T *f = fs + (qq * nc + c) * NF;
            T t = vi * f[0];
#pragma unroll
            for (int d = 0; d < DIM; d++) t += gi[d] * f[1 + d];
            acc[c] += t;
          }
      }
    }
  }
  // the scatter (constrained nodes never)
  if (nB >= 0)
#pragma unroll
    for (int c = 0; c < 3; c++) {
      if (c >= nc) break;
      T *yp = A.y + (int64_t)nB * nc + c;
      if (atomic) sd_atomic_add(yp, acc[c]);
      else *yp += acc[c];
    }
}

// Cells per workgroup and points per chunk: at most one (cell, node) pair per thread
// (CB D <= 256), at most 16 cells, and about 48 KB of LDS for the gathered values and
// one chunk of point fluxes (all points when they fit).
template <typename T> void simplex_dense_shape(int D, int nq, int ncomp, int dim, bool hyper, int &cb, int &qc) {
  const size_t budget = 48 * 1024, nf = (size_t)ncomp * (1 + dim);
  const size_t xper = ((size_t)D * ncomp + (hyper ? (size_t)D * 3 : 0)) * sizeof(T);
  cb = 256 / D;
  if (cb > 16) cb = 16;
  if (cb < 1) cb = 1;
  while (cb > 1 && cb * (xper + nf * sizeof(T) * (size_t)(nq < 16 ? nq : 16)) > budget) cb--;
  size_t room = budget > cb * xper ? (budget - cb * xper) / ((size_t)cb * nf * sizeof(T)) : 1;
  qc = (int)(room < (size_t)nq ? room : (size_t)nq);
  if (qc < 1) qc = 1;
}

template <typename T> int launch_simplex_dense(int dim, const SimplexDenseArgs<T> &a, bool atomic, hipStream_t s) {
  if (a.c1 <= a.c0) return MF_OK;
  if (a.ncomp < 1 || a.ncomp > 3) return fail(MF_EINVAL, "simplex dense kernel: ncomp");
  if (a.cb * a.D > 256 || a.qc < 1) return fail(MF_EINVAL, "simplex dense kernel: workgroup shape");
  const bool hyper = a.u0 != nullptr;
  if (hyper && (dim != 3 || a.ncomp != 3)) return fail(MF_EINVAL, "simplex dense kernel: hyperelastic on vector tets");
  const size_t lds = ((size_t)a.cb * a.D * a.ncomp + (hyper ? (size_t)a.cb * a.D * 3 : 0) +
                      (size_t)a.cb * a.qc * a.ncomp * (1 + dim)) * sizeof(T);
  if (lds > 64 * 1024) return fail(MF_EUNSUPPORTED, "simplex dense kernel: element too large for LDS");
  const int64_t nb = (a.c1 - a.c0 + a.cb - 1) / a.cb;
  const dim3 gr((unsigned)nb), bl(256);
  if (dim == 3 && hyper)
    simplex_dense_kernel<T, 3, true><<<gr, bl, lds, s>>>(a, atomic);
  else if (dim == 3)
    simplex_dense_kernel<T, 3, false><<<gr, bl, lds, s>>>(a, atomic);
  else
    simplex_dense_kernel<T, 2, false><<<gr, bl, lds, s>>>(a, atomic);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

template void simplex_dense_shape<double>(int, int, int, int, bool, int &, int &);
template void simplex_dense_shape<float>(int, int, int, int, bool, int &, int &);
template int launch_simplex_dense<double>(int, const SimplexDenseArgs<double> &, bool, hipStream_t);
template int launch_simplex_dense<float>(int, const SimplexDenseArgs<float> &, bool, hipStream_t);

}  // namespace mf
