// Operator action on bilinear quadrilaterals, Q_k (k = 1..6) on GLL nodes: the
// one-component forms and 2D linear elasticity.
//
// Quads are the 2D tensor-product cells of the paper's sweep (Section 4.1): the
// coordinate map is bilinear, so the Jacobian is evaluated at every quadrature point
// (Section 2.1), and the basis is a tensor product, so the interpolation to the points
// and the integration against the test functions factorise into 1D contractions
// (sum factorisation, Sections 3 and 4.2.4): two passes each way instead of a dense
// D x Q tabulation.
//
// GPU mapping: a workgroup is one 64-lane wavefront; lane p of a cell is quadrature
// point (a, b) = (p % nq, p / nq) of the nq x nq grid (nq <= 8), and 64 / nq^2 cells sit
// side by side in the wavefront (16 for Q1 with 2 x 2 points, one for Q6). Between the
// 1D passes the half-interpolated fields (lane (a, j): point a in x, node j in y) go
// through LDS. The gathered and scattered dof (i, j) of a cell is lane i + (k+1) j.
#include "mf_internal.h"

namespace mf {

namespace {
__device__ __forceinline__ void quad_atomic_add(double *p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void quad_atomic_add(float *p, float v) { unsafeAtomicAdd(p, v); }
}  // namespace

// Cell groups (64 / nq^2 cells side by side) per workgroup, run as a software pipeline.
constexpr int kQuadGroups = 8;

// N = k + 1 nodes and NQ Gauss points per direction. tab: B[a][i] = l_i(g_a) [NQ][N],
// B'[a][i] [NQ][N], weights [NQ], points [NQ]. atomic: device atomics for the scatter,
// else plain read-modify-write (the cells of one launch share no node). ELASTICITY has
// two components (node-interleaved dofs), the others one.
//
// A workgroup takes kQuadGroups consecutive cell groups. While group t is computed, the
// x values, geometry and coefficients of group t+1 and the map entries of group t+2
// are in flight, so the two dependent global loads of a group (map, then x) are hidden
// behind the arithmetic and LDS passes of the groups before it.
template <typename T, int N, int NQ, int KIND>
__global__ void __launch_bounds__(64) quad_kernel(const QuadArgs<T> A, const bool atomic) {
  constexpr int P = NQ * NQ, CPW = 64 / P, D = N * N, H = NQ * N;
  constexpr bool ELAS = KIND == MF_OP_ELASTICITY;
  constexpr int NC = ELAS ? 2 : 1;
  constexpr bool VAL = KIND == MF_OP_MASS || KIND == MF_OP_HELMHOLTZ;
  constexpr bool GRAD = KIND != MF_OP_MASS;
  constexpr bool COEF = KIND == MF_OP_MASS || KIND == MF_OP_POISSON;
  static_assert(NQ >= N && P <= 64, "one lane per point, and every dof has a lane");
  __shared__ T sB[H], sD[H], sw[NQ], sg[NQ];
  __shared__ T U[CPW][NC][D];                 // gathered dof values
  __shared__ T X0[CPW][NC][H], X1[CPW][NC][H];  // (a, j) fields, forward, then backward
  __shared__ T F0[CPW][P], F1[CPW][NC][P], F2[CPW][NC][P];  // value flux, reference fluxes
  const int lane = threadIdx.x;
  const int slot = lane / P, p = lane - slot * P;
  const bool act = slot < CPW;  // the last 64 mod P lanes idle
  // consecutive workgroup ids land on different XCDs: give each XCD a contiguous run of
  // cell groups (its L2 then holds the nodes its neighbouring cells share)
  const int64_t ngrp = (A.c1 - A.c0 + CPW - 1) / CPW, nwg = (ngrp + kQuadGroups - 1) / kQuadGroups;
  const int64_t per = (nwg + 7) / 8;
  const int64_t wg = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (wg >= nwg) return;  // uniform over the workgroup
  const int64_t gbase = wg * kQuadGroups;
  const int ng = (int)(ngrp - gbase < kQuadGroups ? ngrp - gbase : kQuadGroups);  // uniform
  if (lane < H) {
    sB[lane] = A.tab[lane];
    sD[lane] = A.tab[H + lane];
  }
  if (lane < NQ) {
    sw[lane] = A.tab[2 * H + lane];
    sg[lane] = A.tab[2 * H + NQ + lane];
  }
  // stage 1 of group t: is this lane's cell in the launch, and the node of its dof p
  auto load_map = [&](int t, bool &v, int &idx) {
    v = false;
    idx = -1;
    if (t < ng && act) {
      const int64_t cell = A.c0 + (gbase + t) * CPW + slot;
      v = cell < A.c1;
      if (v && A.cell_user) {
        const int64_t u = A.cell_user[cell];
        v = u >= A.ulo && u < A.uhi;
      }
      if (v && p < D) idx = A.map[cell * D + p];
    }
  };
  // stage 2: the dof values, the bilinear map x(xi, eta) = x0 + c1 xi + c2 eta + c3 xi eta
  // (c1, c2, c3 as (x, y) pairs) and the vertex coefficients; a lane without a cell takes
  // the unit square so that its discarded arithmetic stays finite
  auto load_data = [&](int t, bool v, int idx, T *xv, T *gm, T *cf) {
#pragma unroll
    for (int c = 0; c < NC; c++) xv[c] = idx >= 0 ? A.x[(int64_t)idx * NC + c] : T(0);
    gm[0] = T(1);
    gm[1] = T(0);
    gm[2] = T(0);
    gm[3] = T(1);
    gm[4] = T(0);
    gm[5] = T(0);
#pragma unroll
    for (int m = 0; m < 4; m++) cf[m] = T(1);
    if (v) {
      const int64_t cell = A.c0 + (gbase + t) * CPW + slot;
#pragma unroll
      for (int m = 0; m < 6; m++) gm[m] = A.geo[cell * 6 + m];
      if (COEF && A.coef)
#pragma unroll
        for (int m = 0; m < 4; m++) cf[m] = A.coef[cell * 4 + m];
    }
  };
  bool v0, v1;
  int i0, i1;
  T xv0[NC], gm0[6], cf0[4];
  load_map(0, v0, i0);
  load_data(0, v0, i0, xv0, gm0, cf0);
  load_map(1, v1, i1);
  for (int t = 0; t < ng; t++) {
    T xv1[NC], gm1[6], cf1[4];
    bool v2;
    int i2;
    load_data(t + 1, v1, i1, xv1, gm1, cf1);
    load_map(t + 2, v2, i2);
    __syncthreads();  // the previous group's last LDS reads are done
    if (act && p < D)
#pragma unroll
      for (int c = 0; c < NC; c++) U[slot][c][p] = xv0[c];
    __syncthreads();
    // forward x pass, lane (a, j): sum over nodes i in x
    if (act && p < H) {
      const int a = p % NQ, j = p / NQ;
#pragma unroll
      for (int c = 0; c < NC; c++) {
        T s0 = T(0), s1 = T(0);
#pragma unroll
        for (int i = 0; i < N; i++) {
          const T u = U[slot][c][i + N * j];
          s0 += sB[a * N + i] * u;
          if constexpr (GRAD) s1 += sD[a * N + i] * u;
        }
        X0[slot][c][p] = s0;
        if constexpr (GRAD) X1[slot][c][p] = s1;
      }
    }
    __syncthreads();
    // forward y pass and the pointwise fluxes, lane (a, b)
    if (act) {
      const int a = p % NQ, b = p / NQ;
      T u = T(0), gx[NC], gy[NC];  // value and reference gradients at the point
#pragma unroll
      for (int c = 0; c < NC; c++) gx[c] = gy[c] = T(0);
#pragma unroll
      for (int j = 0; j < N; j++) {
#pragma unroll
        for (int c = 0; c < NC; c++) {
          const T x0 = X0[slot][c][a + NQ * j];
          if constexpr (VAL) u += sB[b * N + j] * x0;
          if constexpr (GRAD) {
            gx[c] += sB[b * N + j] * X1[slot][c][a + NQ * j];
            gy[c] += sD[b * N + j] * x0;
          }
        }
      }
      const T xi = sg[a], eta = sg[b];
      // J[r][c] = d x_r / d xi_c
      const T J00 = gm0[0] + gm0[4] * eta, J01 = gm0[2] + gm0[4] * xi;
      const T J10 = gm0[1] + gm0[5] * eta, J11 = gm0[3] + gm0[5] * xi;
      const T det = J00 * J11 - J01 * J10;
      const T wdet = sw[a] * sw[b] * (det < T(0) ? -det : det);
      T cq = T(1);
      if (COEF && A.coef)
        cq = (T(1) - xi) * (T(1) - eta) * cf0[0] + xi * (T(1) - eta) * cf0[1] + (T(1) - xi) * eta * cf0[2] +
             xi * eta * cf0[3];
      T f0 = T(0), P0[NC], P1[NC];
      if constexpr (VAL) f0 = wdet * (KIND == MF_OP_MASS ? cq : T(1)) * u;
      if constexpr (GRAD) {
        // J^{-1} = [[J11, -J01], [-J10, J00]] / det; physical gradient G_a = sum_b
        // (J^{-1})[b][a] g_b, then the reference-direction flux P_b = s sum_a
        // (J^{-1})[b][a] S_a of the physical flux S (the gradient, kappa times it, or
        // the stress)
        const T r = T(1) / det;
        T G[NC][2];
#pragma unroll
        for (int c = 0; c < NC; c++) {
          G[c][0] = (J11 * gx[c] - J10 * gy[c]) * r;
          G[c][1] = (J00 * gy[c] - J01 * gx[c]) * r;
        }
        T S[NC][2];
        if constexpr (ELAS) {
          // sigma = lambda tr(grad u) I + mu (grad u + grad u^T)
          const T tr = A.lam * (G[0][0] + G[1][1]), od = A.mu * (G[0][1] + G[1][0]);
          S[0][0] = tr + T(2) * A.mu * G[0][0];
          S[1][1] = tr + T(2) * A.mu * G[1][1];
          S[0][1] = od;
          S[1][0] = od;
        } else {
          S[0][0] = G[0][0];
          S[0][1] = G[0][1];
        }
        const T sc = wdet * (KIND == MF_OP_POISSON ? cq : T(1)) * r;
#pragma unroll
        for (int c = 0; c < NC; c++) {
          P0[c] = sc * (J11 * S[c][0] - J01 * S[c][1]);
          P1[c] = sc * (J00 * S[c][1] - J10 * S[c][0]);
        }
      }
      F0[slot][p] = f0;
      if constexpr (GRAD)
#pragma unroll
        for (int c = 0; c < NC; c++) {
          F1[slot][c][p] = P0[c];
          F2[slot][c][p] = P1[c];
        }
    }
    __syncthreads();
    // backward y pass, lane (a, j): integrate against the test functions in y
    if (act && p < H) {
      const int a = p % NQ, j = p / NQ;
#pragma unroll
      for (int c = 0; c < NC; c++) {
        T y0 = T(0), y1 = T(0);
#pragma unroll
        for (int b = 0; b < NQ; b++) {
          const int q = a + NQ * b;
          if constexpr (VAL) y0 += sB[b * N + j] * F0[slot][q];
          if constexpr (GRAD) {
            y0 += sD[b * N + j] * F2[slot][c][q];
            y1 += sB[b * N + j] * F1[slot][c][q];
          }
        }
        X0[slot][c][p] = y0;
        if constexpr (GRAD) X1[slot][c][p] = y1;
      }
    }
    __syncthreads();
    // backward x pass, lane (i, j), and the scatter
    if (act && p < D && i0 >= 0) {
      const int i = p % N, j = p / N;
#pragma unroll
      for (int c = 0; c < NC; c++) {
        T v = T(0);
#pragma unroll
        for (int a = 0; a < NQ; a++) {
          v += sB[a * N + i] * X0[slot][c][a + NQ * j];
          if constexpr (GRAD) v += sD[a * N + i] * X1[slot][c][a + NQ * j];
        }
        T *yp = A.y + (int64_t)i0 * NC + c;
        if (atomic) quad_atomic_add(yp, v);
        else *yp += v;
      }
    }
    v0 = v1;
    i0 = i1;
#pragma unroll
    for (int c = 0; c < NC; c++) xv0[c] = xv1[c];
#pragma unroll
    for (int m = 0; m < 6; m++) gm0[m] = gm1[m];
#pragma unroll
    for (int m = 0; m < 4; m++) cf0[m] = cf1[m];
    v1 = v2;
    i1 = i2;
  }
}

// diag(A) on quads: a(phi_d e_c, phi_d e_c) for every dof, sum-factorised. At point
// (a, b) the form restricted to one basis function is m phi^2 + g^T C g with g the
// reference gradient (B'_ai B_bj, B_ai B'_bj) of phi = B_ai B_bj: m = w |det| (c), and
// C = w |det| s J^{-1} J^{-T} (s = kappa or 1), or for elasticity component c
// w |det| (mu J^{-1} J^{-T} + (mu + lambda) k k^T) with k the column c of J^{-1}. The
// sum over b is taken per (a, j), then over a per node (i, j). One workgroup per group
// of 64 / nq^2 cells, lane = point, atomics for the shared nodes.
template <typename T, int N, int NQ, int KIND>
__global__ void __launch_bounds__(64) quad_diag_kernel(const QuadArgs<T> A) {
  constexpr int P = NQ * NQ, CPW = 64 / P, D = N * N, H = NQ * N;
  constexpr bool ELAS = KIND == MF_OP_ELASTICITY;
  constexpr int NC = ELAS ? 2 : 1;
  constexpr bool VAL = KIND == MF_OP_MASS || KIND == MF_OP_HELMHOLTZ;
  constexpr bool GRAD = KIND != MF_OP_MASS;
  constexpr bool COEF = KIND == MF_OP_MASS || KIND == MF_OP_POISSON;
  __shared__ T sB[H], sD[H], sw[NQ], sg[NQ];
  __shared__ T Cq[CPW][NC][4][P];  // m, C00, C01, C11 per point
  __shared__ T Tq[CPW][NC][4][H];  // their sums over b against the y factors, per (a, j)
  const int lane = threadIdx.x;
  const int slot = lane / P, p = lane - slot * P;
  const bool act = slot < CPW;
  const int64_t ngrp = (A.c1 - A.c0 + CPW - 1) / CPW, per = (ngrp + 7) / 8;
  const int64_t grp = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (grp >= ngrp) return;  // uniform over the workgroup
  const int64_t cell = A.c0 + grp * CPW + slot;
  const bool valid = act && cell < A.c1;
  if (lane < H) {
    sB[lane] = A.tab[lane];
    sD[lane] = A.tab[H + lane];
  }
  if (lane < NQ) {
    sw[lane] = A.tab[2 * H + lane];
    sg[lane] = A.tab[2 * H + NQ + lane];
  }
  T gm[6] = {T(1), T(0), T(0), T(1), T(0), T(0)}, cf[4] = {T(1), T(1), T(1), T(1)};
  if (valid) {
#pragma unroll
    for (int m = 0; m < 6; m++) gm[m] = A.geo[cell * 6 + m];
    if (COEF && A.coef)
#pragma unroll
      for (int m = 0; m < 4; m++) cf[m] = A.coef[cell * 4 + m];
  }
  __syncthreads();
  if (act) {
    const int a = p % NQ, b = p / NQ;
    const T xi = sg[a], eta = sg[b];
    const T J00 = gm[0] + gm[4] * eta, J01 = gm[2] + gm[4] * xi;
    const T J10 = gm[1] + gm[5] * eta, J11 = gm[3] + gm[5] * xi;
    const T det = J00 * J11 - J01 * J10;
    const T wdet = sw[a] * sw[b] * (det < T(0) ? -det : det);
    T cq = T(1);
    if (COEF && A.coef)
      cq = (T(1) - xi) * (T(1) - eta) * cf[0] + xi * (T(1) - eta) * cf[1] + (T(1) - xi) * eta * cf[2] +
           xi * eta * cf[3];
    const T rd = T(1) / det;
    // rows of J^{-1}: k0 = (J11, -J01) / det, k1 = (-J10, J00) / det
    const T k00 = J11 * rd, k01 = -J01 * rd, k10 = -J10 * rd, k11 = J00 * rd;
    const T G00 = k00 * k00 + k01 * k01, G01 = k00 * k10 + k01 * k11, G11 = k10 * k10 + k11 * k11;
#pragma unroll
    for (int c = 0; c < NC; c++) {
      T m = T(0), c00 = T(0), c01 = T(0), c11 = T(0);
      if constexpr (VAL) m = wdet * (KIND == MF_OP_MASS ? cq : T(1));
      if constexpr (GRAD) {
        if constexpr (ELAS) {
          const T q0 = c == 0 ? k00 : k01, q1 = c == 0 ? k10 : k11;  // column c of J^{-1}
          const T e = A.mu + A.lam;
          c00 = wdet * (A.mu * G00 + e * q0 * q0);
          c01 = wdet * (A.mu * G01 + e * q0 * q1);
          c11 = wdet * (A.mu * G11 + e * q1 * q1);
        } else {
          const T sc = wdet * (KIND == MF_OP_POISSON ? cq : T(1));
          c00 = sc * G00;
          c01 = sc * G01;
          c11 = sc * G11;
        }
      }
      Cq[slot][c][0][p] = m;
      Cq[slot][c][1][p] = c00;
      Cq[slot][c][2][p] = c01;
      Cq[slot][c][3][p] = c11;
    }
  }
  __syncthreads();
  // lane (a, j): T0 = sum_b (m + C00 ...) split by which factor carries the derivative
  // in y: B_bj^2 multiplies m and C00, B_bj B'_bj multiplies C01, B'_bj^2 multiplies C11
  if (act && p < H) {
    const int a = p % NQ, j = p / NQ;
#pragma unroll
    for (int c = 0; c < NC; c++) {
      T t0 = T(0), t1 = T(0), t2 = T(0), t3 = T(0);
#pragma unroll
      for (int b = 0; b < NQ; b++) {
        const int q = a + NQ * b;
        const T bb = sB[b * N + j], db = sD[b * N + j];
        t0 += bb * bb * Cq[slot][c][0][q];
        t1 += bb * bb * Cq[slot][c][1][q];
        t2 += bb * db * Cq[slot][c][2][q];
        t3 += db * db * Cq[slot][c][3][q];
      }
      Tq[slot][c][0][p] = t0;
      Tq[slot][c][1][p] = t1;
      Tq[slot][c][2][p] = t2;
      Tq[slot][c][3][p] = t3;
    }
  }
  __syncthreads();
  // lane (i, j): sum over a with B_ai^2 (value and C11), B'_ai^2 (C00), 2 B_ai B'_ai (C01)
  if (valid && p < D) {
    const int idx = A.map[cell * D + p];
    if (idx >= 0) {
      const int i = p % N, j = p / N;
#pragma unroll
      for (int c = 0; c < NC; c++) {
        T v = T(0);
#pragma unroll
        for (int a = 0; a < NQ; a++) {
          const T ba = sB[a * N + i], da = sD[a * N + i];
          const int h = a + NQ * j;
          v += ba * ba * (Tq[slot][c][0][h] + Tq[slot][c][3][h]) + da * da * Tq[slot][c][1][h] +
               T(2) * ba * da * Tq[slot][c][2][h];
        }
        quad_atomic_add(A.y + (int64_t)idx * NC + c, v);
      }
    }
  }
}

template <typename T, int N, int NQ, int KIND>
static int launch_quad_diag_nk(const QuadArgs<T> &a, hipStream_t s) {
  constexpr int CPW = 64 / (NQ * NQ);
  const int64_t ngrp = (a.c1 - a.c0 + CPW - 1) / CPW;
  const dim3 g((unsigned)(((ngrp + 7) / 8) * 8)), b(64);
  quad_diag_kernel<T, N, NQ, KIND><<<g, b, 0, s>>>(a);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

template <typename T, int N, int NQ, int KIND>
static int launch_quad_nk(const QuadArgs<T> &a, bool atomic, hipStream_t s) {
  constexpr int CPW = 64 / (NQ * NQ);
  const int64_t ngrp = (a.c1 - a.c0 + CPW - 1) / CPW, nwg = (ngrp + kQuadGroups - 1) / kQuadGroups;
  const dim3 g((unsigned)(((nwg + 7) / 8) * 8)), b(64);
  quad_kernel<T, N, NQ, KIND><<<g, b, 0, s>>>(a, atomic);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

template <typename T, int N, int NQ>
static int launch_quad_nq(int kind, const QuadArgs<T> &a, bool atomic, bool diag, hipStream_t s) {
  if (diag) {
    switch (kind) {
      case MF_OP_MASS: return launch_quad_diag_nk<T, N, NQ, MF_OP_MASS>(a, s);
      case MF_OP_HELMHOLTZ: return launch_quad_diag_nk<T, N, NQ, MF_OP_HELMHOLTZ>(a, s);
      case MF_OP_LAPLACIAN: return launch_quad_diag_nk<T, N, NQ, MF_OP_LAPLACIAN>(a, s);
      case MF_OP_POISSON: return launch_quad_diag_nk<T, N, NQ, MF_OP_POISSON>(a, s);
      case MF_OP_ELASTICITY: return launch_quad_diag_nk<T, N, NQ, MF_OP_ELASTICITY>(a, s);
    }
    return fail(MF_EUNSUPPORTED, "quad operator kind");
  }
  switch (kind) {
    case MF_OP_MASS: return launch_quad_nk<T, N, NQ, MF_OP_MASS>(a, atomic, s);
    case MF_OP_HELMHOLTZ: return launch_quad_nk<T, N, NQ, MF_OP_HELMHOLTZ>(a, atomic, s);
    case MF_OP_LAPLACIAN: return launch_quad_nk<T, N, NQ, MF_OP_LAPLACIAN>(a, atomic, s);
    case MF_OP_POISSON: return launch_quad_nk<T, N, NQ, MF_OP_POISSON>(a, atomic, s);
    case MF_OP_ELASTICITY: return launch_quad_nk<T, N, NQ, MF_OP_ELASTICITY>(a, atomic, s);
  }
  return fail(MF_EUNSUPPORTED, "quad operator kind");
}

template <typename T, int N>
static int launch_quad_n(int nq, int kind, const QuadArgs<T> &a, bool atomic, bool diag, hipStream_t s) {
  if (nq == N) return launch_quad_nq<T, N, N>(kind, a, atomic, diag, s);
  if constexpr (N < 8)
    if (nq == N + 1) return launch_quad_nq<T, N, N + 1>(kind, a, atomic, diag, s);
  return fail(MF_EUNSUPPORTED, "quad: nq1d must be k+1 or k+2 (at most 8)");
}

template <typename T>
int launch_quad(int k, int nq, int kind, const QuadArgs<T> &a, bool atomic, hipStream_t s, bool diag) {
  if (a.c1 <= a.c0) return MF_OK;
  switch (k) {
    case 1: return launch_quad_n<T, 2>(nq, kind, a, atomic, diag, s);
    case 2: return launch_quad_n<T, 3>(nq, kind, a, atomic, diag, s);
    case 3: return launch_quad_n<T, 4>(nq, kind, a, atomic, diag, s);
    case 4: return launch_quad_n<T, 5>(nq, kind, a, atomic, diag, s);
    case 5: return launch_quad_n<T, 6>(nq, kind, a, atomic, diag, s);
    case 6: return launch_quad_n<T, 7>(nq, kind, a, atomic, diag, s);
  }
  return fail(MF_EUNSUPPORTED, "quad degree (1..6)");
}

template int launch_quad<double>(int, int, int, const QuadArgs<double> &, bool, hipStream_t, bool);
template int launch_quad<float>(int, int, int, const QuadArgs<float> &, bool, hipStream_t, bool);

}  // namespace mf
