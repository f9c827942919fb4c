// Scalar operators (mass, Helmholtz, Laplacian with one or three components, Poisson)
// on trilinear hexahedra with the paper's quadrature of k+2 Gauss points per direction
// (Table 2's hex rows count Q = k + 2), where the points outnumber the nodes and the
// pencil kernel's one-lane-per-node-line mapping does not apply.
//
// The basis is a tensor product, so the action factorises into 1D contractions
// (Sections 3 and 4.2.4) with the rectangular q x n tables B = l_i(g_a) and
// B' = l_i'(g_a): forward x, y and z passes give the value (mass terms) and the three
// reference derivatives at every point, the pointwise stage evaluates the Jacobian of
// the trilinear map there (Section 2.1) and forms the reference fluxes, and the
// transposed passes integrate against the test basis. A thread per quadrature point
// (the layout of the elasticity kernel): one cell per workgroup of q^3 threads rounded
// up to wavefronts, or 64 / q^3 cells per wavefront when q^3 <= 32; partial
// contractions sit in two LDS buffers per cell. Components are processed in turn.
#include "mf_internal.h"

namespace mf {

namespace {
__device__ __forceinline__ void hexq_atomic_add(double *p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void hexq_atomic_add(float *p, float v) { unsafeAtomicAdd(p, v); }
}  // namespace

template <typename T, int N, int NQ, int KIND>
__global__ void __launch_bounds__(512) hex_q_kernel(const HexQArgs<T> A, const bool atomic) {
  constexpr bool GRAD = KIND != MF_OP_MASS;
  constexpr bool MASS = KIND == MF_OP_MASS || KIND == MF_OP_HELMHOLTZ;
  constexpr bool COEF = KIND == MF_OP_MASS || KIND == MF_OP_POISSON;
  constexpr int D = N * N * N, SX = NQ * N * N, SY = NQ * NQ * N, P = NQ * NQ * NQ, H = NQ * N;
  constexpr int CPB = P <= 32 ? 64 / P : 1;
  constexpr int LA = (3 * SY > D ? 3 * SY : D), LB = (2 * SX > 4 * P ? 2 * SX : 4 * P);
  static_assert(NQ >= N, "every node needs a thread");
  __shared__ T sB[H], sD[H], sw[NQ], sg[NQ];
  __shared__ T bufA[CPB][LA];
  __shared__ T bufB[CPB][LB];
  const int tid = threadIdx.x;
  const int slot = tid / P, t = tid - slot * P;
  const bool act = slot < CPB;
  const int64_t ngrp = (A.c1 - A.c0 + CPB - 1) / CPB, per = (ngrp + 7) / 8;
  const int64_t gi0 = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;  // contiguous runs per XCD
  if (gi0 >= ngrp) return;  // uniform over the workgroup
  const int64_t cell = A.c0 + gi0 * CPB + slot;
  bool valid = act && cell < A.c1;
  if (valid && A.cell_user) {
    const int64_t u = A.cell_user[cell];
    valid = u >= A.ulo && u < A.uhi;
  }
  if (tid < H) {
    sB[tid] = A.tab[tid];
    sD[tid] = A.tab[H + tid];
  }
  if (tid < NQ) {
    sw[tid] = A.tab[2 * H + tid];
    sg[tid] = A.tab[2 * H + NQ + tid];
  }
  int idx = -1, gi = -1;  // node of dof t in y, and its position in x
  if (act && t < D && valid) {
    idx = A.map[cell * D + t];
    gi = A.gmap ? A.gmap[cell * D + t] : idx;
  }
  const int nc = A.ncomp;
  // geometry of this thread's point (a, b, e); a thread of an empty slot takes the
  // unit cube so that its discarded arithmetic stays finite
  T C[3][3], det = T(1), kq = T(1), wq = T(0);
  const bool gv = (CPB == 1 && act) || valid;
  if (act && t < P) {
    const int a = t % NQ, b = (t / NQ) % NQ, e = t / (NQ * NQ);
    const T x1 = A.tab[2 * H + NQ + a], x2 = A.tab[2 * H + NQ + b], x3 = A.tab[2 * H + NQ + e];
    wq = A.tab[2 * H + a] * A.tab[2 * H + b] * A.tab[2 * H + e];
    T J[3][3];
    const int64_t cg = gv ? cell : 0;
#pragma unroll
    for (int r = 0; r < 3; r++) {
      const T *gc = A.geo + cg * 24;
      const T c1 = gv ? gc[r] : T(r == 0), c2 = gv ? gc[3 + r] : T(r == 1), c3 = gv ? gc[6 + r] : T(r == 2),
              c4 = gv ? gc[9 + r] : T(0), c5 = gv ? gc[12 + r] : T(0), c6 = gv ? gc[15 + r] : T(0),
              c7 = gv ? gc[18 + r] : T(0);
      J[r][0] = c1 + c4 * x2 + c5 * x3 + c7 * x2 * x3;
      J[r][1] = c2 + c4 * x1 + c6 * x3 + c7 * x1 * x3;
      J[r][2] = c3 + c5 * x1 + c6 * x2 + c7 * x1 * x2;
    }
    C[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    C[0][1] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    C[0][2] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    C[1][0] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    C[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    C[1][2] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    C[2][0] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    C[2][1] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    C[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    det = J[0][0] * C[0][0] + J[0][1] * C[0][1] + J[0][2] * C[0][2];
    if (COEF && A.coef && gv) {
      const T *K = A.coef + cg * 8;
      kq = K[0] + K[1] * x1 + K[2] * x2 + K[3] * x3 + K[4] * x1 * x2 + K[5] * x1 * x3 + K[6] * x2 * x3 +
           K[7] * x1 * x2 * x3;
    }
  }
  __syncthreads();  // tables in LDS
  for (int c = 0; c < nc; c++) {
    if (act && t < D) bufA[slot][t] = gi >= 0 ? A.x[(int64_t)gi * nc + c] : T(0);
    __syncthreads();
    // x pass, thread (a, j, l): X0 = B_x U, X1 = B'_x U
    if (act && t < SX) {
      const int a = t % NQ, j = (t / NQ) % N, l = t / (NQ * N);
      T s0 = T(0), s1 = T(0);
#pragma unroll
      for (int i = 0; i < N; i++) {
        const T u = bufA[slot][i + N * (j + N * l)];
        s0 += sB[a * N + i] * u;
        if constexpr (GRAD) s1 += sD[a * N + i] * u;
      }
      bufB[slot][t] = s0;
      if constexpr (GRAD) bufB[slot][SX + t] = s1;
    }
    __syncthreads();
    // y pass, thread (a, b, l): Y00 = B_y X0, Y01 = B'_y X0, Y10 = B_y X1
    if (act && t < SY) {
      const int a = t % NQ, b = (t / NQ) % NQ, l = t / (NQ * NQ);
      T y00 = T(0), y01 = T(0), y10 = T(0);
#pragma unroll
      for (int j = 0; j < N; j++) {
        const T x0 = bufB[slot][a + NQ * (j + N * l)];
        y00 += sB[b * N + j] * x0;
        if constexpr (GRAD) {
          y01 += sD[b * N + j] * x0;
          y10 += sB[b * N + j] * bufB[slot][SX + a + NQ * (j + N * l)];
        }
      }
      bufA[slot][t] = y00;
      if constexpr (GRAD) {
        bufA[slot][SY + t] = y01;
        bufA[slot][2 * SY + t] = y10;
      }
    }
    __syncthreads();
    // z pass and the pointwise fluxes, thread = point (a, b, e)
    if (act && t < P) {
      const int a = t % NQ, b = (t / NQ) % NQ, e = t / (NQ * NQ);
      T u = T(0), g0 = T(0), g1 = T(0), g2 = T(0);
#pragma unroll
      for (int l = 0; l < N; l++) {
        const int h = a + NQ * (b + NQ * l);
        const T y00 = bufA[slot][h];
        if constexpr (MASS) u += sB[e * N + l] * y00;
        if constexpr (GRAD) {
          g0 += sB[e * N + l] * bufA[slot][2 * SY + h];
          g1 += sB[e * N + l] * bufA[slot][SY + h];
          g2 += sD[e * N + l] * y00;
        }
      }
      const T adet = det < T(0) ? -det : det;
      if constexpr (GRAD) {
        // physical gradient Gp[r] = sum_d C[r][d] g_d / det; reference flux
        // F[d] = w |det| kappa / det sum_r C[r][d] Gp[r]
        const T rd = T(1) / det;
        T Gp[3];
#pragma unroll
        for (int r = 0; r < 3; r++) Gp[r] = (C[r][0] * g0 + C[r][1] * g1 + C[r][2] * g2) * rd;
        const T s = wq * adet * rd * (KIND == MF_OP_POISSON ? kq : T(1));
#pragma unroll
        for (int d = 0; d < 3; d++) bufB[slot][d * P + t] = s * (C[0][d] * Gp[0] + C[1][d] * Gp[1] + C[2][d] * Gp[2]);
      }
      if constexpr (MASS) bufB[slot][3 * P + t] = wq * adet * (KIND == MF_OP_MASS ? kq : T(1)) * u;
    }
    __syncthreads();
    // backward z, thread (a, b, l): Zx = B_z F0, Zy = B_z F1, Zz = B'_z F2 + B_z M
    if (act && t < SY) {
      const int a = t % NQ, b = (t / NQ) % NQ, l = t / (NQ * NQ);
      T zx = T(0), zy = T(0), zz = T(0);
#pragma unroll
      for (int e = 0; e < NQ; e++) {
        const int q = a + NQ * (b + NQ * e);
        if constexpr (GRAD) {
          zx += sB[e * N + l] * bufB[slot][q];
          zy += sB[e * N + l] * bufB[slot][P + q];
          zz += sD[e * N + l] * bufB[slot][2 * P + q];
        }
        if constexpr (MASS) zz += sB[e * N + l] * bufB[slot][3 * P + q];
      }
      bufA[slot][t] = zx;
      bufA[slot][SY + t] = zy;
      bufA[slot][2 * SY + t] = zz;
    }
    __syncthreads();
    // backward y, thread (a, j, l): Vx = B_y Zx, Vb = B'_y Zy + B_y Zz
    if (act && t < SX) {
      const int a = t % NQ, j = (t / NQ) % N, l = t / (NQ * N);
      T vx = T(0), vb = T(0);
#pragma unroll
      for (int b = 0; b < NQ; b++) {
        const int h = a + NQ * (b + NQ * l);
        if constexpr (GRAD) {
          vx += sB[b * N + j] * bufA[slot][h];
          vb += sD[b * N + j] * bufA[slot][SY + h];
        }
        vb += sB[b * N + j] * bufA[slot][2 * SY + h];
      }
      bufB[slot][t] = vx;
      bufB[slot][SX + t] = vb;
    }
    __syncthreads();
    // backward x, thread (i, j, l): v = B'_x Vx + B_x Vb, and the scatter
    if (act && t < D && idx >= 0) {
      const int i = t % N, j = (t / N) % N, l = t / (N * N);
      T v = T(0);
#pragma unroll
      for (int a = 0; a < NQ; a++) {
        const int h = a + NQ * (j + N * l);
        if constexpr (GRAD) v += sD[a * N + i] * bufB[slot][h];
        v += sB[a * N + i] * bufB[slot][SX + h];
      }
      T *yp = A.y + (int64_t)idx * nc + c;
      if (atomic) hexq_atomic_add(yp, v);
      else *yp += v;  // cells of one launch share no node
    }
    __syncthreads();  // the buffers are reused by the next component
  }
}

template <typename T, int N, int NQ>
static int launch_hexq_nq(int kind, const HexQArgs<T> &a, bool atomic, hipStream_t s) {
  constexpr int P = NQ * NQ * NQ, CPB = P <= 32 ? 64 / P : 1;
  const int64_t ngrp = (a.c1 - a.c0 + CPB - 1) / CPB;
  const dim3 g((unsigned)(((ngrp + 7) / 8) * 8)), b((unsigned)(CPB > 1 ? 64 : (P + 63) / 64 * 64));
  switch (kind) {
    case MF_OP_MASS: hex_q_kernel<T, N, NQ, MF_OP_MASS><<<g, b, 0, s>>>(a, atomic); break;
    case MF_OP_HELMHOLTZ: hex_q_kernel<T, N, NQ, MF_OP_HELMHOLTZ><<<g, b, 0, s>>>(a, atomic); break;
    case MF_OP_LAPLACIAN: hex_q_kernel<T, N, NQ, MF_OP_LAPLACIAN><<<g, b, 0, s>>>(a, atomic); break;
    case MF_OP_POISSON: hex_q_kernel<T, N, NQ, MF_OP_POISSON><<<g, b, 0, s>>>(a, atomic); break;
    default: return fail(MF_EUNSUPPORTED, "hex (k+2 points): operator kind");
  }
  MF_HIP(hipGetLastError());
  return MF_OK;
}

template <typename T>
int launch_hex_q(int k, int nq, int kind, const HexQArgs<T> &a, bool atomic, hipStream_t s) {
  if (a.c1 <= a.c0) return MF_OK;
  if (nq != k + 2 || nq > 7) return fail(MF_EUNSUPPORTED, "hex scalar operators: nq1d must be k+1 or k+2 (<= 7)");
  switch (k) {
    case 1: return launch_hexq_nq<T, 2, 3>(kind, a, atomic, s);
    case 2: return launch_hexq_nq<T, 3, 4>(kind, a, atomic, s);
    case 3: return launch_hexq_nq<T, 4, 5>(kind, a, atomic, s);
    case 4: return launch_hexq_nq<T, 5, 6>(kind, a, atomic, s);
    case 5: return launch_hexq_nq<T, 6, 7>(kind, a, atomic, s);
  }
  return fail(MF_EUNSUPPORTED, "hex scalar operators with k+2 points: degree 1..5");
}

template int launch_hex_q<double>(int, int, int, const HexQArgs<double> &, bool, hipStream_t);
template int launch_hex_q<float>(int, int, int, const HexQArgs<float> &, bool, hipStream_t);

}  // namespace mf
