// Linear elasticity on trilinear hexahedra, Q1..Q6 on GLL nodes, three node-interleaved
// components: int sigma(u) : grad v with sigma = lambda tr(grad u) I + mu (grad u +
// grad u^T) (the paper's vector operator on the tensor-product cell, Section 4.1), and
// the St-Venant-Kirchhoff tangent at a displacement u0 (supplementary operator list:
// F = I + grad u0, E = (F^T F - I)/2, S = lambda tr(E) I + 2 mu E; the Gateaux
// derivative of int F S : grad v in the direction u is int (grad u S + F dS) : grad v
// with dS = S(dE), dE = (grad u^T F + F^T grad u)/2).
//
// The basis is a tensor product, so the action factorises into 1D contractions
// (Sections 3 and 4.2.4): three passes forward (values and reference gradients of each
// component at the points), the pointwise stress with the Jacobian of the trilinear map
// evaluated at every point (Section 2.1), and three passes back. A thread per quadrature
// point; one cell per workgroup (rounded up to whole wavefronts), or 64 / nq^3 cells in
// one wavefront when a cell has at most 32 points (Q1: 8, Q2: 2); between the passes the
// partial contractions sit in two ping-pong LDS buffers per cell (70 KB in FP64 for Q6
// with 8 points: within gfx950's 160 KB per workgroup, two workgroups per CU).
#include "mf_internal.h"

namespace mf {

namespace {
__device__ __forceinline__ void hex_el_atomic_add(double *p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void hex_el_atomic_add(float *p, float v) { unsafeAtomicAdd(p, v); }

// Forward passes of one cell: the three components' nodal values in bA [3][n^3] give
// their reference gradients g[c][d] at this thread's point (t < q^3; zeros elsewhere).
// Contains workgroup barriers: every thread of the workgroup calls it.
template <typename T, int N, int NQ>
__device__ __forceinline__ void hex_el_forward(T *bA, T *bB, const T *sB, const T *sD, const bool act, const int t,
                                               T (&g)[3][3]) {
  constexpr int D = N * N * N, SX = NQ * N * N, SY = NQ * NQ * N, P = NQ * NQ * NQ;
  // x pass, thread (a, j, l): X0 = sum_i B[a][i] U[i, j, l], X1 with B'
  if (act && t < SX) {
    const int a = t % NQ, j = (t / NQ) % N, l = t / (NQ * N);
#pragma unroll
    for (int c = 0; c < 3; c++) {
      T s0 = T(0), s1 = T(0);
#pragma unroll
      for (int i = 0; i < N; i++) {
        const T u = bA[c * D + i + N * (j + N * l)];
        s0 += sB[a * N + i] * u;
        s1 += sD[a * N + i] * u;
      }
      bB[c * SX + t] = s0;
      bB[(3 + c) * SX + t] = s1;
    }
  }
  __syncthreads();
  // y pass, thread (a, b, l): Y00 = B_y X0, Y01 = B'_y X0, Y10 = B_y X1
  if (act && t < SY) {
    const int a = t % NQ, b = (t / NQ) % NQ, l = t / (NQ * NQ);
#pragma unroll
    for (int c = 0; c < 3; c++) {
      T y00 = T(0), y01 = T(0), y10 = T(0);
#pragma unroll
      for (int j = 0; j < N; j++) {
        const T x0 = bB[c * SX + a + NQ * (j + N * l)], x1 = bB[(3 + c) * SX + a + NQ * (j + N * l)];
        y00 += sB[b * N + j] * x0;
        y01 += sD[b * N + j] * x0;
        y10 += sB[b * N + j] * x1;
      }
      bA[c * SY + t] = y00;
      bA[(3 + c) * SY + t] = y01;
      bA[(6 + c) * SY + t] = y10;
    }
  }
  __syncthreads();
  // z pass, thread = point (a, b, e): g[c][d], reference derivative d of component c
#pragma unroll
  for (int c = 0; c < 3; c++) g[c][0] = g[c][1] = g[c][2] = T(0);
  if (act && t < P) {
    const int a = t % NQ, b = (t / NQ) % NQ, e = t / (NQ * NQ);
#pragma unroll
    for (int c = 0; c < 3; c++) {
      T gx = T(0), gy = T(0), gz = T(0);
#pragma unroll
      for (int l = 0; l < N; l++) {
        const int h = a + NQ * (b + NQ * l);
        gx += sB[e * N + l] * bA[(6 + c) * SY + h];
        gy += sB[e * N + l] * bA[(3 + c) * SY + h];
        gz += sD[e * N + l] * bA[c * SY + h];
      }
      g[c][0] = gx;
      g[c][1] = gy;
      g[c][2] = gz;
    }
  }
}
}  // namespace

// N = k + 1 nodes and NQ Gauss points per direction. tab: B[a][i] = l_i(g_a) [NQ][N],
// B'[a][i], weights [NQ], points [NQ]. geo: [cell][24], coefficient m = 1..7 of the
// trilinear map x = c0 + c1 xi1 + c2 xi2 + c3 xi3 + c4 xi1 xi2 + c5 xi1 xi3 + c6 xi2 xi3
// + c7 xi1 xi2 xi3 at 3 (m - 1) + coordinate.
template <typename T, int N, int NQ, bool HYPER>
__global__ void __launch_bounds__(512) hex_elasticity_kernel(const HexElasArgs<T> A, const bool atomic) {
  constexpr int D = N * N * N, SX = NQ * N * N, SY = NQ * NQ * N, P = NQ * NQ * NQ, H = NQ * N;
  constexpr int CPB = P <= 32 ? 64 / P : 1;  // cells per workgroup (Q1: 8, Q2: 2)
  static_assert(NQ >= N, "every node needs a thread");
  __shared__ T sB[H], sD[H], sw[NQ], sg[NQ];
  __shared__ T bufA[CPB][9 * SY];  // dofs, then the y-pass fields, then the backward z fields
  __shared__ T bufB[CPB][9 * P];   // x-pass fields, then the point fluxes, then the backward y fields
  const int tid = threadIdx.x;
  const int slot = tid / P, t = tid - slot * P;  // cell of the workgroup, thread within it
  const bool act = slot < CPB;
  // consecutive workgroup ids land on different XCDs: each XCD takes a contiguous run
  const int64_t ngrp = (A.c1 - A.c0 + CPB - 1) / CPB, per = (ngrp + 7) / 8;
  const int64_t gi0 = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
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
  int idx = -1, gi = -1, gu = -1;  // node of dof t in y (internal numbering), in x, in u0
  if (act && t < D && valid) {
    idx = A.map[cell * D + t];
    gi = A.gmap ? A.gmap[cell * D + t] : idx;
    if constexpr (HYPER) gu = A.u0map ? A.u0map[cell * D + t] : idx;
  }
  T g0[3][3];  // reference gradient of u0 at this thread's point (HYPER)
  if constexpr (HYPER) {
    if (act && t < D)
#pragma unroll
      for (int c = 0; c < 3; c++) bufA[slot][c * D + t] = gu >= 0 ? A.u0[(int64_t)gu * 3 + c] : T(0);
    __syncthreads();
    hex_el_forward<T, N, NQ>(bufA[slot], bufB[slot], sB, sD, act, t, g0);
    __syncthreads();  // bufA is loaded again below
  }
  if (act && t < D)
#pragma unroll
    for (int c = 0; c < 3; c++) bufA[slot][c * D + t] = gi >= 0 ? A.x[(int64_t)gi * 3 + c] : T(0);
  __syncthreads();
  T g[3][3];  // g[c][d]: reference derivative d of component c
  hex_el_forward<T, N, NQ>(bufA[slot], bufB[slot], sB, sD, act, t, g);
  // the stress, thread = point (a, b, e)
  if (act && t < P) {
    const int a = t % NQ, b = (t / NQ) % NQ, e = t / (NQ * NQ);
    const T x1 = sg[a], x2 = sg[b], x3 = sg[e];
    // with several cells per workgroup a thread without a cell takes the unit cube, so that
    // its discarded arithmetic stays finite; with one, every active thread's cell index is
    // in range (a cell left out of a range apply only skips its scatter)
    const bool gv = CPB == 1 || valid;
    T J[3][3];  // J[r][d] = d x_r / d xi_d
#pragma unroll
    for (int r = 0; r < 3; r++) {
      const T *gc = A.geo + cell * 24;
      const T c1 = gv ? gc[r] : T(r == 0), c2 = gv ? gc[3 + r] : T(r == 1), c3 = gv ? gc[6 + r] : T(r == 2),
              c4 = gv ? gc[9 + r] : T(0), c5 = gv ? gc[12 + r] : T(0), c6 = gv ? gc[15 + r] : T(0),
              c7 = gv ? gc[18 + r] : T(0);
      J[r][0] = c1 + c4 * x2 + c5 * x3 + c7 * x2 * x3;
      J[r][1] = c2 + c4 * x1 + c6 * x3 + c7 * x1 * x3;
      J[r][2] = c3 + c5 * x1 + c6 * x2 + c7 * x1 * x2;
    }
    // inverse by cofactors: K[d][r] = d xi_d / d x_r = C[r][d] / det
    T C[3][3];
    C[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    C[0][1] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    C[0][2] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    C[1][0] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    C[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    C[1][2] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    C[2][0] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    C[2][1] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    C[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const T det = J[0][0] * C[0][0] + J[0][1] * C[0][1] + J[0][2] * C[0][2];
    const T rd = T(1) / det;
    // physical gradient G[c][r] = sum_d K[d][r] g[c][d]
    T G[3][3];
#pragma unroll
    for (int c = 0; c < 3; c++)
#pragma unroll
      for (int r = 0; r < 3; r++) G[c][r] = (C[r][0] * g[c][0] + C[r][1] * g[c][1] + C[r][2] * g[c][2]) * rd;
    const T wdet = sw[a] * sw[b] * sw[e] * (det < T(0) ? -det : det) * rd;
    // stress Sg[c][r] against d v_c / d x_r, then the reference flux
    // F[c][d] = w |det| sum_r K[d][r] Sg[c][r]
    T Sg[3][3];
    if constexpr (HYPER) {
      T F[3][3], S[3][3], dS[3][3];
#pragma unroll
      for (int c = 0; c < 3; c++)
#pragma unroll
        for (int r = 0; r < 3; r++)
          F[c][r] = (c == r ? T(1) : T(0)) + (C[r][0] * g0[c][0] + C[r][1] * g0[c][1] + C[r][2] * g0[c][2]) * rd;
      T trE = T(0), trdE = T(0);
#pragma unroll
      for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
          T ff = T(0), gf = T(0);
#pragma unroll
          for (int k = 0; k < 3; k++) {
            ff += F[k][i] * F[k][j];
            gf += G[k][i] * F[k][j] + F[k][i] * G[k][j];
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
        for (int r = 0; r < 3; r++) {
          T v = T(0);
#pragma unroll
          for (int k = 0; k < 3; k++) v += G[c][k] * S[k][r] + F[c][k] * dS[k][r];
          Sg[c][r] = v;
        }
    } else {
      const T tr = A.lam * (G[0][0] + G[1][1] + G[2][2]);
#pragma unroll
      for (int c = 0; c < 3; c++)
#pragma unroll
        for (int r = 0; r < 3; r++) Sg[c][r] = A.mu * (G[c][r] + G[r][c]) + (r == c ? tr : T(0));
    }
#pragma unroll
    for (int c = 0; c < 3; c++)
#pragma unroll
      for (int d = 0; d < 3; d++)
        bufB[slot][(3 * d + c) * P + t] = wdet * (C[0][d] * Sg[c][0] + C[1][d] * Sg[c][1] + C[2][d] * Sg[c][2]);
  }
  __syncthreads();
  // backward z, thread (a, b, l): Zx = B_z Fx, Zy = B_z Fy, Zz = B'_z Fz
  if (act && t < SY) {
    const int a = t % NQ, b = (t / NQ) % NQ, l = t / (NQ * NQ);
#pragma unroll
    for (int c = 0; c < 3; c++) {
      T zx = T(0), zy = T(0), zz = T(0);
#pragma unroll
      for (int e = 0; e < NQ; e++) {
        const int q = a + NQ * (b + NQ * e);
        zx += sB[e * N + l] * bufB[slot][c * P + q];
        zy += sB[e * N + l] * bufB[slot][(3 + c) * P + q];
        zz += sD[e * N + l] * bufB[slot][(6 + c) * P + q];
      }
      bufA[slot][c * SY + t] = zx;
      bufA[slot][(3 + c) * SY + t] = zy;
      bufA[slot][(6 + c) * SY + t] = zz;
    }
  }
  __syncthreads();
  // backward y, thread (a, j, l): Vx = B_y Zx, Vb = B'_y Zy + B_y Zz
  if (act && t < SX) {
    const int a = t % NQ, j = (t / NQ) % N, l = t / (NQ * N);
#pragma unroll
    for (int c = 0; c < 3; c++) {
      T vx = T(0), vb = T(0);
#pragma unroll
      for (int b = 0; b < NQ; b++) {
        const int h = a + NQ * (b + NQ * l);
        vx += sB[b * N + j] * bufA[slot][c * SY + h];
        vb += sD[b * N + j] * bufA[slot][(3 + c) * SY + h] + sB[b * N + j] * bufA[slot][(6 + c) * SY + h];
      }
      bufB[slot][c * SX + t] = vx;
      bufB[slot][(3 + c) * SX + t] = vb;
    }
  }
  __syncthreads();
  // backward x, thread (i, j, l), and the scatter
  if (act && t < D && idx >= 0) {
    const int i = t % N, j = (t / N) % N, l = t / (N * N);
#pragma unroll
    for (int c = 0; c < 3; c++) {
      T v = T(0);
#pragma unroll
      for (int a = 0; a < NQ; a++) {
        const int h = a + NQ * (j + N * l);
        v += sD[a * N + i] * bufB[slot][c * SX + h] + sB[a * N + i] * bufB[slot][(3 + c) * SX + h];
      }
      T *yp = A.y + (int64_t)idx * 3 + c;
      if (atomic) hex_el_atomic_add(yp, v);
      else *yp += v;
    }
  }
}

template <typename T, int N, int NQ>
static int launch_hex_el_nq(const HexElasArgs<T> &a, bool atomic, hipStream_t s) {
  constexpr int P = NQ * NQ * NQ, CPB = P <= 32 ? 64 / P : 1;
  const int64_t ngrp = (a.c1 - a.c0 + CPB - 1) / CPB;
  const dim3 g((unsigned)(((ngrp + 7) / 8) * 8)), b((unsigned)(CPB > 1 ? 64 : (P + 63) / 64 * 64));
  if (a.u0)
    hex_elasticity_kernel<T, N, NQ, true><<<g, b, 0, s>>>(a, atomic);
  else
    hex_elasticity_kernel<T, N, NQ, false><<<g, b, 0, s>>>(a, atomic);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

template <typename T, int N>
static int launch_hex_el_n(int nq, const HexElasArgs<T> &a, bool atomic, hipStream_t s) {
  if (nq == N) return launch_hex_el_nq<T, N, N>(a, atomic, s);
  if (nq == N + 1) return launch_hex_el_nq<T, N, N + 1>(a, atomic, s);
  return fail(MF_EUNSUPPORTED, "hex elasticity: nq1d must be k+1 or k+2");
}

template <typename T>
int launch_hex_elasticity(int k, int nq, const HexElasArgs<T> &a, bool atomic, hipStream_t s) {
  if (a.c1 <= a.c0) return MF_OK;
  switch (k) {
    case 1: return launch_hex_el_n<T, 2>(nq, a, atomic, s);
    case 2: return launch_hex_el_n<T, 3>(nq, a, atomic, s);
    case 3: return launch_hex_el_n<T, 4>(nq, a, atomic, s);
    case 4: return launch_hex_el_n<T, 5>(nq, a, atomic, s);
    case 5: return launch_hex_el_n<T, 6>(nq, a, atomic, s);
    case 6: return launch_hex_el_n<T, 7>(nq, a, atomic, s);
  }
  return fail(MF_EUNSUPPORTED, "hex elasticity degree (1..6)");
}

template int launch_hex_elasticity<double>(int, int, const HexElasArgs<double> &, bool, hipStream_t);
template int launch_hex_elasticity<float>(int, int, const HexElasArgs<float> &, bool, hipStream_t);

}  // namespace mf
