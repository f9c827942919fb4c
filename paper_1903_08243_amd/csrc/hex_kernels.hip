// Sum-factorised operator action on trilinear hexahedra (Q_k, GLL nodes,
// tensor Gauss quadrature with n = k+1 points per direction).
//
// What is computed is the paper's global assembly of the action (Section 2.2,
// Listing 3: gather through cell2dof, zeroed local tensor, local kernel,
// scatter-increment) with the local kernel of Section 2.1 (Jacobian at every
// quadrature point for the multilinear map, |det J|, quadrature loop), where
// the change of basis to and from quadrature points is sum-factorised on the
// tensor-product cell (Section 3 and Section 4.2.4: per-direction 1D loops
// instead of dense tabulation).
//
// GPU mapping (gfx950): a workgroup holds EPB = floor(256 / n^2) cells; each
// cell owns n^2 threads and three n^3 LDS buffers. A thread always holds one
// "pencil" (a 1D line of n values) in registers, so each 1D contraction is a
// register-only product with the uniform table (kernel-argument / scalar
// loads) and LDS is only used to switch the pencil direction between stages.
// Forward:  z-contraction (B) -> y (B) -> x (B), x-derivative (collocation D)
//           -> y-derivative (D) -> z-derivative (D, in registers)
// Pointwise: Jacobian from the cell's trilinear coefficients (two FMAs per
//           entry per point), adjugate rows, G = w |det|^{-1} adj adj^T,
//           fluxes F = coef G grad_ref u and mass term w |det| coef u.
// Backward: transposes in the reverse order, then atomic scatter-add.
#include "mf_internal.h"

namespace mf {

enum { K_MASS = MF_OP_MASS, K_HELM = MF_OP_HELMHOLTZ, K_LAP = MF_OP_LAPLACIAN, K_POIS = MF_OP_POISSON };

template <typename T, int N> struct HexTabD {
  T B[N][N];
  T D[N][N];
  T g[N];
  T w[N];
  T dB[N][N];
};

__device__ __forceinline__ void atomic_add_f(double *p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add_f(float *p, float v) { unsafeAtomicAdd(p, v); }

template <int N> constexpr int hex_epb() { return 256 / (N * N); }

// ---------------------------------------------------------------------------------- apply
template <typename T, int N, int KIND>
__global__ void __launch_bounds__(256) hex_apply_kernel(const HexArgs<T> A, const HexTabD<T, N> tb) {
  constexpr int NN = N * N, N3 = NN * N, EPB = hex_epb<N>();
  constexpr bool GRAD = KIND != K_MASS;
  constexpr bool MASS = KIND == K_MASS || KIND == K_HELM;
  constexpr bool COEF = KIND == K_MASS || KIND == K_POIS;
  __shared__ T s0[EPB * N3];
  __shared__ T s1[GRAD ? EPB * N3 : 1];
  __shared__ T s2[GRAD ? EPB * N3 : 1];
  __shared__ T sg[EPB * 32];

  const int t = threadIdx.x;
  const int le = t / NN, p = t - le * NN;
  const int pa = p % N, pb = p / N;
  const int64_t cell0 = A.c0 + (int64_t)blockIdx.x * EPB;
  const int64_t cell = cell0 + le;
  const bool valid = cell < A.c1;

  for (int i = t; i < EPB * 32; i += EPB * NN) {
    const int e = i >> 5, j = i & 31;
    const int64_t c = cell0 + e;
    T v = T(0);
    if (c < A.c1) {
      if (j < 24) v = A.geo[c * 24 + j];
      else if (COEF && A.coef) v = A.coef[c * 8 + (j - 24)];
      else if (j == 24) v = T(1);  // coefficient 1 when absent
    }
    sg[i] = v;
  }
  __syncthreads();

  T *u0 = s0 + le * N3;
  T *u1 = s1 + (GRAD ? le * N3 : 0);
  T *u2 = s2 + (GRAD ? le * N3 : 0);
  const T *G = sg + le * 32;

  // Per-thread geometry for the pointwise stage: this thread owns points (pa, pb, *).
  const T x1 = tb.g[pa], x2 = tb.g[pb];
  T A1[3], B1[3], A2[3], B2[3], A3[3];
#pragma unroll
  for (int d = 0; d < 3; d++) {
    const T c1 = G[0 + d], c2 = G[3 + d], c3 = G[6 + d], c4 = G[9 + d], c5 = G[12 + d],
            c6 = G[15 + d], c7 = G[18 + d];
    A1[d] = c1 + c4 * x2;
    B1[d] = c5 + c7 * x2;
    A2[d] = c2 + c4 * x1;
    B2[d] = c6 + c7 * x1;
    A3[d] = c3 + c5 * x1 + c6 * x2 + c7 * x1 * x2;
  }
  T ka = T(1), kb = T(0);
  if (COEF) {
    const T *K = G + 24;
    ka = K[0] + K[1] * x1 + K[2] * x2 + K[4] * x1 * x2;
    kb = K[3] + K[5] * x1 + K[6] * x2 + K[7] * x1 * x2;
  }
  const T wab = tb.w[pa] * tb.w[pb];
  const int32_t *cmap = A.map + (valid ? cell : 0) * N3;
  const int nc = A.ncomp;

  for (int comp = 0; comp < nc; comp++) {
    T r[N], v[N];
    // ---- gather z-pencil (i, j) = (pa, pb), contract z with B
#pragma unroll
    for (int l = 0; l < N; l++) {
      const int idx = valid ? cmap[pa + N * pb + NN * l] : -1;
      r[l] = idx >= 0 ? A.x[(int64_t)idx * nc + comp] : T(0);
    }
#pragma unroll
    for (int c = 0; c < N; c++) {
      T s = T(0);
#pragma unroll
      for (int l = 0; l < N; l++) s += tb.B[c][l] * r[l];
      u0[c * NN + pb * N + pa] = s;
    }
    __syncthreads();
    // ---- y-pencil (x = pa, z = pb): contract y with B
#pragma unroll
    for (int yy = 0; yy < N; yy++) r[yy] = u0[pb * NN + yy * N + pa];
#pragma unroll
    for (int b = 0; b < N; b++) {
      T s = T(0);
#pragma unroll
      for (int yy = 0; yy < N; yy++) s += tb.B[b][yy] * r[yy];
      u0[pb * NN + b * N + pa] = s;
    }
    __syncthreads();
    // ---- x-pencil (y = pa, z = pb): contract x with B -> u at points; x-derivative
#pragma unroll
    for (int xx = 0; xx < N; xx++) r[xx] = u0[pb * NN + pa * N + xx];
#pragma unroll
    for (int a = 0; a < N; a++) {
      T s = T(0);
#pragma unroll
      for (int xx = 0; xx < N; xx++) s += tb.B[a][xx] * r[xx];
      v[a] = s;
    }
#pragma unroll
    for (int a = 0; a < N; a++) u0[pb * NN + pa * N + a] = v[a];
    if constexpr (GRAD) {
#pragma unroll
      for (int a = 0; a < N; a++) {
        T s = T(0);
#pragma unroll
        for (int b = 0; b < N; b++) s += tb.D[a][b] * v[b];
        u1[pb * NN + pa * N + a] = s;
      }
      __syncthreads();
      // ---- y-pencil (x = pa, z = pb): y-derivative of u
#pragma unroll
      for (int yy = 0; yy < N; yy++) r[yy] = u0[pb * NN + yy * N + pa];
#pragma unroll
      for (int b = 0; b < N; b++) {
        T s = T(0);
#pragma unroll
        for (int yy = 0; yy < N; yy++) s += tb.D[b][yy] * r[yy];
        u2[pb * NN + b * N + pa] = s;
      }
    }
    __syncthreads();
    // ---- pointwise on z-pencil (a, b) = (pa, pb)
    {
      T uz[N], f2[N];
#pragma unroll
      for (int c = 0; c < N; c++) uz[c] = u0[c * NN + pb * N + pa];
#pragma unroll
      for (int c = 0; c < N; c++) {
        const T x3 = tb.g[c];
        T j1[3], j2[3];
#pragma unroll
        for (int d = 0; d < 3; d++) {
          j1[d] = A1[d] + x3 * B1[d];
          j2[d] = A2[d] + x3 * B2[d];
        }
        const T *j3 = A3;
        // adjugate rows: r0 = j2 x j3, r1 = j3 x j1, r2 = j1 x j2  (J^{-1} = rows / det)
        const T r0[3] = {j2[1] * j3[2] - j2[2] * j3[1], j2[2] * j3[0] - j2[0] * j3[2],
                         j2[0] * j3[1] - j2[1] * j3[0]};
        const T det = j1[0] * r0[0] + j1[1] * r0[1] + j1[2] * r0[2];
        const T adet = det < T(0) ? -det : det;
        const T wq = wab * tb.w[c];
        const T kq = COEF ? ka + kb * x3 : T(1);
        T mterm = T(0);
        if constexpr (MASS) mterm = wq * adet * kq * uz[c];
        if constexpr (GRAD) {
          const T r1[3] = {j3[1] * j1[2] - j3[2] * j1[1], j3[2] * j1[0] - j3[0] * j1[2],
                           j3[0] * j1[1] - j3[1] * j1[0]};
          const T r2[3] = {j1[1] * j2[2] - j1[2] * j2[1], j1[2] * j2[0] - j1[0] * j2[2],
                           j1[0] * j2[1] - j1[1] * j2[0]};
          const T sc = wq * kq / adet;
          // d(u)/d(ref x), d/d(ref y) from LDS, d/d(ref z) from the register pencil
          T dz = T(0);
#pragma unroll
          for (int cc = 0; cc < N; cc++) dz += tb.D[c][cc] * uz[cc];
          const T dx = u1[c * NN + pb * N + pa];
          const T dy = u2[c * NN + pb * N + pa];
          // physical gradient times |det| pieces: e_b = r_b . (adj^T d) ; F = sc * adj adj^T d
          const T gx = r0[0] * dx + r1[0] * dy + r2[0] * dz;
          const T gy = r0[1] * dx + r1[1] * dy + r2[1] * dz;
          const T gz = r0[2] * dx + r1[2] * dy + r2[2] * dz;
          const T f0 = sc * (r0[0] * gx + r0[1] * gy + r0[2] * gz);
          const T f1 = sc * (r1[0] * gx + r1[1] * gy + r1[2] * gz);
          f2[c] = sc * (r2[0] * gx + r2[1] * gy + r2[2] * gz);
          u1[c * NN + pb * N + pa] = f0;
          u2[c * NN + pb * N + pa] = f1;
        }
        v[c] = mterm;
      }
      if constexpr (GRAD) {
        // z-transpose of the derivative: v[c] += sum_c' D[c'][c] f2[c']
#pragma unroll
        for (int c = 0; c < N; c++) {
          T s = v[c];
#pragma unroll
          for (int cc = 0; cc < N; cc++) s += tb.D[cc][c] * f2[cc];
          v[c] = s;
        }
      }
#pragma unroll
      for (int c = 0; c < N; c++) u0[c * NN + pb * N + pa] = v[c];
    }
    __syncthreads();
    if constexpr (GRAD) {
      // ---- y-pencil (x = pa, z = pb): add D^T along y of f1
#pragma unroll
      for (int yy = 0; yy < N; yy++) r[yy] = u2[pb * NN + yy * N + pa];
#pragma unroll
      for (int b = 0; b < N; b++) {
        T s = u0[pb * NN + b * N + pa];
#pragma unroll
        for (int yy = 0; yy < N; yy++) s += tb.D[yy][b] * r[yy];
        u0[pb * NN + b * N + pa] = s;
      }
      __syncthreads();
    }
    // ---- x-pencil (y = pa, z = pb): add D^T along x of f0, then B^T along x
#pragma unroll
    for (int a = 0; a < N; a++) v[a] = u0[pb * NN + pa * N + a];
    if constexpr (GRAD) {
#pragma unroll
      for (int a = 0; a < N; a++) r[a] = u1[pb * NN + pa * N + a];
#pragma unroll
      for (int a = 0; a < N; a++) {
        T s = v[a];
#pragma unroll
        for (int aa = 0; aa < N; aa++) s += tb.D[aa][a] * r[aa];
        v[a] = s;
      }
    }
#pragma unroll
    for (int i = 0; i < N; i++) {
      T s = T(0);
#pragma unroll
      for (int a = 0; a < N; a++) s += tb.B[a][i] * v[a];
      u0[pb * NN + pa * N + i] = s;
    }
    __syncthreads();
    // ---- y-pencil (x = pa, z = pb): B^T along y
#pragma unroll
    for (int b = 0; b < N; b++) r[b] = u0[pb * NN + b * N + pa];
#pragma unroll
    for (int j = 0; j < N; j++) {
      T s = T(0);
#pragma unroll
      for (int b = 0; b < N; b++) s += tb.B[b][j] * r[b];
      u0[pb * NN + j * N + pa] = s;
    }
    __syncthreads();
    // ---- z-pencil (i, j) = (pa, pb): B^T along z, scatter-add
#pragma unroll
    for (int c = 0; c < N; c++) r[c] = u0[c * NN + pb * N + pa];
#pragma unroll
    for (int l = 0; l < N; l++) {
      T s = T(0);
#pragma unroll
      for (int c = 0; c < N; c++) s += tb.B[c][l] * r[c];
      const int idx = valid ? cmap[pa + N * pb + NN * l] : -1;
      if (idx >= 0) atomic_add_f(&A.y[(int64_t)idx * nc + comp], s);
    }
    if (comp + 1 < nc) __syncthreads();
  }
}

// ---------------------------------------------------------------------------------- diagonal
// diag_i = sum_q [ grad_ref phi_i^T G grad_ref phi_i + m phi_i^2 ], one thread per cell node;
// the per-point G (6) and mass factor m are computed once per point into LDS.
template <int N> constexpr int hexd_epb() { return (N * N * N >= 256) ? 1 : 256 / (N * N * N); }

template <typename T, int N, int KIND>
__global__ void __launch_bounds__(512) hex_diag_kernel(const HexArgs<T> A, const HexTabD<T, N> tb) {
  constexpr int N3 = N * N * N, EPB = hexd_epb<N>();
  constexpr bool GRAD = KIND != K_MASS;
  constexpr bool MASS = KIND == K_MASS || KIND == K_HELM;
  constexpr bool COEF = KIND == K_MASS || KIND == K_POIS;
  __shared__ T sG[EPB][7][N3];
  const int t = threadIdx.x;
  const int le = t / N3, p = t - le * N3;
  const int64_t cell = A.c0 + (int64_t)blockIdx.x * EPB + le;
  const bool valid = cell < A.c1;
  const int64_t cg = valid ? cell : A.c0;
  {
    const int a = p % N, b = (p / N) % N, c = p / (N * N);
    const T *G = A.geo + cg * 24;
    const T x1 = tb.g[a], x2 = tb.g[b], x3 = tb.g[c];
    T j1[3], j2[3], j3[3];
    for (int d = 0; d < 3; d++) {
      const T c1 = G[0 + d], c2 = G[3 + d], c3 = G[6 + d], c4 = G[9 + d], c5 = G[12 + d],
              c6 = G[15 + d], c7 = G[18 + d];
      j1[d] = c1 + c4 * x2 + c5 * x3 + c7 * x2 * x3;
      j2[d] = c2 + c4 * x1 + c6 * x3 + c7 * x1 * x3;
      j3[d] = c3 + c5 * x1 + c6 * x2 + c7 * x1 * x2;
    }
    const T r0[3] = {j2[1] * j3[2] - j2[2] * j3[1], j2[2] * j3[0] - j2[0] * j3[2], j2[0] * j3[1] - j2[1] * j3[0]};
    const T r1[3] = {j3[1] * j1[2] - j3[2] * j1[1], j3[2] * j1[0] - j3[0] * j1[2], j3[0] * j1[1] - j3[1] * j1[0]};
    const T r2[3] = {j1[1] * j2[2] - j1[2] * j2[1], j1[2] * j2[0] - j1[0] * j2[2], j1[0] * j2[1] - j1[1] * j2[0]};
    const T det = j1[0] * r0[0] + j1[1] * r0[1] + j1[2] * r0[2];
    const T adet = det < T(0) ? -det : det;
    const T wq = tb.w[a] * tb.w[b] * tb.w[c];
    T kq = T(1);
    if (COEF && A.coef) {
      const T *K = A.coef + cg * 8;
      kq = K[0] + K[1] * x1 + K[2] * x2 + K[3] * x3 + K[4] * x1 * x2 + K[5] * x1 * x3 + K[6] * x2 * x3 +
           K[7] * x1 * x2 * x3;
    }
    const T sc = GRAD ? wq * kq / adet : T(0);
    auto dot = [](const T *u, const T *v) { return u[0] * v[0] + u[1] * v[1] + u[2] * v[2]; };
    sG[le][0][p] = sc * dot(r0, r0);
    sG[le][1][p] = sc * dot(r0, r1);
    sG[le][2][p] = sc * dot(r0, r2);
    sG[le][3][p] = sc * dot(r1, r1);
    sG[le][4][p] = sc * dot(r1, r2);
    sG[le][5][p] = sc * dot(r2, r2);
    sG[le][6][p] = MASS ? wq * adet * kq : T(0);
  }
  __syncthreads();
  const int i = p % N, j = (p / N) % N, l = p / (N * N);
  T acc = T(0);
  for (int c = 0; c < N; c++)
    for (int b = 0; b < N; b++)
      for (int a = 0; a < N; a++) {
        const int q = a + N * (b + N * c);
        const T bi = tb.B[a][i], bj = tb.B[b][j], bl = tb.B[c][l];
        const T vv = bi * bj * bl;
        T s = sG[le][6][q] * vv * vv;
        if (GRAD) {
          const T d0 = tb.dB[a][i] * bj * bl, d1 = bi * tb.dB[b][j] * bl, d2 = bi * bj * tb.dB[c][l];
          s += sG[le][0][q] * d0 * d0 + sG[le][3][q] * d1 * d1 + sG[le][5][q] * d2 * d2 +
               T(2) * (sG[le][1][q] * d0 * d1 + sG[le][2][q] * d0 * d2 + sG[le][4][q] * d1 * d2);
        }
        acc += s;
      }
  if (valid) {
    const int idx = A.map[cell * N3 + p];
    if (idx >= 0)
      for (int comp = 0; comp < A.ncomp; comp++) atomic_add_f(&A.y[(int64_t)idx * A.ncomp + comp], acc);
  }
}

// ---------------------------------------------------------------------------------- launchers
template <typename T, int N>
static int launch_apply_n(int kind, const HexArgs<T> &a, const void *tab, hipStream_t s) {
  const HexTabD<T, N> &tb = *static_cast<const HexTabD<T, N> *>(tab);
  constexpr int EPB = hex_epb<N>();
  const int64_t nc = a.c1 - a.c0;
  if (nc <= 0) return MF_OK;
  dim3 grid((unsigned)((nc + EPB - 1) / EPB)), block(EPB * N * N);
  switch (kind) {
    case K_MASS: hex_apply_kernel<T, N, K_MASS><<<grid, block, 0, s>>>(a, tb); break;
    case K_HELM: hex_apply_kernel<T, N, K_HELM><<<grid, block, 0, s>>>(a, tb); break;
    case K_LAP: hex_apply_kernel<T, N, K_LAP><<<grid, block, 0, s>>>(a, tb); break;
    case K_POIS: hex_apply_kernel<T, N, K_POIS><<<grid, block, 0, s>>>(a, tb); break;
    default: return fail(MF_EUNSUPPORTED, "hex kernel: operator kind");
  }
  MF_HIP(hipGetLastError());
  return MF_OK;
}

template <typename T, int N>
static int launch_diag_n(int kind, const HexArgs<T> &a, const void *tab, hipStream_t s) {
  const HexTabD<T, N> &tb = *static_cast<const HexTabD<T, N> *>(tab);
  constexpr int EPB = hexd_epb<N>();
  const int64_t nc = a.c1 - a.c0;
  if (nc <= 0) return MF_OK;
  dim3 grid((unsigned)((nc + EPB - 1) / EPB)), block(EPB * N * N * N);
  switch (kind) {
    case K_MASS: hex_diag_kernel<T, N, K_MASS><<<grid, block, 0, s>>>(a, tb); break;
    case K_HELM: hex_diag_kernel<T, N, K_HELM><<<grid, block, 0, s>>>(a, tb); break;
    case K_LAP: hex_diag_kernel<T, N, K_LAP><<<grid, block, 0, s>>>(a, tb); break;
    case K_POIS: hex_diag_kernel<T, N, K_POIS><<<grid, block, 0, s>>>(a, tb); break;
    default: return fail(MF_EUNSUPPORTED, "hex diagonal: operator kind");
  }
  MF_HIP(hipGetLastError());
  return MF_OK;
}

template <typename T>
int launch_hex_apply(int N, int kind, const HexArgs<T> &a, const void *tab, hipStream_t s) {
  switch (N) {
    case 2: return launch_apply_n<T, 2>(kind, a, tab, s);
    case 3: return launch_apply_n<T, 3>(kind, a, tab, s);
    case 4: return launch_apply_n<T, 4>(kind, a, tab, s);
    case 5: return launch_apply_n<T, 5>(kind, a, tab, s);
    case 6: return launch_apply_n<T, 6>(kind, a, tab, s);
    case 7: return launch_apply_n<T, 7>(kind, a, tab, s);
  }
  return fail(MF_EUNSUPPORTED, "hex kernel: degree");
}

template <typename T>
int launch_hex_diag(int N, int kind, const HexArgs<T> &a, const void *tab, hipStream_t s) {
  switch (N) {
    case 2: return launch_diag_n<T, 2>(kind, a, tab, s);
    case 3: return launch_diag_n<T, 3>(kind, a, tab, s);
    case 4: return launch_diag_n<T, 4>(kind, a, tab, s);
    case 5: return launch_diag_n<T, 5>(kind, a, tab, s);
    case 6: return launch_diag_n<T, 6>(kind, a, tab, s);
    case 7: return launch_diag_n<T, 7>(kind, a, tab, s);
  }
  return fail(MF_EUNSUPPORTED, "hex diagonal: degree");
}

template int launch_hex_apply<double>(int, int, const HexArgs<double> &, const void *, hipStream_t);
template int launch_hex_apply<float>(int, int, const HexArgs<float> &, const void *, hipStream_t);
template int launch_hex_diag<double>(int, int, const HexArgs<double> &, const void *, hipStream_t);
template int launch_hex_diag<float>(int, int, const HexArgs<float> &, const void *, hipStream_t);

// Size of the table struct the launchers expect for (T, N); used by the host setup.
template <typename T> size_t hex_table_bytes(int N) {
  switch (N) {
    case 2: return sizeof(HexTabD<T, 2>);
    case 3: return sizeof(HexTabD<T, 3>);
    case 4: return sizeof(HexTabD<T, 4>);
    case 5: return sizeof(HexTabD<T, 5>);
    case 6: return sizeof(HexTabD<T, 6>);
    case 7: return sizeof(HexTabD<T, 7>);
  }
  return 0;
}
template size_t hex_table_bytes<double>(int);
template size_t hex_table_bytes<float>(int);

}  // namespace mf
