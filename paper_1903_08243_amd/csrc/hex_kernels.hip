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
// GPU mapping (gfx950): a workgroup of WPB 64-wide wavefronts (one for n <= 5)
// holds EPB = floor(64 WPB / n^2) cells; each cell owns n^2 lanes and three n^3
// LDS buffers. With one wavefront, the LDS exchanges between stages need no
// cross-wavefront barrier and wavefronts on a SIMD run independently; n = 6 and 7
// use 2 and 4 wavefronts to keep more lanes busy. Lanes left over
// (64 WPB - EPB n^2) mirror an active lane: they compute the same pencil and store
// the same values, but never scatter.
// A thread always holds one "pencil" (a 1D line of n values) in registers, so
// each 1D contraction is a register-only product with compile-time tables
// and LDS is only used to switch the pencil direction between stages.
// Forward:  z-contraction (B) -> y (B) -> x (B), x-derivative (collocation D)
//           -> y-derivative (D) -> z-derivative (D, in registers)
// Pointwise: Jacobian from the cell's trilinear coefficients (two FMAs per
//           entry per point), adjugate rows, G = w |det|^{-1} adj adj^T,
//           fluxes F = coef G grad_ref u and mass term w |det| coef u.
// Backward: transposes in the reverse order, then atomic scatter-add.
#include <type_traits>

#include "hex_common.h"

namespace mf {

// Wavefronts per workgroup of the apply kernel: a workgroup holds floor(64 WPB / n^2)
// cells, so n = 6 (36 lanes per cell) and n = 7 (49) keep 84% and 96% of their lanes
// busy with 2 and 4 wavefronts instead of 56% and 77% with one. The batched kernel
// always uses one wavefront.
template <int N> constexpr int hex_wpb() { return N == 6 ? 2 : N == 7 ? 4 : 1; }
template <int N, int WPB = 1> constexpr int hex_epb() { return WPB * 64 / (N * N); }

// Padded LDS layout of one cell's n^3 buffer: entry (x, y, z) at z*SZ + y*SY + x,
// cells SE apart. The strides are chosen (by an offline search over the three
// pencil access patterns of a wavefront) to spread 8-byte accesses over the LDS
// banks; the natural strides n, n^2, n^3 put the y- and x-pencil accesses of a
// quarter-wavefront on a few banks.
template <int N> struct HexLds;
template <> struct HexLds<2> { static constexpr int SY = 2, SZ = 5, SE = 12; };
template <> struct HexLds<3> { static constexpr int SY = 3, SZ = 9, SE = 27; };
template <> struct HexLds<4> { static constexpr int SY = 4, SZ = 19, SE = 80; };
template <> struct HexLds<5> { static constexpr int SY = 5, SZ = 25, SE = 135; };
template <> struct HexLds<6> { static constexpr int SY = 9, SZ = 54, SE = 324; };
template <> struct HexLds<7> { static constexpr int SY = 7, SZ = 52, SE = 364; };

// ---------------------------------------------------------------------------------- apply

// Padded n^3 LDS buffers per cell: one without gradients; with gradients three, or
// two from n = 6 on (the stage order of hex_pencil_stages2, which keeps the
// x-derivative and the x-flux in registers: LDS, not registers, is what limits the
// resident wavefronts of the Q5 and Q6 kernels).
template <int N, bool GRAD> constexpr int hex_nbuf() { return GRAD ? (N >= 6 ? 2 : 3) : 1; }

// LDS (in units of T) one workgroup needs for degree n-1: the stage buffers, 32
// geometry values per cell and, with more than one wavefront, one buffer that mirror
// lanes write into (never read).
template <typename T, int N, bool GRAD, int WPB = 1> constexpr int hex_lds_size() {
  return hex_epb<N, WPB>() * (HexLds<N>::SE * hex_nbuf<N, GRAD>() + 32) + (WPB > 1 ? HexLds<N>::SE : 0) +
         (sizeof(T) == 4 ? 128 : 0);
}

#define IX(x, y, z) ((z) * SZ + (y) * SY + (x))
// The sum-factorised action of one cell on the calling thread's pencil (pa, pb, *):
// on entry r holds the cell's nodal values on that z-pencil, on exit the local
// result on the same pencil. Gc: the cell's 32 geometry and coefficient entries in
// LDS; u0, u1, u2: its three padded n^3 LDS buffers (u0 alone without gradients),
// read through u* and written through w* (the same buffers, or for a mirror lane a
// discard area, so its stores need no branch).
// Contains workgroup barriers, so every thread of the workgroup calls it.
template <typename T, int N, int KIND, int WPB>
__device__ __forceinline__ void hex_pencil_stages(T (&r)[N], const T *Gc, const T *u0, const T *u1, const T *u2,
                                                  T *w0, T *w1, T *w2, const int pa, const int pb) {
  using TB = TabT<T, N>;
  constexpr bool GRAD = KIND != K_MASS;
  constexpr bool MASS = KIND == K_MASS || KIND == K_HELM;
  constexpr bool COEF = KIND == K_MASS || KIND == K_POIS;
  constexpr int SY = HexLds<N>::SY, SZ = HexLds<N>::SZ;
  const T x1 = TB::g(pa), x2 = TB::g(pb);
  const T wab = TB::w(pa) * TB::w(pb);
  {
    // Per-thread geometry for the pointwise stage: this thread owns points (pa, pb, *).
    T A1[3], B1[3], A2[3], B2[3], A3[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
      const T c1 = Gc[0 + d], c2 = Gc[3 + d], c3 = Gc[6 + d], c4 = Gc[9 + d], c5 = Gc[12 + d],
              c6 = Gc[15 + d], c7 = Gc[18 + d];
      A1[d] = c1 + c4 * x2;
      B1[d] = c5 + c7 * x2;
      A2[d] = c2 + c4 * x1;
      B2[d] = c6 + c7 * x1;
      A3[d] = c3 + c5 * x1 + c6 * x2 + c7 * x1 * x2;
    }
    T ka = T(1), kb = T(0);
    if (COEF) {
      const T *K = Gc + 24;
      ka = K[0] + K[1] * x1 + K[2] * x2 + K[4] * x1 * x2;
      kb = K[3] + K[5] * x1 + K[6] * x2 + K[7] * x1 * x2;
    }

    {
      T v[N];
      // ---- z-pencil (i, j) = (pa, pb): contract z with B
      eo_contract<T, N, MatB<N>, 1>(r, v);
  #pragma unroll
      for (int c = 0; c < N; c++) w0[IX(pa, pb, c)] = v[c];
      __syncthreads();
      // ---- y-pencil (x = pa, z = pb): contract y with B
  #pragma unroll
      for (int yy = 0; yy < N; yy++) r[yy] = u0[IX(pa, yy, pb)];
      eo_contract<T, N, MatB<N>, 1>(r, v);
  #pragma unroll
      for (int b = 0; b < N; b++) w0[IX(pa, b, pb)] = v[b];
      __syncthreads();
      // ---- x-pencil (y = pa, z = pb): contract x with B -> u at points; x-derivative
  #pragma unroll
      for (int xx = 0; xx < N; xx++) r[xx] = u0[IX(xx, pa, pb)];
      eo_contract<T, N, MatB<N>, 1>(r, v);
  #pragma unroll
      for (int a = 0; a < N; a++) w0[IX(a, pa, pb)] = v[a];
      if constexpr (GRAD) {
        eo_contract<T, N, MatD<N>, -1>(v, r);
  #pragma unroll
        for (int a = 0; a < N; a++) w1[IX(a, pa, pb)] = r[a];
        __syncthreads();
        // ---- y-pencil (x = pa, z = pb): y-derivative of u
  #pragma unroll
        for (int yy = 0; yy < N; yy++) r[yy] = u0[IX(pa, yy, pb)];
        eo_contract<T, N, MatD<N>, -1>(r, v);
  #pragma unroll
        for (int b = 0; b < N; b++) w2[IX(pa, b, pb)] = v[b];
      }
      __syncthreads();
      // ---- pointwise on z-pencil (a, b) = (pa, pb)
      {
        T uz[N], f2[N], dzv[N];
  #pragma unroll
        for (int c = 0; c < N; c++) uz[c] = u0[IX(pa, pb, c)];
        if constexpr (GRAD) eo_contract<T, N, MatD<N>, -1>(uz, dzv);
  #pragma unroll
        for (int c = 0; c < N; c++) {
          const T x3 = TB::g(c);
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
          const T wq = wab * TB::w(c);
          const T kq = COEF ? ka + kb * x3 : T(1);
          T mterm = T(0);
          if constexpr (MASS) mterm = wq * adet * kq * uz[c];
          if constexpr (GRAD) {
            const T r1[3] = {j3[1] * j1[2] - j3[2] * j1[1], j3[2] * j1[0] - j3[0] * j1[2],
                             j3[0] * j1[1] - j3[1] * j1[0]};
            const T r2[3] = {j1[1] * j2[2] - j1[2] * j2[1], j1[2] * j2[0] - j1[0] * j2[2],
                             j1[0] * j2[1] - j1[1] * j2[0]};
            const T sc = wq * kq * recip(adet);
            // d(u)/d(ref x), d/d(ref y) from LDS, d/d(ref z) from the register pencil
            const T dz = dzv[c];
            const T dx = u1[IX(pa, pb, c)];
            const T dy = u2[IX(pa, pb, c)];
            // physical gradient times |det| pieces: e_b = r_b . (adj^T d) ; F = sc * adj adj^T d
            const T gx = r0[0] * dx + r1[0] * dy + r2[0] * dz;
            const T gy = r0[1] * dx + r1[1] * dy + r2[1] * dz;
            const T gz = r0[2] * dx + r1[2] * dy + r2[2] * dz;
            const T f0 = sc * (r0[0] * gx + r0[1] * gy + r0[2] * gz);
            const T f1 = sc * (r1[0] * gx + r1[1] * gy + r1[2] * gz);
            f2[c] = sc * (r2[0] * gx + r2[1] * gy + r2[2] * gz);
            w1[IX(pa, pb, c)] = f0;
            w2[IX(pa, pb, c)] = f1;
          }
          v[c] = mterm;
        }
        if constexpr (GRAD) {
          // z-transpose of the derivative: v[c] += sum_c' D[c'][c] f2[c']
          eo_contract<T, N, MatDt<N>, -1>(f2, dzv);
  #pragma unroll
          for (int c = 0; c < N; c++) v[c] += dzv[c];
        }
  #pragma unroll
        for (int c = 0; c < N; c++) w0[IX(pa, pb, c)] = v[c];
      }
      __syncthreads();
      if constexpr (GRAD) {
        // ---- y-pencil (x = pa, z = pb): add D^T along y of f1
  #pragma unroll
        for (int yy = 0; yy < N; yy++) r[yy] = u2[IX(pa, yy, pb)];
        eo_contract<T, N, MatDt<N>, -1>(r, v);
  #pragma unroll
        for (int b = 0; b < N; b++) {
          const T s = u0[IX(pa, b, pb)] + v[b];
          w0[IX(pa, b, pb)] = s;
        }
        __syncthreads();
      }
      // ---- x-pencil (y = pa, z = pb): add D^T along x of f0, then B^T along x
  #pragma unroll
      for (int a = 0; a < N; a++) v[a] = u0[IX(a, pa, pb)];
      if constexpr (GRAD) {
  #pragma unroll
        for (int a = 0; a < N; a++) r[a] = u1[IX(a, pa, pb)];
        T dv[N];
        eo_contract<T, N, MatDt<N>, -1>(r, dv);
  #pragma unroll
        for (int a = 0; a < N; a++) v[a] += dv[a];
      }
      eo_contract<T, N, MatBt<N>, 1>(v, r);
  #pragma unroll
      for (int i = 0; i < N; i++) w0[IX(i, pa, pb)] = r[i];
      __syncthreads();
      // ---- y-pencil (x = pa, z = pb): B^T along y
  #pragma unroll
      for (int b = 0; b < N; b++) r[b] = u0[IX(pa, b, pb)];
      eo_contract<T, N, MatBt<N>, 1>(r, v);
  #pragma unroll
      for (int j = 0; j < N; j++) w0[IX(pa, j, pb)] = v[j];
      __syncthreads();
      // ---- z-pencil (i, j) = (pa, pb): B^T along z, scatter-add
  #pragma unroll
      for (int c = 0; c < N; c++) r[c] = u0[IX(pa, pb, c)];
      eo_contract<T, N, MatBt<N>, 1>(r, v);
  #pragma unroll
      for (int l = 0; l < N; l++) r[l] = v[l];
    }
  }
}

// The gradient kinds' action with two stage buffers U and V per cell (n >= 6): the
// pointwise stage runs on x-pencils, whose lanes keep u from the x pass in registers
// (its x-derivative is taken there); the z- and y-derivatives come through V and U (the y one in
// place over u), the z- and y-fluxes go back through V and U and the x-flux stays in
// registers. Same contract as hex_pencil_stages (on entry r holds the nodal z-pencil
// (pa, pb, *), on exit the local result on it); one more barrier, a third less LDS.
template <typename T, int N, int KIND, int WPB>
__device__ __forceinline__ void hex_pencil_stages2(T (&r)[N], const T *Gc, const T *u0, const T *u1, T *w0, T *w1,
                                                   const int pa, const int pb) {
  using TB = TabT<T, N>;
  constexpr bool MASS = KIND == K_HELM;
  constexpr bool COEF = KIND == K_POIS;
  constexpr int SY = HexLds<N>::SY, SZ = HexLds<N>::SZ;
  // this lane's x-pencil in the pointwise stage: y = g(pa), z = g(pb), x varies. Along
  // it the Jacobian columns are j1 = P1, j2 = P2 + x Q2, j3 = P3 + x Q3 (trilinear map)
  const T x2 = TB::g(pa), x3 = TB::g(pb);
  const T wyz = TB::w(pa) * TB::w(pb);
  T P1[3], P2[3], Q2[3], P3[3], Q3[3];
#pragma unroll
  for (int d = 0; d < 3; d++) {
    const T c1 = Gc[0 + d], c2 = Gc[3 + d], c3 = Gc[6 + d], c4 = Gc[9 + d], c5 = Gc[12 + d], c6 = Gc[15 + d],
            c7 = Gc[18 + d];
    P1[d] = c1 + c4 * x2 + (c5 + c7 * x2) * x3;
    P2[d] = c2 + c6 * x3;
    Q2[d] = c4 + c7 * x3;
    P3[d] = c3 + c6 * x2;
    Q3[d] = c5 + c7 * x2;
  }
  T ka = T(1), kb = T(0);
  if (COEF) {
    const T *K = Gc + 24;
    ka = K[0] + K[2] * x2 + (K[3] + K[6] * x2) * x3;
    kb = K[1] + K[4] * x2 + (K[5] + K[7] * x2) * x3;
  }
  T v[N], ux[N], dxv[N];
  // ---- z-pencil (x, y) = (pa, pb): B along z
  eo_contract<T, N, MatB<N>, 1>(r, v);
#pragma unroll
  for (int c = 0; c < N; c++) w0[IX(pa, pb, c)] = v[c];
  __syncthreads();
  // ---- y-pencil (x = pa, z = pb): B along y
#pragma unroll
  for (int yy = 0; yy < N; yy++) r[yy] = u0[IX(pa, yy, pb)];
  eo_contract<T, N, MatB<N>, 1>(r, v);
#pragma unroll
  for (int b = 0; b < N; b++) w0[IX(pa, b, pb)] = v[b];
  __syncthreads();
  // ---- x-pencil (y = pa, z = pb): B along x -> u at the points (kept in registers)
#pragma unroll
  for (int xx = 0; xx < N; xx++) r[xx] = u0[IX(xx, pa, pb)];
  eo_contract<T, N, MatB<N>, 1>(r, ux);
#pragma unroll
  for (int a = 0; a < N; a++) w0[IX(a, pa, pb)] = ux[a];
  __syncthreads();
  // ---- z-pencil (x = pa, y = pb): z-derivative into V
#pragma unroll
  for (int c = 0; c < N; c++) r[c] = u0[IX(pa, pb, c)];
  eo_contract<T, N, MatD<N>, -1>(r, v);
#pragma unroll
  for (int c = 0; c < N; c++) w1[IX(pa, pb, c)] = v[c];
  __syncthreads();
  // ---- y-pencil (x = pa, z = pb): y-derivative over u in U (each lane its own pencil)
#pragma unroll
  for (int yy = 0; yy < N; yy++) r[yy] = u0[IX(pa, yy, pb)];
  eo_contract<T, N, MatD<N>, -1>(r, v);
#pragma unroll
  for (int b = 0; b < N; b++) w0[IX(pa, b, pb)] = v[b];
  __syncthreads();
  // ---- pointwise on the x-pencil (y = pa, z = pb); the x-derivative from the kept u
  {
    T f0[N];
    eo_contract<T, N, MatD<N>, -1>(ux, dxv);
#pragma unroll
    for (int a = 0; a < N; a++) {
      const T x1 = TB::g(a);
      const T *j1 = P1;
      T j2[3], j3[3];
#pragma unroll
      for (int d = 0; d < 3; d++) {
        j2[d] = P2[d] + x1 * Q2[d];
        j3[d] = P3[d] + x1 * Q3[d];
      }
      // adjugate rows: r0 = j2 x j3, r1 = j3 x j1, r2 = j1 x j2  (J^{-1} = rows / det)
      const T r0[3] = {j2[1] * j3[2] - j2[2] * j3[1], j2[2] * j3[0] - j2[0] * j3[2], j2[0] * j3[1] - j2[1] * j3[0]};
      const T r1[3] = {j3[1] * j1[2] - j3[2] * j1[1], j3[2] * j1[0] - j3[0] * j1[2], j3[0] * j1[1] - j3[1] * j1[0]};
      const T r2[3] = {j1[1] * j2[2] - j1[2] * j2[1], j1[2] * j2[0] - j1[0] * j2[2], j1[0] * j2[1] - j1[1] * j2[0]};
      const T det = j1[0] * r0[0] + j1[1] * r0[1] + j1[2] * r0[2];
      const T adet = det < T(0) ? -det : det;
      const T wq = wyz * TB::w(a);
      const T kq = COEF ? ka + kb * x1 : T(1);
      const T sc = wq * kq * recip(adet);
      const T dx = dxv[a], dy = u0[IX(a, pa, pb)], dz = u1[IX(a, pa, pb)];
      const T gx = r0[0] * dx + r1[0] * dy + r2[0] * dz;
      const T gy = r0[1] * dx + r1[1] * dy + r2[1] * dz;
      const T gz = r0[2] * dx + r1[2] * dy + r2[2] * dz;
      f0[a] = sc * (r0[0] * gx + r0[1] * gy + r0[2] * gz);
      w0[IX(a, pa, pb)] = sc * (r1[0] * gx + r1[1] * gy + r1[2] * gz);
      w1[IX(a, pa, pb)] = sc * (r2[0] * gx + r2[1] * gy + r2[2] * gz);
      if constexpr (MASS) ux[a] = wq * adet * ux[a];
    }
    // x-transpose of the derivative, in registers (plus the mass term)
    eo_contract<T, N, MatDt<N>, -1>(f0, v);
    if constexpr (MASS) {
#pragma unroll
      for (int a = 0; a < N; a++) v[a] += ux[a];
    }
  }
  __syncthreads();
  // ---- z-pencil (x = pa, y = pb): D^T along z of the z-flux in V; y-pencil (x = pa,
  // z = pb): D^T along y of the y-flux in U (disjoint buffers, each lane its own pencils)
  {
    T t[N], q[N];
#pragma unroll
    for (int c = 0; c < N; c++) t[c] = u1[IX(pa, pb, c)];
    eo_contract<T, N, MatDt<N>, -1>(t, q);
#pragma unroll
    for (int c = 0; c < N; c++) w1[IX(pa, pb, c)] = q[c];
#pragma unroll
    for (int yy = 0; yy < N; yy++) t[yy] = u0[IX(pa, yy, pb)];
    eo_contract<T, N, MatDt<N>, -1>(t, q);
#pragma unroll
    for (int b = 0; b < N; b++) w0[IX(pa, b, pb)] = q[b];
  }
  __syncthreads();
  // ---- x-pencil (y = pa, z = pb): sum the three terms, B^T along x
#pragma unroll
  for (int a = 0; a < N; a++) v[a] += u0[IX(a, pa, pb)] + u1[IX(a, pa, pb)];
  eo_contract<T, N, MatBt<N>, 1>(v, r);
#pragma unroll
  for (int i = 0; i < N; i++) w0[IX(i, pa, pb)] = r[i];
  __syncthreads();
  // ---- y-pencil (x = pa, z = pb): B^T along y
#pragma unroll
  for (int b = 0; b < N; b++) r[b] = u0[IX(pa, b, pb)];
  eo_contract<T, N, MatBt<N>, 1>(r, v);
#pragma unroll
  for (int j = 0; j < N; j++) w0[IX(pa, j, pb)] = v[j];
  __syncthreads();
  // ---- z-pencil (x, y) = (pa, pb): B^T along z
#pragma unroll
  for (int c = 0; c < N; c++) r[c] = u0[IX(pa, pb, c)];
  eo_contract<T, N, MatBt<N>, 1>(r, v);
#pragma unroll
  for (int l = 0; l < N; l++) r[l] = v[l];
}

// Processes cell batch b (cells c0 + b*EPB ... c0 + b*EPB + EPB - 1) of one operator
// on the calling wavefront, using `lds` (hex_lds_size<T, N, GRAD>() values).
// PATCH: b is a patch of EPB cell slots (cell arrays in slot order); the results are
// summed into the patch's nodes in LDS and each node written once (HexArgs patch
// fields), instead of the atomic or coloured scatter into y.
template <typename T, int N, int KIND, bool ATOMIC, int WPB = 1, bool PATCH = false>
__device__ __forceinline__ void hex_cells(const HexArgs<T> &A, const int64_t b, const int comp, T *lds) {
  using TB = TabT<T, N>;
  constexpr int NN = N * N, N3 = NN * N, EPB = hex_epb<N, WPB>();
  constexpr bool GRAD = KIND != K_MASS;
  constexpr bool MASS = KIND == K_MASS || KIND == K_HELM;
  constexpr bool COEF = KIND == K_MASS || KIND == K_POIS;
  constexpr int SY = HexLds<N>::SY, SZ = HexLds<N>::SZ, SE = HexLds<N>::SE;
  constexpr int NBUF = hex_nbuf<N, GRAD>();
  T *const base = lds;
  T *s0 = base;
  T *s1 = base + (NBUF > 1 ? EPB * SE : 0);
  T *s2 = base + (NBUF > 2 ? 2 * EPB * SE : 0);
  T *sg = base + NBUF * EPB * SE;

  const int t = threadIdx.x;
  const bool mirror = t >= EPB * NN;
  // A mirror lane duplicates the pencil of lane t - EPB n^2. In a one-wavefront
  // workgroup it runs in lockstep with that lane, so its identical LDS stores are
  // harmless; across wavefronts its in-place read-then-write could interleave with
  // the original's, so there it writes into a discard buffer instead. It never
  // scatters.
  const int tt = mirror ? t - EPB * NN : t;
  const int le = tt / NN, p = tt - le * NN;
  const int pa = p % N, pb = p / N;
  const int nc = A.ncomp;

  // One batch of EPB cells per call: map, geometry and the first component's
  // gathers are issued together, then each component is processed in turn.
  int idx_cur[N], gidx[N];  // scatter (internal node) and gather positions
  int first = 0x7fffffff;   // nodes from this id up are first touched by this cell
  {
    const int64_t c = A.c0 + b * EPB + le;
    bool ok = c < A.c1;
    if (ok && A.cell_user) {
      const int64_t u = A.cell_user[c];
      ok = u >= A.ulo && u < A.uhi;
    }
    if (!ATOMIC && !PATCH && ok && A.first) first = A.first[c];
    const int64_t off = (ok ? c : A.c0) * N3 + pa + N * pb;
#pragma unroll
    for (int l = 0; l < N; l++) idx_cur[l] = ok ? A.map[off + NN * l] : -1;
#pragma unroll
    for (int l = 0; l < N; l++) gidx[l] = A.gmap ? (ok ? A.gmap[off + NN * l] : -1) : idx_cur[l];
  }
  for (int i = t; i < EPB * 32; i += 64 * WPB) {
    const int e = i >> 5, j = i & 31;
    const int64_t c = A.c0 + b * EPB + e;
    T v = T(0);
    if (c < A.c1) {
      if (j < 24) v = A.geo[c * 24 + j];
      else if (COEF && A.coef) v = A.coef[c * 8 + (j - 24)];
      else if (j == 24) v = T(1);  // coefficient 1 when absent
    } else if (j == 0 || j == 4 || j == 8) {
      v = T(1);  // cells past the end: unit-cube geometry keeps the arithmetic finite
    }
    sg[i] = v;
  }
  __syncthreads();

  T *u0 = s0 + le * SE;
  T *u1 = s1 + (NBUF > 1 ? le * SE : 0);
  T *u2 = s2 + (NBUF > 2 ? le * SE : 0);
  const T *Gc = sg + le * 32;
  // One component per call: the body has no loop over components, so the compiler
  // materialises the table constants at their uses instead of keeping them live
  // across iterations (which doubled the register count).
  T yv[N], r[N];
#pragma unroll
  for (int l = 0; l < N; l++) r[l] = gidx[l] >= 0 ? A.x[(int64_t)gidx[l] * nc + comp] : T(0);
  if constexpr (!ATOMIC && !PATCH) {
    // no other cell of this launch touches these nodes: read y now, write it at the end
    // (nodes this cell touches first are stored without reading)
#pragma unroll
    for (int l = 0; l < N; l++)
      yv[l] = (!mirror && idx_cur[l] >= 0 && idx_cur[l] < first) ? A.y[(int64_t)idx_cur[l] * nc + comp] : T(0);
  }
  T *dump = sg + EPB * 32;  // the discard buffer (WPB > 1)
  const bool discard = WPB > 1 && mirror;
  if constexpr (NBUF == 2)
    hex_pencil_stages2<T, N, KIND, WPB>(r, Gc, u0, u1, discard ? dump : u0, discard ? dump : u1, pa, pb);
  else
    hex_pencil_stages<T, N, KIND, WPB>(r, Gc, u0, u1, u2, discard ? dump : u0, discard ? dump : u1,
                                       discard ? dump : u2, pa, pb);
  if constexpr (PATCH) {
    __syncthreads();  // every lane has finished reading the stage buffers, reused below
    const int n0 = A.pnptr[b], nn = A.pnptr[b + 1] - n0;
    // nn <= EPB n^3 <= the stage buffers' size. FP32 sums are kept in FP64 where the
    // workgroup's LDS holds them (LDS FP32 atomic adds measured several times slower
    // than FP64 ones)
    using Acc = std::conditional_t<(sizeof(T) == 4 && 2 * EPB * N3 <= hex_lds_size<T, N, GRAD, WPB>()), double, T>;
    Acc *acc = reinterpret_cast<Acc *>(base);
    for (int e = t; e < nn; e += 64 * WPB) acc[e] = Acc(0);
    __syncthreads();
    if (!mirror) {
      const uint16_t *lp = A.plmap + (b * EPB + le) * N3 + pa + N * pb;
#pragma unroll
      for (int l = 0; l < N; l++) {
        const int li = lp[NN * l];
        if (li != kSlotSkip) atomicAdd(&acc[li], (Acc)r[l]);
      }
    }
    __syncthreads();
    for (int e = t; e < nn; e += 64 * WPB) {
      const int32_t o = A.pout[n0 + e];
      if (o & kSharedOut) {
        A.psbuf[(int64_t)(o & (kSharedOut - 1)) * nc + comp] = (T)acc[e];
      } else {
        T *d = A.y + (int64_t)o * nc + comp;
        *d = A.accumulate ? *d + (T)acc[e] : (T)acc[e];
      }
    }
    __syncthreads();
    return;
  }
#pragma unroll
  for (int l = 0; l < N; l++) {
    const int idx = mirror ? -1 : idx_cur[l];
    if (idx >= 0) {
      if constexpr (ATOMIC) atomic_add_f(&A.y[(int64_t)idx * nc + comp], r[l]);
      else A.y[(int64_t)idx * nc + comp] = yv[l] + r[l];
    }
  }
  __syncthreads();
}

#undef IX

// Resident wavefronts per SIMD the compiler must allow (register cap 512 / waves):
// the FP64 gradient kernels from n = 6 on fit four wavefronts per SIMD in LDS, which
// Helmholtz reaches only under the 128-register cap (a spill of under 64 bytes per
// lane; measured 3 % faster than three wavefronts without it).
template <typename T, int N, int KIND> constexpr int hex_min_waves() {
  return (sizeof(T) == 8 && N >= 6 && KIND != K_MASS) ? 4 : 1;
}

// Work item = (cell batch, component): the ncomp components of a batch are
// consecutive items, so they run on the same XCD at about the same time and share
// the cache lines of their interleaved values.
template <typename T, int N, int KIND, bool ATOMIC>
__global__ void __launch_bounds__(64 * hex_wpb<N>(), (hex_min_waves<T, N, KIND>())) hex_apply_kernel(const HexArgs<T> A) {
  constexpr int WPB = hex_wpb<N>(), EPB = hex_epb<N, WPB>();
  __shared__ __align__(16) T lds[hex_lds_size<T, N, KIND != K_MASS, WPB>()];
  const int64_t nb = (A.c1 - A.c0 + EPB - 1) / EPB;  // cell batches
  const int64_t vb = xcd_batch(blockIdx.x, nb * A.ncomp);
  // the grid has fewer than 2^31 items, so the split uses 32-bit division
  if (vb < nb * A.ncomp) hex_cells<T, N, KIND, ATOMIC, WPB>(A, (int)vb / A.ncomp, (int)vb % A.ncomp, lds);
}

// Patch scatter: one workgroup per (patch of EPB cells, component).
template <typename T, int N, int KIND>
__global__ void __launch_bounds__(64 * hex_wpb<N>()) hex_patch_kernel(const HexArgs<T> A, const int npatch) {
  constexpr int WPB = hex_wpb<N>();
  __shared__ __align__(16) T lds[hex_lds_size<T, N, KIND != K_MASS, WPB>()];
  const int64_t vb = xcd_batch(blockIdx.x, (int64_t)npatch * A.ncomp);
  if (vb < (int64_t)npatch * A.ncomp)
    hex_cells<T, N, KIND, false, WPB, true>(A, (int)vb / A.ncomp, (int)vb % A.ncomp, lds);
}

template <typename T, int N>
static int launch_patch_n(int kind, const HexArgs<T> &a, int npatch, hipStream_t s) {
  constexpr int WPB = hex_wpb<N>();
  if (npatch <= 0) return MF_OK;
  dim3 grid((unsigned)xcd_grid((int64_t)npatch * a.ncomp)), block(64 * WPB);
  switch (kind) {
    case K_MASS: hex_patch_kernel<T, N, K_MASS><<<grid, block, 0, s>>>(a, npatch); break;
    case K_HELM: hex_patch_kernel<T, N, K_HELM><<<grid, block, 0, s>>>(a, npatch); break;
    case K_LAP: hex_patch_kernel<T, N, K_LAP><<<grid, block, 0, s>>>(a, npatch); break;
    case K_POIS: hex_patch_kernel<T, N, K_POIS><<<grid, block, 0, s>>>(a, npatch); break;
    default: return fail(MF_EUNSUPPORTED, "hex patch kernel: operator kind");
  }
  MF_HIP(hipGetLastError());
  return MF_OK;
}

template <typename T>
int launch_hex_cell_patches(int N, int kind, const HexArgs<T> &a, int npatch, hipStream_t s) {
  switch (N) {
    case 3: return launch_patch_n<T, 3>(kind, a, npatch, s);
    case 4: return launch_patch_n<T, 4>(kind, a, npatch, s);
    case 5: return launch_patch_n<T, 5>(kind, a, npatch, s);
    case 6: return launch_patch_n<T, 6>(kind, a, npatch, s);
    case 7: return launch_patch_n<T, 7>(kind, a, npatch, s);
  }
  return fail(MF_EUNSUPPORTED, "hex patch kernel: degree");
}
template int launch_hex_cell_patches<double>(int, int, const HexArgs<double> &, int, hipStream_t);
template int launch_hex_cell_patches<float>(int, int, const HexArgs<float> &, int, hipStream_t);
int hex_cells_per_patch(int N) {
  switch (N) {
    case 3: return hex_epb<3, hex_wpb<3>()>();
    case 4: return hex_epb<4, hex_wpb<4>()>();
    case 5: return hex_epb<5, hex_wpb<5>()>();
    case 6: return hex_epb<6, hex_wpb<6>()>();
    case 7: return hex_epb<7, hex_wpb<7>()>();
  }
  return 0;
}

// ---------------------------------------------------------------------------------- batched apply
// One persistent launch applies many operators (uneven sizes and degrees): each
// wavefront walks a device work list of (operator, batch range) items and runs the
// degree's code path. Items of operators whose solve has stopped are skipped.
template <typename T> struct HexBatchOp {
  HexArgs<T> a;
  int N;
  int pad;
};
struct HexBatchItem {
  int32_t op;
  int32_t pad;
  int64_t b0, b1;  // cell batches [b0, b1) of the operator (EPB(N) cells each)
};

template <typename T, int KIND, bool PERSIST>
__global__ void __launch_bounds__(64) hex_batch_kernel(const HexBatchOp<T> *__restrict__ ops,
                                                       const HexBatchItem *__restrict__ items, int nitems,
                                                       const int *__restrict__ stop, int stop_stride) {
  constexpr bool GRAD = KIND != K_MASS;
  constexpr int L2 = hex_lds_size<T, 2, GRAD>(), L3 = hex_lds_size<T, 3, GRAD>(), L4 = hex_lds_size<T, 4, GRAD>(),
                L5 = hex_lds_size<T, 5, GRAD>(), L6 = hex_lds_size<T, 6, GRAD>();
  constexpr int LA = L2 > L3 ? L2 : L3, LB = L4 > L5 ? L4 : L5, LC = LA > LB ? LA : LB;
  constexpr int LM = LC > L6 ? LC : L6;
  __shared__ __align__(16) T lds[LM];
  if constexpr (PERSIST) {
    // wavefronts stride over the work list and the batch ranges of their items
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
      const HexBatchItem w = items[it];
      if (stop && stop[(int64_t)w.op * stop_stride]) continue;
      const HexArgs<T> A = ops[w.op].a;
      for (int64_t b = w.b0; b < w.b1; b++) {
        switch (ops[w.op].N) {
          case 2: hex_cells<T, 2, KIND, true>(A, b, 0, lds); break;
          case 3: hex_cells<T, 3, KIND, true>(A, b, 0, lds); break;
          case 4: hex_cells<T, 4, KIND, true>(A, b, 0, lds); break;
          case 5: hex_cells<T, 5, KIND, true>(A, b, 0, lds); break;
          case 6: hex_cells<T, 6, KIND, true>(A, b, 0, lds); break;
        }
        __syncthreads();
      }
    }
  } else {
    // one wavefront per single-batch item: no loop, so the compiler keeps the
    // tables as rematerialised constants instead of loop-invariant registers
    const int64_t wi = xcd_batch(blockIdx.x, nitems);  // contiguous item ranges per XCD
    if (wi >= nitems) return;
    const HexBatchItem w = items[wi];
    if (stop && stop[(int64_t)w.op * stop_stride]) return;
    const HexArgs<T> A = ops[w.op].a;
    switch (ops[w.op].N) {
      case 2: hex_cells<T, 2, KIND, true>(A, w.b0, 0, lds); break;
      case 3: hex_cells<T, 3, KIND, true>(A, w.b0, 0, lds); break;
      case 4: hex_cells<T, 4, KIND, true>(A, w.b0, 0, lds); break;
      case 5: hex_cells<T, 5, KIND, true>(A, w.b0, 0, lds); break;
      case 6: hex_cells<T, 6, KIND, true>(A, w.b0, 0, lds); break;
    }
  }
}

// grid <= 0: one wavefront per work item (items must then hold one batch each);
// grid > 0: a persistent grid of that many wavefronts.
template <typename T>
int launch_hex_batch(int kind, const void *ops, const void *items, int nitems, int grid, const int *stop,
                     int stop_stride, hipStream_t s) {
  if (nitems <= 0) return MF_OK;
  const HexBatchOp<T> *o = (const HexBatchOp<T> *)ops;
  const HexBatchItem *w = (const HexBatchItem *)items;
  const bool persist = grid > 0;
  const unsigned g = persist ? (unsigned)grid : (unsigned)xcd_grid(nitems);
#define MF_BATCH_LAUNCH(K)                                                                    \
  if (persist) hex_batch_kernel<T, K, true><<<g, 64, 0, s>>>(o, w, nitems, stop, stop_stride); \
  else hex_batch_kernel<T, K, false><<<g, 64, 0, s>>>(o, w, nitems, stop, stop_stride);
  switch (kind) {
    case K_MASS: MF_BATCH_LAUNCH(K_MASS) break;
    case K_HELM: MF_BATCH_LAUNCH(K_HELM) break;
    case K_LAP: MF_BATCH_LAUNCH(K_LAP) break;
    case K_POIS: MF_BATCH_LAUNCH(K_POIS) break;
    default: return fail(MF_EUNSUPPORTED, "batched kernel: operator kind");
  }
#undef MF_BATCH_LAUNCH
  MF_HIP(hipGetLastError());
  return MF_OK;
}
template int launch_hex_batch<double>(int, const void *, const void *, int, int, const int *, int, hipStream_t);
template int launch_hex_batch<float>(int, const void *, const void *, int, int, const int *, int, hipStream_t);

size_t hex_batch_op_bytes(int precision) {
  return precision == MF_F64 ? sizeof(HexBatchOp<double>) : sizeof(HexBatchOp<float>);
}
size_t hex_batch_item_bytes() { return sizeof(HexBatchItem); }
int hex_cells_per_batch(int N) { return 64 / (N * N); }

// ---------------------------------------------------------------------------------- diagonal
// diag_i = sum_q [ grad_ref phi_i^T G grad_ref phi_i + m phi_i^2 ], one thread per cell node;
// the per-point G (6) and mass factor m are computed once per point into LDS.
template <int N> constexpr int hexd_epb() { return (N * N * N >= 256) ? 1 : 256 / (N * N * N); }

template <typename T, int N, int KIND>
__global__ void __launch_bounds__(512) hex_diag_kernel(const HexArgs<T> A) {
  using TB = TabT<T, N>;
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
    const T x1 = TB::g(a), x2 = TB::g(b), x3 = TB::g(c);
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
    const T wq = TB::w(a) * TB::w(b) * TB::w(c);
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
        const T bi = TB::B(a, i), bj = TB::B(b, j), bl = TB::B(c, l);
        const T vv = bi * bj * bl;
        T s = sG[le][6][q] * vv * vv;
        if (GRAD) {
          const T d0 = TB::dB(a, i) * bj * bl, d1 = bi * TB::dB(b, j) * bl, d2 = bi * bj * TB::dB(c, l);
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
template <typename T, int N, bool AT>
static int launch_apply_na(int kind, const HexArgs<T> &a, hipStream_t s) {
  constexpr int WPB = hex_wpb<N>(), EPB = hex_epb<N, WPB>();
  const int64_t nc = a.c1 - a.c0;
  if (nc <= 0) return MF_OK;
  const int64_t nb = (nc + EPB - 1) / EPB;
  void *fn = nullptr;
  switch (kind) {
    case K_MASS: fn = (void *)hex_apply_kernel<T, N, K_MASS, AT>; break;
    case K_HELM: fn = (void *)hex_apply_kernel<T, N, K_HELM, AT>; break;
    case K_LAP: fn = (void *)hex_apply_kernel<T, N, K_LAP, AT>; break;
    case K_POIS: fn = (void *)hex_apply_kernel<T, N, K_POIS, AT>; break;
    default: return fail(MF_EUNSUPPORTED, "hex kernel: operator kind");
  }
  (void)fn;
  dim3 grid((unsigned)xcd_grid(nb * a.ncomp)), block(64 * WPB);  // one (cell batch, component) per workgroup
  switch (kind) {
    case K_MASS: hex_apply_kernel<T, N, K_MASS, AT><<<grid, block, 0, s>>>(a); break;
    case K_HELM: hex_apply_kernel<T, N, K_HELM, AT><<<grid, block, 0, s>>>(a); break;
    case K_LAP: hex_apply_kernel<T, N, K_LAP, AT><<<grid, block, 0, s>>>(a); break;
    case K_POIS: hex_apply_kernel<T, N, K_POIS, AT><<<grid, block, 0, s>>>(a); break;
  }
  MF_HIP(hipGetLastError());
  return MF_OK;
}

template <typename T, int N>
static int launch_apply_n(int kind, const HexArgs<T> &a, bool atomic, hipStream_t s) {
  return atomic ? launch_apply_na<T, N, true>(kind, a, s) : launch_apply_na<T, N, false>(kind, a, s);
}

template <typename T, int N>
static int launch_diag_n(int kind, const HexArgs<T> &a, hipStream_t s) {
  constexpr int EPB = hexd_epb<N>();
  const int64_t nc = a.c1 - a.c0;
  if (nc <= 0) return MF_OK;
  dim3 grid((unsigned)((nc + EPB - 1) / EPB)), block(EPB * N * N * N);
  switch (kind) {
    case K_MASS: hex_diag_kernel<T, N, K_MASS><<<grid, block, 0, s>>>(a); break;
    case K_HELM: hex_diag_kernel<T, N, K_HELM><<<grid, block, 0, s>>>(a); break;
    case K_LAP: hex_diag_kernel<T, N, K_LAP><<<grid, block, 0, s>>>(a); break;
    case K_POIS: hex_diag_kernel<T, N, K_POIS><<<grid, block, 0, s>>>(a); break;
    default: return fail(MF_EUNSUPPORTED, "hex diagonal: operator kind");
  }
  MF_HIP(hipGetLastError());
  return MF_OK;
}

template <typename T>
int launch_hex_apply(int N, int kind, const HexArgs<T> &a, bool atomic, hipStream_t s) {
  switch (N) {
    case 2: return atomic ? launch_apply_n<T, 2>(kind, a, true, s) : launch_hex_q1_coloured<T>(kind, a, s);
    case 3: return launch_apply_n<T, 3>(kind, a, atomic, s);
    case 4: return launch_apply_n<T, 4>(kind, a, atomic, s);
    case 5: return launch_apply_n<T, 5>(kind, a, atomic, s);
    case 6: return launch_apply_n<T, 6>(kind, a, atomic, s);
    case 7: return launch_apply_n<T, 7>(kind, a, atomic, s);
  }
  return fail(MF_EUNSUPPORTED, "hex kernel: degree");
}

template <typename T>
int launch_hex_diag(int N, int kind, const HexArgs<T> &a, hipStream_t s) {
  switch (N) {
    case 2: return launch_diag_n<T, 2>(kind, a, s);
    case 3: return launch_diag_n<T, 3>(kind, a, s);
    case 4: return launch_diag_n<T, 4>(kind, a, s);
    case 5: return launch_diag_n<T, 5>(kind, a, s);
    case 6: return launch_diag_n<T, 6>(kind, a, s);
    case 7: return launch_diag_n<T, 7>(kind, a, s);
  }
  return fail(MF_EUNSUPPORTED, "hex diagonal: degree");
}

template int launch_hex_apply<double>(int, int, const HexArgs<double> &, bool, hipStream_t);
template int launch_hex_apply<float>(int, int, const HexArgs<float> &, bool, hipStream_t);
template int launch_hex_diag<double>(int, int, const HexArgs<double> &, hipStream_t);
template int launch_hex_diag<float>(int, int, const HexArgs<float> &, hipStream_t);



}  // namespace mf
