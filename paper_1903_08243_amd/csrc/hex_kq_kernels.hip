// Scalar operators (mass, Helmholtz, Laplacian with one or three components, Poisson)
// on trilinear hexahedra with the paper's quadrature of Q = k+2 Gauss points per
// direction (Table 2's hex rows), sum-factorised on pencils like the k+1 kernel.
//
// The nodal values of Q_k are interpolated to the Q^3 points by three rectangular
// passes with B[a][i] = l_i(g_a) (Q x N, N = k+1; Sections 3 and 4.2.4). The
// interpolant is a polynomial of degree k < Q in each direction, so the collocation
// derivative on the Q Gauss points differentiates it exactly: from there on the
// stages are those of the k+1 kernel on Q-point pencils (derivatives, the pointwise
// Jacobian of the trilinear map and the fluxes of Section 2.1, the transposed
// derivatives), and three transposed rectangular passes with B^T integrate back to
// the nodes.
//
// GPU mapping: a lane holds one pencil; a cell owns Q^2 lanes (the point pencils of
// the middle stages); the first and last passes have N^2 and N Q pencils, so some of
// the cell's lanes idle there. A workgroup of WPB wavefronts holds EPB = floor(64 WPB /
// Q^2) cells and three padded Q^3 LDS buffers per cell (two from Q = 6 on, where the
// pointwise stage runs on x-pencils whose lanes keep u and the x-flux in registers);
// one workgroup per (cell batch, component).
#include "hex_common.h"

namespace mf {

namespace {

// Rectangular interpolation matrices of the k+2 rule and their transposes.
template <int N> struct MatBR { static constexpr double at(int a, int i) { return HexR<N>::B[a][i]; } };
template <int N> struct MatBRt { static constexpr double at(int i, int a) { return HexR<N>::B[a][i]; } };

// out[a] = sum_i M(a, i) in[i] for an NO x NI matrix with the reflection symmetry
// M(NO-1-a, NI-1-i) = SIGN M(a, i) (symmetric points and nodes): the even and odd
// parts of the input give each output pair (a, NO-1-a) from two half-size products.
template <int NI, int NO, typename M, int SIGN> constexpr bool rect_reflection_symmetric() {
  for (int a = 0; a < NO; a++)
    for (int i = 0; i < NI; i++) {
      const double d = M::at(a, i) - SIGN * M::at(NO - 1 - a, NI - 1 - i);
      const double m = M::at(a, i) < 0 ? -M::at(a, i) : M::at(a, i);
      if ((d < 0 ? -d : d) > 1e-13 * (m > 1 ? m : 1)) return false;
    }
  return true;
}

template <typename T, int NI, int NO, typename M, int SIGN>
__device__ __forceinline__ void eo_rect(const T *in, T *out) {
  static_assert(rect_reflection_symmetric<NI, NO, M, SIGN>(), "1D table lacks the reflection symmetry");
  constexpr int HI = NI / 2, HO = NO / 2;
  T e[HI > 0 ? HI : 1], o[HI > 0 ? HI : 1];
#pragma unroll
  for (int i = 0; i < HI; i++) {
    e[i] = in[i] + in[NI - 1 - i];
    o[i] = in[i] - in[NI - 1 - i];
  }
#pragma unroll
  for (int a = 0; a < HO; a++) {
    T pe = T(0), po = T(0);
#pragma unroll
    for (int i = 0; i < HI; i++) {
      pe += T(0.5 * (M::at(a, i) + M::at(a, NI - 1 - i))) * e[i];
      po += T(0.5 * (M::at(a, i) - M::at(a, NI - 1 - i))) * o[i];
    }
    if constexpr (NI % 2 == 1) pe += T(M::at(a, HI)) * in[HI];
    out[a] = pe + po;
    out[NO - 1 - a] = SIGN > 0 ? pe - po : po - pe;
  }
  if constexpr (NO % 2 == 1) {
    T m = T(0);
#pragma unroll
    for (int i = 0; i < HI; i++) m += T(M::at(HO, i)) * (SIGN > 0 ? e[i] : o[i]);
    if constexpr (NI % 2 == 1 && SIGN > 0) m += T(M::at(HO, HI)) * in[HI];
    out[HO] = m;
  }
}

// Padded LDS layout of one cell's Q^3 buffer: entry (x, y, z) at z SZ + y SY + x
// (the strides of the k+1 kernel for the same pencil length; for 8 points, strides
// that keep the three pencil directions of a wavefront on distinct banks).
template <int Q> struct KqLds;
template <> struct KqLds<3> { static constexpr int SY = 3, SZ = 9, SE = 27; };
template <> struct KqLds<4> { static constexpr int SY = 4, SZ = 19, SE = 80; };
template <> struct KqLds<5> { static constexpr int SY = 5, SZ = 25, SE = 135; };
template <> struct KqLds<6> { static constexpr int SY = 9, SZ = 54, SE = 324; };
template <> struct KqLds<7> { static constexpr int SY = 7, SZ = 52, SE = 364; };
template <> struct KqLds<8> { static constexpr int SY = 9, SZ = 72, SE = 576; };

}  // namespace

template <int Q> constexpr int hexkq_wpb() { return Q == 6 ? 2 : Q == 7 ? 4 : 1; }  // Q = 8: a wavefront per cell
template <int Q> constexpr int hexkq_epb() { return hexkq_wpb<Q>() * 64 / (Q * Q); }
// Q^3 buffers per cell: one without gradients; with gradients three, or two from
// Q = 6 on (pointwise stage on x-pencils, as in the k+1 kernel from n = 6 on)
template <int Q, bool GRAD> constexpr int hexkq_nbuf() { return GRAD ? (Q >= 6 ? 2 : 3) : 1; }
template <int Q, bool GRAD> constexpr int hexkq_lds() {
  return hexkq_epb<Q>() * (KqLds<Q>::SE * hexkq_nbuf<Q, GRAD>() + 32);
}

// FP64 kernels with two buffers: capped at 128 VGPRs, four wavefronts per SIMD (what
// their LDS allows at Q = 7 and 8)
template <typename T, int Q, int KIND> constexpr int hexkq_min_waves() {
  return (sizeof(T) == 8 && hexkq_nbuf<Q, KIND != MF_OP_MASS>() == 2) ? 4 : 1;
}

#define KQ(x, y, z) ((z) * SZ + (y) * SY + (x))
template <typename T, int N, int Q, int KIND, bool ATOMIC>
__global__ void __launch_bounds__(64 * hexkq_wpb<Q>(), (hexkq_min_waves<T, Q, KIND>()))
    hex_kq_kernel(const HexQArgs<T> A) {
  using TB = TabT<T, Q>;  // Gauss points, weights and collocation derivative of the Q-point rule
  constexpr int WPB = hexkq_wpb<Q>(), EPB = hexkq_epb<Q>(), QQ = Q * Q, NN = N * N, N3 = NN * N;
  constexpr bool GRAD = KIND != MF_OP_MASS;
  constexpr bool MASS = KIND == MF_OP_MASS || KIND == MF_OP_HELMHOLTZ;
  constexpr bool COEF = KIND == MF_OP_MASS || KIND == MF_OP_POISSON;
  constexpr int NBUF = hexkq_nbuf<Q, GRAD>();
  constexpr bool TWO = NBUF == 2;
  constexpr int SY = KqLds<Q>::SY, SZ = KqLds<Q>::SZ, SE = KqLds<Q>::SE;
  __shared__ __align__(16) T lds[hexkq_lds<Q, GRAD>()];
  const int nc = A.ncomp;
  const int64_t nb = (A.c1 - A.c0 + EPB - 1) / EPB;
  const int64_t item = xcd_batch(blockIdx.x, nb * nc);
  if (item >= nb * nc) return;  // whole workgroup
  const int64_t b = item / nc;
  const int comp = (int)(item % nc);
  const int t = threadIdx.x;
  const bool act = t < EPB * QQ;  // lanes past the last cell idle through every stage
  const int tt = act ? t : 0;
  const int le = tt / QQ, p = tt - le * QQ;
  const int pa = p % Q, pb = p / Q;
  T *s0 = lds, *s1 = lds + (NBUF > 1 ? EPB * SE : 0), *s2 = lds + (NBUF > 2 ? 2 * EPB * SE : 0);
  T *sg = lds + NBUF * EPB * SE;
  // map entries of this lane's nodal z-pencil (pa, pb, *), pa, pb < N
  const bool nodal = act && pa < N && pb < N;
  int idx[N], gidx[N];
  {
    const int64_t c = A.c0 + b * EPB + le;
    bool ok = nodal && c < A.c1;
    if (ok && A.cell_user) {
      const int64_t u = A.cell_user[c];
      ok = u >= A.ulo && u < A.uhi;
    }
    const int64_t off = (ok ? c : A.c0) * N3 + pa + N * pb;
#pragma unroll
    for (int l = 0; l < N; l++) idx[l] = ok ? A.map[off + NN * l] : -1;
#pragma unroll
    for (int l = 0; l < N; l++) gidx[l] = A.gmap ? (ok ? A.gmap[off + NN * l] : -1) : idx[l];
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
  T r[Q], v[Q];
#pragma unroll
  for (int l = 0; l < N; l++) r[l] = gidx[l] >= 0 ? A.x[(int64_t)gidx[l] * nc + comp] : T(0);
  __syncthreads();
  T *u0 = s0 + le * SE, *u1 = s1 + (NBUF > 1 ? le * SE : 0), *u2 = s2 + (NBUF > 2 ? le * SE : 0);
  const T *Gc = sg + le * 32;
  // ---- z: nodal pencil (pa, pb, *) -> Q points along z
  if (nodal) {
    eo_rect<T, N, Q, MatBR<N>, 1>(r, v);
#pragma unroll
    for (int c = 0; c < Q; c++) u0[KQ(pa, pb, c)] = v[c];
  }
  __syncthreads();
  // ---- y: pencil (x node pa, *, z point pb) -> Q points along y
  if (act && pa < N) {
#pragma unroll
    for (int yy = 0; yy < N; yy++) r[yy] = u0[KQ(pa, yy, pb)];
    eo_rect<T, N, Q, MatBR<N>, 1>(r, v);
#pragma unroll
    for (int c = 0; c < Q; c++) u0[KQ(pa, c, pb)] = v[c];
  }
  __syncthreads();
  if constexpr (!TWO) {
    // per-lane geometry of the point pencil (pa, pb, *) for the pointwise stage
    const T x1 = TB::g(pa), x2 = TB::g(pb);
    const T wab = TB::w(pa) * TB::w(pb);
    T A1[3], B1[3], A2[3], B2[3], A3[3];
  #pragma unroll
    for (int d = 0; d < 3; d++) {
      const T c1 = Gc[0 + d], c2 = Gc[3 + d], c3 = Gc[6 + d], c4 = Gc[9 + d], c5 = Gc[12 + d], c6 = Gc[15 + d],
              c7 = Gc[18 + d];
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
    // ---- x: pencil (*, y point pa, z point pb) -> u at the points; x-derivative
    if (act) {
  #pragma unroll
      for (int xx = 0; xx < N; xx++) r[xx] = u0[KQ(xx, pa, pb)];
      eo_rect<T, N, Q, MatBR<N>, 1>(r, v);
  #pragma unroll
      for (int a = 0; a < Q; a++) u0[KQ(a, pa, pb)] = v[a];
      if constexpr (GRAD) {
        eo_contract<T, Q, MatD<Q>, -1>(v, r);
  #pragma unroll
        for (int a = 0; a < Q; a++) u1[KQ(a, pa, pb)] = r[a];
      }
    }
    __syncthreads();
    if constexpr (GRAD) {
      // ---- y-derivative on pencil (x = pa, *, z = pb)
      if (act) {
  #pragma unroll
        for (int yy = 0; yy < Q; yy++) r[yy] = u0[KQ(pa, yy, pb)];
        eo_contract<T, Q, MatD<Q>, -1>(r, v);
  #pragma unroll
        for (int c = 0; c < Q; c++) u2[KQ(pa, c, pb)] = v[c];
      }
      __syncthreads();
    }
    // ---- pointwise on z-pencil (pa, pb, *)
    if (act) {
      T uz[Q], f2[Q], dzv[Q];
  #pragma unroll
      for (int c = 0; c < Q; c++) uz[c] = u0[KQ(pa, pb, c)];
      if constexpr (GRAD) eo_contract<T, Q, MatD<Q>, -1>(uz, dzv);
  #pragma unroll
      for (int c = 0; c < Q; c++) {
        const T x3 = TB::g(c);
        T j1[3], j2[3];
  #pragma unroll
        for (int d = 0; d < 3; d++) {
          j1[d] = A1[d] + x3 * B1[d];
          j2[d] = A2[d] + x3 * B2[d];
        }
        const T *j3 = A3;
        // adjugate rows: r0 = j2 x j3, r1 = j3 x j1, r2 = j1 x j2 (J^{-1} = rows / det)
        const T r0[3] = {j2[1] * j3[2] - j2[2] * j3[1], j2[2] * j3[0] - j2[0] * j3[2], j2[0] * j3[1] - j2[1] * j3[0]};
        const T det = j1[0] * r0[0] + j1[1] * r0[1] + j1[2] * r0[2];
        const T adet = det < T(0) ? -det : det;
        const T wq = wab * TB::w(c);
        const T kq = COEF ? ka + kb * x3 : T(1);
        T mterm = T(0);
        if constexpr (MASS) mterm = wq * adet * kq * uz[c];
        if constexpr (GRAD) {
          const T r1[3] = {j3[1] * j1[2] - j3[2] * j1[1], j3[2] * j1[0] - j3[0] * j1[2], j3[0] * j1[1] - j3[1] * j1[0]};
          const T r2[3] = {j1[1] * j2[2] - j1[2] * j2[1], j1[2] * j2[0] - j1[0] * j2[2], j1[0] * j2[1] - j1[1] * j2[0]};
          const T sc = wq * kq * recip(adet);
          const T dz = dzv[c], dx = u1[KQ(pa, pb, c)], dy = u2[KQ(pa, pb, c)];
          const T gx = r0[0] * dx + r1[0] * dy + r2[0] * dz;
          const T gy = r0[1] * dx + r1[1] * dy + r2[1] * dz;
          const T gz = r0[2] * dx + r1[2] * dy + r2[2] * dz;
          u1[KQ(pa, pb, c)] = sc * (r0[0] * gx + r0[1] * gy + r0[2] * gz);
          u2[KQ(pa, pb, c)] = sc * (r1[0] * gx + r1[1] * gy + r1[2] * gz);
          f2[c] = sc * (r2[0] * gx + r2[1] * gy + r2[2] * gz);
        }
        v[c] = mterm;
      }
      if constexpr (GRAD) {
        eo_contract<T, Q, MatDt<Q>, -1>(f2, dzv);
  #pragma unroll
        for (int c = 0; c < Q; c++) v[c] += dzv[c];
      }
  #pragma unroll
      for (int c = 0; c < Q; c++) u0[KQ(pa, pb, c)] = v[c];
    }
    __syncthreads();
    if constexpr (GRAD) {
      // ---- y-pencil (x = pa, z = pb): add D^T along y of the y-flux
      if (act) {
  #pragma unroll
        for (int yy = 0; yy < Q; yy++) r[yy] = u2[KQ(pa, yy, pb)];
        eo_contract<T, Q, MatDt<Q>, -1>(r, v);
  #pragma unroll
        for (int c = 0; c < Q; c++) u0[KQ(pa, c, pb)] += v[c];
      }
      __syncthreads();
    }
    // ---- x-pencil (y = pa, z = pb): add D^T along x of the x-flux, then B^T to x nodes
    if (act) {
  #pragma unroll
      for (int a = 0; a < Q; a++) v[a] = u0[KQ(a, pa, pb)];
      if constexpr (GRAD) {
  #pragma unroll
        for (int a = 0; a < Q; a++) r[a] = u1[KQ(a, pa, pb)];
        T dv[Q];
        eo_contract<T, Q, MatDt<Q>, -1>(r, dv);
  #pragma unroll
        for (int a = 0; a < Q; a++) v[a] += dv[a];
      }
      eo_rect<T, Q, N, MatBRt<N>, 1>(v, r);
  #pragma unroll
      for (int i = 0; i < N; i++) u0[KQ(i, pa, pb)] = r[i];
    }
    __syncthreads();
  } else {
    // ---- x: pencil (*, y point pa, z point pb) -> u at the points, kept in registers
    T ux[Q];
    if (act) {
#pragma unroll
      for (int xx = 0; xx < N; xx++) r[xx] = u0[KQ(xx, pa, pb)];
      eo_rect<T, N, Q, MatBR<N>, 1>(r, ux);
#pragma unroll
      for (int a = 0; a < Q; a++) u0[KQ(a, pa, pb)] = ux[a];
    }
    __syncthreads();
    // ---- z-derivative on pencil (x = pa, y = pb) into V
    if (act) {
#pragma unroll
      for (int c = 0; c < Q; c++) r[c] = u0[KQ(pa, pb, c)];
      eo_contract<T, Q, MatD<Q>, -1>(r, v);
#pragma unroll
      for (int c = 0; c < Q; c++) u1[KQ(pa, pb, c)] = v[c];
    }
    __syncthreads();
    // ---- y-derivative on pencil (x = pa, z = pb), in place over u in U
    if (act) {
#pragma unroll
      for (int yy = 0; yy < Q; yy++) r[yy] = u0[KQ(pa, yy, pb)];
      eo_contract<T, Q, MatD<Q>, -1>(r, v);
#pragma unroll
      for (int c = 0; c < Q; c++) u0[KQ(pa, c, pb)] = v[c];
    }
    __syncthreads();
    // ---- pointwise on the x-pencil (y = pa, z = pb): Jacobian columns j1 = P1,
    // j2 = P2 + x Q2, j3 = P3 + x Q3 along it; the x-flux stays in registers
    if (act) {
      const T x2 = TB::g(pa), x3 = TB::g(pb);
      const T wyz = TB::w(pa) * TB::w(pb);
      T P1[3], P2[3], Q2[3], P3[3], Q3[3];
#pragma unroll
      for (int d = 0; d < 3; d++) {
        const T c1 = Gc[0 + d], c2 = Gc[3 + d], c3 = Gc[6 + d], c4 = Gc[9 + d], c5 = Gc[12 + d],
                c6 = Gc[15 + d], c7 = Gc[18 + d];
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
      T f0[Q], dxv[Q];
      eo_contract<T, Q, MatD<Q>, -1>(ux, dxv);
#pragma unroll
      for (int a = 0; a < Q; a++) {
        const T x1 = TB::g(a);
        const T *j1 = P1;
        T j2[3], j3[3];
#pragma unroll
        for (int d = 0; d < 3; d++) {
          j2[d] = P2[d] + x1 * Q2[d];
          j3[d] = P3[d] + x1 * Q3[d];
        }
        const T r0[3] = {j2[1] * j3[2] - j2[2] * j3[1], j2[2] * j3[0] - j2[0] * j3[2], j2[0] * j3[1] - j2[1] * j3[0]};
        const T r1[3] = {j3[1] * j1[2] - j3[2] * j1[1], j3[2] * j1[0] - j3[0] * j1[2], j3[0] * j1[1] - j3[1] * j1[0]};
        const T r2[3] = {j1[1] * j2[2] - j1[2] * j2[1], j1[2] * j2[0] - j1[0] * j2[2], j1[0] * j2[1] - j1[1] * j2[0]};
        const T det = j1[0] * r0[0] + j1[1] * r0[1] + j1[2] * r0[2];
        const T adet = det < T(0) ? -det : det;
        const T wq = wyz * TB::w(a);
        const T kq = COEF ? ka + kb * x1 : T(1);
        const T sc = wq * kq * recip(adet);
        const T dx = dxv[a], dy = u0[KQ(a, pa, pb)], dz = u1[KQ(a, pa, pb)];
        const T gx = r0[0] * dx + r1[0] * dy + r2[0] * dz;
        const T gy = r0[1] * dx + r1[1] * dy + r2[1] * dz;
        const T gz = r0[2] * dx + r1[2] * dy + r2[2] * dz;
        f0[a] = sc * (r0[0] * gx + r0[1] * gy + r0[2] * gz);
        u0[KQ(a, pa, pb)] = sc * (r1[0] * gx + r1[1] * gy + r1[2] * gz);
        u1[KQ(a, pa, pb)] = sc * (r2[0] * gx + r2[1] * gy + r2[2] * gz);
        if constexpr (MASS) ux[a] = wq * adet * kq * ux[a];
      }
      eo_contract<T, Q, MatDt<Q>, -1>(f0, v);
      if constexpr (MASS) {
#pragma unroll
        for (int a = 0; a < Q; a++) v[a] += ux[a];
      }
    }
    __syncthreads();
    // ---- D^T along z of the z-flux in V (pencil x = pa, y = pb) and along y of the
    // y-flux in U (pencil x = pa, z = pb): disjoint buffers, each lane its own pencils
    if (act) {
      T t[Q], q[Q];
#pragma unroll
      for (int c = 0; c < Q; c++) t[c] = u1[KQ(pa, pb, c)];
      eo_contract<T, Q, MatDt<Q>, -1>(t, q);
#pragma unroll
      for (int c = 0; c < Q; c++) u1[KQ(pa, pb, c)] = q[c];
#pragma unroll
      for (int yy = 0; yy < Q; yy++) t[yy] = u0[KQ(pa, yy, pb)];
      eo_contract<T, Q, MatDt<Q>, -1>(t, q);
#pragma unroll
      for (int c = 0; c < Q; c++) u0[KQ(pa, c, pb)] = q[c];
    }
    __syncthreads();
    // ---- x-pencil (y = pa, z = pb): sum the three terms, B^T to x nodes
    if (act) {
#pragma unroll
      for (int a = 0; a < Q; a++) v[a] += u0[KQ(a, pa, pb)] + u1[KQ(a, pa, pb)];
      eo_rect<T, Q, N, MatBRt<N>, 1>(v, r);
#pragma unroll
      for (int i = 0; i < N; i++) u0[KQ(i, pa, pb)] = r[i];
    }
    __syncthreads();
  }
  // ---- y: pencil (x node pa, *, z point pb), B^T to y nodes
  if (act && pa < N) {
#pragma unroll
    for (int c = 0; c < Q; c++) v[c] = u0[KQ(pa, c, pb)];
    eo_rect<T, Q, N, MatBRt<N>, 1>(v, r);
#pragma unroll
    for (int j = 0; j < N; j++) u0[KQ(pa, j, pb)] = r[j];
  }
  __syncthreads();
  // ---- z: nodal pencil (pa, pb, *), B^T to z nodes, scatter
  if (nodal) {
#pragma unroll
    for (int c = 0; c < Q; c++) v[c] = u0[KQ(pa, pb, c)];
    eo_rect<T, Q, N, MatBRt<N>, 1>(v, r);
#pragma unroll
    for (int l = 0; l < N; l++) {
      if (idx[l] >= 0) {
        T *yp = A.y + (int64_t)idx[l] * nc + comp;
        if constexpr (ATOMIC) atomic_add_f(yp, r[l]);
        else *yp += r[l];  // cells of one launch share no node
      }
    }
  }
}
#undef KQ

template <typename T, int N, int Q, int KIND>
static int launch_hexkq_kind(const HexQArgs<T> &a, bool atomic, hipStream_t s) {
  constexpr int EPB = hexkq_epb<Q>();
  const int64_t nb = (a.c1 - a.c0 + EPB - 1) / EPB;
  const dim3 g((unsigned)xcd_grid(nb * a.ncomp)), bl(64 * hexkq_wpb<Q>());
  if (atomic) hex_kq_kernel<T, N, Q, KIND, true><<<g, bl, 0, s>>>(a);
  else hex_kq_kernel<T, N, Q, KIND, false><<<g, bl, 0, s>>>(a);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

template <typename T, int N>
static int launch_hexkq_n(int kind, const HexQArgs<T> &a, bool atomic, hipStream_t s) {
  switch (kind) {
    case MF_OP_MASS: return launch_hexkq_kind<T, N, N + 1, MF_OP_MASS>(a, atomic, s);
    case MF_OP_HELMHOLTZ: return launch_hexkq_kind<T, N, N + 1, MF_OP_HELMHOLTZ>(a, atomic, s);
    case MF_OP_LAPLACIAN: return launch_hexkq_kind<T, N, N + 1, MF_OP_LAPLACIAN>(a, atomic, s);
    case MF_OP_POISSON: return launch_hexkq_kind<T, N, N + 1, MF_OP_POISSON>(a, atomic, s);
  }
  return fail(MF_EUNSUPPORTED, "hex (k+2 points): operator kind");
}

template <typename T>
int launch_hex_kq(int k, int nq, int kind, const HexQArgs<T> &a, bool atomic, hipStream_t s) {
  if (a.c1 <= a.c0) return MF_OK;
  if (nq != k + 2 || nq > 8) return fail(MF_EUNSUPPORTED, "hex scalar operators: nq1d must be k+1 or k+2");
  switch (k) {
    case 1: return launch_hexkq_n<T, 2>(kind, a, atomic, s);
    case 2: return launch_hexkq_n<T, 3>(kind, a, atomic, s);
    case 3: return launch_hexkq_n<T, 4>(kind, a, atomic, s);
    case 4: return launch_hexkq_n<T, 5>(kind, a, atomic, s);
    case 5: return launch_hexkq_n<T, 6>(kind, a, atomic, s);
    case 6: return launch_hexkq_n<T, 7>(kind, a, atomic, s);
  }
  return fail(MF_EUNSUPPORTED, "hex scalar operators with k+2 points: degree 1..6");
}

template int launch_hex_kq<double>(int, int, int, const HexQArgs<double> &, bool, hipStream_t);
template int launch_hex_kq<float>(int, int, int, const HexQArgs<float> &, bool, hipStream_t);

}  // namespace mf
