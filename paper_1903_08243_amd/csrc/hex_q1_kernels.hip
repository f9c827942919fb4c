// Q1 (trilinear hex, n = 2) actions with one cell per lane, the layout of the
// paper's cross-element vectorisation (Section 3.2: elements across SIMD lanes), for
// the operators of the other hex kernels (Section 2.1 local kernel, Section 2.2
// gather / increment): the coloured form over block-interleaved cell arrays and the
// patch form that accumulates compact cell patches in LDS.
#include "hex_common.h"

namespace mf {

// ---------------------------------------------------------------------------------- Q1
// The Q1 (n = 2) cell action on one lane: geometry G (c1..c7, three components
// each), the coefficient's monomial coefficients K (used when the kind has one), the
// 8 nodal values xv (index i + 2 j + 4 l, x fastest) -> the 8 local results yv.
// Per point the gradient is the collocation derivative of the point values, and the
// test side is accumulated straight into the 8 point values before the transposed
// interpolation.
template <typename T, int KIND>
__device__ __forceinline__ void q1_cell(const T (&G)[21], const T (&K)[8], const T (&xv)[8], T (&yv)[8]) {
  constexpr int N = 2;
  using TB = TabT<T, N>;
  constexpr bool GRAD = KIND != K_MASS;
  constexpr bool MASS = KIND == K_MASS || KIND == K_HELM;
  constexpr bool COEF = KIND == K_MASS || KIND == K_POIS;
  // values at the points: u = (B x B x B) x
  T u[8], t[8];
#pragma unroll
  for (int l = 0; l < 4; l++) {  // along x
    const T e0 = xv[2 * l], e1 = xv[2 * l + 1];
    t[2 * l] = TB::B(0, 0) * e0 + TB::B(0, 1) * e1;
    t[2 * l + 1] = TB::B(1, 0) * e0 + TB::B(1, 1) * e1;
  }
#pragma unroll
  for (int l = 0; l < 2; l++)  // along y
#pragma unroll
    for (int a = 0; a < 2; a++) {
      const T e0 = t[a + 4 * l], e1 = t[a + 2 + 4 * l];
      u[a + 4 * l] = TB::B(0, 0) * e0 + TB::B(0, 1) * e1;
      u[a + 2 + 4 * l] = TB::B(1, 0) * e0 + TB::B(1, 1) * e1;
    }
#pragma unroll
  for (int p = 0; p < 4; p++) {  // along z
    const T e0 = u[p], e1 = u[p + 4];
    t[p] = TB::B(0, 0) * e0 + TB::B(0, 1) * e1;
    t[p + 4] = TB::B(1, 0) * e0 + TB::B(1, 1) * e1;
  }
#pragma unroll
  for (int q = 0; q < 8; q++) u[q] = t[q];

  // pointwise; the mass term and the transposed derivatives of the fluxes are
  // accumulated in t at the points
#pragma unroll
  for (int q = 0; q < 8; q++) t[q] = T(0);
#pragma unroll
  for (int q = 0; q < 8; q++) {
    const int a = q & 1, b = (q >> 1) & 1, cc = q >> 2;
    const T x1 = TB::g(a), x2 = TB::g(b), x3 = TB::g(cc);
    T j1[3], j2[3], j3[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
      const T c1 = G[0 + d], c2 = G[3 + d], c3 = G[6 + d], c4 = G[9 + d], c5 = G[12 + d], c6 = G[15 + d],
              c7 = G[18 + d];
      j1[d] = c1 + c4 * x2 + (c5 + c7 * x2) * x3;
      j2[d] = c2 + c4 * x1 + (c6 + c7 * x1) * x3;
      j3[d] = c3 + c5 * x1 + (c6 + c7 * x1) * x2;
    }
    const T r0[3] = {j2[1] * j3[2] - j2[2] * j3[1], j2[2] * j3[0] - j2[0] * j3[2], j2[0] * j3[1] - j2[1] * j3[0]};
    const T det = j1[0] * r0[0] + j1[1] * r0[1] + j1[2] * r0[2];
    const T adet = det < T(0) ? -det : det;
    const T wq = TB::w(a) * TB::w(b) * TB::w(cc);
    T kq = T(1);
    if constexpr (COEF)
      kq = K[0] + K[1] * x1 + K[2] * x2 + K[4] * x1 * x2 + (K[3] + K[5] * x1 + K[6] * x2 + K[7] * x1 * x2) * x3;
    if constexpr (MASS) t[q] += wq * adet * kq * u[q];
    if constexpr (GRAD) {
      const T r1[3] = {j3[1] * j1[2] - j3[2] * j1[1], j3[2] * j1[0] - j3[0] * j1[2], j3[0] * j1[1] - j3[1] * j1[0]};
      const T r2[3] = {j1[1] * j2[2] - j1[2] * j2[1], j1[2] * j2[0] - j1[0] * j2[2], j1[0] * j2[1] - j1[1] * j2[0]};
      const T sc = wq * kq * recip(adet);
      // reference gradient by collocation on the two points of each direction
      const int qx = q ^ 1, qy = q ^ 2, qz = q ^ 4;
      const T dx = TB::D(a, a) * u[q] + TB::D(a, 1 - a) * u[qx];
      const T dy = TB::D(b, b) * u[q] + TB::D(b, 1 - b) * u[qy];
      const T dz = TB::D(cc, cc) * u[q] + TB::D(cc, 1 - cc) * u[qz];
      const T gx = r0[0] * dx + r1[0] * dy + r2[0] * dz;
      const T gy = r0[1] * dx + r1[1] * dy + r2[1] * dz;
      const T gz = r0[2] * dx + r1[2] * dy + r2[2] * dz;
      const T f0 = sc * (r0[0] * gx + r0[1] * gy + r0[2] * gz);
      const T f1 = sc * (r1[0] * gx + r1[1] * gy + r1[2] * gz);
      const T f2 = sc * (r2[0] * gx + r2[1] * gy + r2[2] * gz);
      // transposed collocation derivatives: point q's flux reaches q and its neighbour
      t[q] += TB::D(a, a) * f0 + TB::D(b, b) * f1 + TB::D(cc, cc) * f2;
      t[qx] += TB::D(a, 1 - a) * f0;
      t[qy] += TB::D(b, 1 - b) * f1;
      t[qz] += TB::D(cc, 1 - cc) * f2;
    }
  }

  // transposed interpolation back to the nodes: (B^T x B^T x B^T) t
#pragma unroll
  for (int p = 0; p < 4; p++) {  // along z
    const T e0 = t[p], e1 = t[p + 4];
    u[p] = TB::B(0, 0) * e0 + TB::B(1, 0) * e1;
    u[p + 4] = TB::B(0, 1) * e0 + TB::B(1, 1) * e1;
  }
#pragma unroll
  for (int l = 0; l < 2; l++)  // along y
#pragma unroll
    for (int a = 0; a < 2; a++) {
      const T e0 = u[a + 4 * l], e1 = u[a + 2 + 4 * l];
      t[a + 4 * l] = TB::B(0, 0) * e0 + TB::B(1, 0) * e1;
      t[a + 2 + 4 * l] = TB::B(0, 1) * e0 + TB::B(1, 1) * e1;
    }
#pragma unroll
  for (int l = 0; l < 4; l++) {  // along x
    const T e0 = t[2 * l], e1 = t[2 * l + 1];
    yv[2 * l] = TB::B(0, 0) * e0 + TB::B(1, 0) * e1;
    yv[2 * l + 1] = TB::B(0, 1) * e0 + TB::B(1, 1) * e1;
  }
}

// Q1 with one cell per lane, for the coloured scatter. A Q1 cell has 8 nodes, so the
// pencil kernel's LDS stages and barriers cost more than its arithmetic. Here a
// wavefront owns an aligned block of 64 cells and every stage keeps its 8 values in
// registers. The map, geometry and coefficient of degree-1 operators are stored a
// second time in blocks of 64 cells, entry-major inside a block
// ([cell / 64][entry][cell % 64]), so each per-entry load of a wavefront reads one
// contiguous segment. The cells of one launch share no node, so the result is added
// to y with plain loads and stores. (With atomics, the 64 lanes of an atomic
// instruction would hit 64 different cells' cache lines; the atomic scatter uses the
// pencil kernel, whose lanes of one cell hit neighbouring nodes.)
template <typename T, int KIND>
__global__ void __launch_bounds__(64) hex_q1_kernel(const HexArgs<T> A) {
  constexpr bool COEF = KIND == K_MASS || KIND == K_POIS;
  const int64_t b0 = A.c0 >> 6, nblk = ((A.c1 + 63) >> 6) - b0;
  const int64_t vb = xcd_batch(blockIdx.x, nblk * A.ncomp);
  if (vb >= nblk * A.ncomp) return;
  const int64_t blk = b0 + (int)vb / A.ncomp;  // the grid has fewer than 2^31 items
  const int comp = (int)vb % A.ncomp;
  const int lane = threadIdx.x;
  const int64_t c = blk * 64 + lane;  // the arrays are padded to whole blocks
  bool ok = c >= A.c0 && c < A.c1;
  if (ok && A.cell_user) {
    const int64_t u = A.cell_user[c];
    ok = u >= A.ulo && u < A.uhi;
  }
  const int nc = A.ncomp;
  int idx[8];
  T xv[8], yv[8], G[21], K[8];
#pragma unroll
  for (int i = 0; i < 8; i++) {
    const int32_t m = A.map[(blk * 8 + i) * 64 + lane];
    idx[i] = ok ? m : -1;
  }
#pragma unroll
  for (int i = 0; i < 8; i++) xv[i] = idx[i] >= 0 ? A.x[(int64_t)idx[i] * nc + comp] : T(0);
#pragma unroll
  for (int j = 0; j < 21; j++) G[j] = A.geo[(blk * 24 + j) * 64 + lane];
#pragma unroll
  for (int j = 0; j < 8; j++) K[j] = (COEF && A.coef) ? A.coef[(blk * 8 + j) * 64 + lane] : T(j == 0 ? 1 : 0);
  q1_cell<T, KIND>(G, K, xv, yv);
#pragma unroll
  for (int i = 0; i < 8; i++)
    if (idx[i] >= 0) {
      T *dst = &A.y[(int64_t)idx[i] * nc + comp];
      *dst += yv[i];
    }
}

// Q1 over patches, for full applies: a workgroup takes one patch of up to
// kPatchCells cells that are close in space (cells in Morton order of their
// centroids), gathers the patch's nodes from x and their vertex coordinates into LDS
// once, lets each lane compute whole cells from LDS and add their results into a
// per-patch LDS accumulator, and finally writes every patch node once: nodes no other
// patch touches with a plain read-modify-write, the others (the patch surface) with
// one device atomic each. Against the coloured launches (every colour reads and
// writes every node) this moves x and y about once per apply, and against the atomic
// scatter it issues about one device atomic per cell instead of eight. In FP64 the
// cell geometry (the trilinear map's coefficients) is rebuilt from the 8 corner
// coordinates gathered into LDS: 24 bytes per vertex, shared by its cells, instead of
// 192 stored bytes per cell. In FP32 the 24 stored per-slot values (precomputed in
// FP64, rounded once) are read instead: rebuilding them in FP32 would lose accuracy to
// cancellation, and in FP64 it measured slower than the 96 stored bytes.
template <typename T> constexpr bool q1_patch_coords() { return sizeof(T) == 8; }

template <typename T, int KIND>
__device__ __forceinline__ void q1_patch_slot_load(const HexPatchArgs<T> &P, int p, int s, uint16_t (&li)[8],
                                                   T (&K)[8], T (&G)[21]) {
  constexpr bool COEF = KIND == K_MASS || KIND == K_POIS;
  // slot s of patch p: entry e at ((p * cap / 64 + s / 64) * E + e) * 64 + s % 64. A
  // slot number past the capacity reads slot 0 (a branch here costs registers) and is
  // marked empty.
  const bool have = s < P.cap;
  const int ss = have ? s : 0;
  const int64_t blk = (int64_t)p * (P.cap / 64) + ss / 64;
  const int lane = ss % 64;
#pragma unroll
  for (int i = 0; i < 8; i++) li[i] = have ? P.lmap[(blk * 8 + i) * 64 + lane] : kPatchEmpty;
#pragma unroll
  for (int j = 0; j < 8; j++) K[j] = (COEF && P.coef) ? P.coef[(blk * 8 + j) * 64 + lane] : T(j == 0 ? 1 : 0);
  if constexpr (!q1_patch_coords<T>()) {
#pragma unroll
    for (int j = 0; j < 21; j++) G[j] = P.geo[(blk * 24 + j) * 64 + lane];
  }
}

template <typename T, int KIND>
__device__ __forceinline__ void q1_patch_slot(const uint16_t (&li)[8], const T (&K)[8], T (&G)[21], const T *sx,
                                              const double *sxyz, double *sy) {
  if (li[0] == kPatchEmpty) return;  // a slot past the patch's cells (a real cell has all 8)
  T xv[8], yv[8];
#pragma unroll
  for (int i = 0; i < 8; i++) xv[i] = sx[li[i]];
  if constexpr (q1_patch_coords<T>()) {
#pragma unroll
    for (int d = 0; d < 3; d++) {
      double X[8];
#pragma unroll
      for (int v = 0; v < 8; v++) X[v] = sxyz[3 * li[v] + d];
      // monomial coefficients c1..c7 of the trilinear map (vertex v at (v&1, v>>1&1, v>>2&1))
      G[0 + d] = T(X[1] - X[0]);
      G[3 + d] = T(X[2] - X[0]);
      G[6 + d] = T(X[4] - X[0]);
      G[9 + d] = T(X[3] - X[1] - X[2] + X[0]);
      G[12 + d] = T(X[5] - X[1] - X[4] + X[0]);
      G[15 + d] = T(X[6] - X[2] - X[4] + X[0]);
      G[18 + d] = T(X[7] - X[3] - X[5] - X[6] + X[1] + X[2] + X[4] - X[0]);
    }
  }
  q1_cell<T, KIND>(G, K, xv, yv);
#pragma unroll
  for (int i = 0; i < 8; i++) atomic_add_f(&sy[li[i]], (double)yv[i]);
}

// Three wavefronts per SIMD where the registers allow it without spilling much (the
// coefficient kinds need more and keep two).
template <int KIND> constexpr int q1_patch_waves() { return KIND == K_POIS ? 2 : 3; }

template <typename T, int KIND>
__global__ void __launch_bounds__(kPatchThreads, q1_patch_waves<KIND>()) hex_q1_patch_kernel(const HexPatchArgs<T> P) {
  static_assert(kPatchCells == 2 * kPatchThreads, "two cell slots per thread");
  constexpr bool XYZ = q1_patch_coords<T>();
  extern __shared__ __align__(16) unsigned char patch_lds[];
  // node sums in FP64 for both precisions (LDS FP32 atomic adds measured several
  // times slower than FP64 ones)
  double *sxyz = (double *)patch_lds;
  double *sy = sxyz + (XYZ ? 3 * P.max_nodes : 0);
  T *sx = (T *)(sy + P.max_nodes);
  const int64_t item = xcd_batch(blockIdx.x, P.npatch * P.ncomp);
  if (item >= P.npatch * P.ncomp) return;
  const int p = (int)item / P.ncomp, comp = (int)item % P.ncomp, nc = P.ncomp;
  const int t = threadIdx.x;
  // the first slot's map is requested before the gathers, so its latency overlaps them
  uint16_t li[8];
  T K[8], G[21];
  q1_patch_slot_load<T, KIND>(P, p, t, li, K, G);
  const int n0 = P.node_ptr[p], nn = P.node_ptr[p + 1] - n0;
  for (int i = t; i < nn; i += kPatchThreads) {
    const int32_t e = P.nodes[n0 + i];
    const int64_t id = e & kPatchIdMask;
    const int64_t g = P.gnodes ? P.gnodes[n0 + i] : id;
    const T xv = P.x[g * nc + comp];  // a constrained node's value is read, then replaced by 0
    sx[i] = (e & kPatchFixed) ? T(0) : xv;
    sy[i] = 0.0;
    if constexpr (XYZ) {
      sxyz[3 * i] = P.xyz[3 * id];
      sxyz[3 * i + 1] = P.xyz[3 * id + 1];
      sxyz[3 * i + 2] = P.xyz[3 * id + 2];
    }
  }
  __syncthreads();
  q1_patch_slot<T, KIND>(li, K, G, sx, sxyz, sy);
  q1_patch_slot_load<T, KIND>(P, p, t + kPatchThreads, li, K, G);
  q1_patch_slot<T, KIND>(li, K, G, sx, sxyz, sy);
  __syncthreads();
  for (int i = t; i < nn; i += kPatchThreads) {
    const int32_t e = P.nodes[n0 + i];
    if (e & kPatchFixed) continue;
    T *dst = &P.y[(int64_t)(e & kPatchIdMask) * nc + comp];
    if (e & kPatchShared) atomic_add_f(dst, (T)sy[i]);
    else *dst += (T)sy[i];
  }
}

template <typename T>
int launch_hex_patches(int N, int kind, const HexPatchArgs<T> &a, hipStream_t s) {
  if (a.npatch <= 0) return MF_OK;
  if (N != 2) return fail(MF_EUNSUPPORTED, "hex patch kernel: degree");
  const dim3 grid((unsigned)xcd_grid((int64_t)a.npatch * a.ncomp)), block(kPatchThreads);
  const size_t lds = (size_t)a.max_nodes * ((q1_patch_coords<T>() ? 3 * sizeof(double) : 0) + sizeof(double) + sizeof(T));
  switch (kind) {
    case K_MASS: hex_q1_patch_kernel<T, K_MASS><<<grid, block, lds, s>>>(a); break;
    case K_HELM: hex_q1_patch_kernel<T, K_HELM><<<grid, block, lds, s>>>(a); break;
    case K_LAP: hex_q1_patch_kernel<T, K_LAP><<<grid, block, lds, s>>>(a); break;
    case K_POIS: hex_q1_patch_kernel<T, K_POIS><<<grid, block, lds, s>>>(a); break;
    default: return fail(MF_EUNSUPPORTED, "hex patch kernel: operator kind");
  }
  MF_HIP(hipGetLastError());
  return MF_OK;
}
template int launch_hex_patches<double>(int, int, const HexPatchArgs<double> &, hipStream_t);
template int launch_hex_patches<float>(int, int, const HexPatchArgs<float> &, hipStream_t);

template <typename T>
int launch_hex_q1_coloured(int kind, const HexArgs<T> &a, hipStream_t s) {
  if (a.c1 <= a.c0) return MF_OK;
  const int64_t nblk = ((a.c1 + 63) >> 6) - (a.c0 >> 6);
  const dim3 grid((unsigned)xcd_grid(nblk * a.ncomp)), block(64);
  switch (kind) {
    case K_MASS: hex_q1_kernel<T, K_MASS><<<grid, block, 0, s>>>(a); break;
    case K_HELM: hex_q1_kernel<T, K_HELM><<<grid, block, 0, s>>>(a); break;
    case K_LAP: hex_q1_kernel<T, K_LAP><<<grid, block, 0, s>>>(a); break;
    case K_POIS: hex_q1_kernel<T, K_POIS><<<grid, block, 0, s>>>(a); break;
    default: return fail(MF_EUNSUPPORTED, "hex kernel: operator kind");
  }
  MF_HIP(hipGetLastError());
  return MF_OK;
}

template int launch_hex_q1_coloured<double>(int, const HexArgs<double> &, hipStream_t);
template int launch_hex_q1_coloured<float>(int, const HexArgs<float> &, hipStream_t);

}  // namespace mf
