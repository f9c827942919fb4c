// Internal declarations shared by the host setup code and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mf.h"

namespace mf {

// ------------------------------------------------------------------ errors
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);
#define MF_HIP(call)                                                            \
  do {                                                                          \
    hipError_t e_ = (call);                                                     \
    if (e_ != hipSuccess)                                                       \
      return ::mf::fail(MF_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ------------------------------------------------------------------ tables (host, FP64)
}  // namespace mf
#include "tables.h"
namespace mf {

// ------------------------------------------------------------------ objects
struct DeviceBuffer {
  void *ptr = nullptr;
  size_t bytes = 0;
  ~DeviceBuffer() { if (ptr) (void)hipFree(ptr); }
  int alloc(size_t b);
  template <class T> T *as() const { return static_cast<T *>(ptr); }
};

}  // namespace mf

struct mf_mesh {
  int cell_type = 0, gdim = 0, nvc = 0;
  int64_t nverts = 0, ncells = 0;
  std::vector<double> coords;
  std::vector<int32_t> cell2vert;
};

struct mf_space {
  // the space keeps its own copy of the mesh data, so destroying the mesh first is safe
  int cell_type = 0, gdim = 0, nvc = 0;
  int64_t nverts = 0, ncells = 0;
  std::vector<double> coords;
  std::vector<int32_t> cell2vert;
  int degree = 0, ncomp = 0, D = 0;
  int64_t nnodes = 0;
  std::vector<int32_t> cell2node;      // user numbering, as given
  // Internal node numbering: nodes numbered in order of first appearance when the
  // cells are traversed in order, so the nodes of consecutive cells are close in
  // memory. The kernels use only the internal numbering.
  std::vector<int32_t> user_of_int;    // internal node -> user node
  std::vector<int32_t> int_of_user;    // user node -> internal node
  // Internal cell order: cells sorted by colour (a greedy first-fit colouring in
  // which no two cells of one colour share a vertex, hence no node), original
  // order within a colour. colour_ptr[c] .. colour_ptr[c+1] are colour c's cells.
  std::vector<int32_t> cell_user_of_int;  // internal cell -> user cell
  std::vector<int64_t> colour_ptr;
  std::vector<int32_t> cell2node_int;  // internal cell order, internal node numbering
  std::vector<int32_t> cell2vert_int;  // internal cell order
  uint64_t numbering_id = 0;           // equal ids <=> identical internal numbering
  bool identity = false;               // internal numbering equals the user numbering
};

namespace mf {

// Launch parameters of the hex sum-factorised kernel, per precision.
template <typename T> struct HexArgs {
  // [cell][entry] arrays; the degree-1 apply kernel takes the block-interleaved
  // copies ([cell/64][entry][cell%64], padded to whole blocks) instead
  const int32_t *map;  // ncells x N^3 node ids (negative: constrained, -1-node)
  const T *geo;        // ncells x 24: trilinear coefficient vectors c1..c7 (x3), pad
  const T *coef;       // ncells x 8 monomial coefficients of the vertex coefficient, or null
  const T *x;
  T *y;
  int64_t c0, c1;      // internal cell range
  int ncomp;
  const int32_t *cell_user;  // if set: only cells whose user index is in [ulo, uhi)
  int64_t ulo, uhi;
  // if set (pencil kernel only): x is gathered at these positions instead of at map
  // (same layout as map; negative = constrained), e.g. a half-permuted input
  const int32_t *gmap;
  // if set (pencil kernel, colour-by-colour overwrite applies only): per internal cell
  // the lowest node id that the cell touches first in launch order. Nodes are numbered
  // by first touch, so the cell touches node n first exactly when n >= first[cell]:
  // it then stores its contribution without reading y, which needs no prior clearing.
  const int32_t *first;
  // patch scatter (hex_patch_kernel; the cell arrays above are then in patch-slot
  // order, EPB slots per patch): per slot and node the index in its patch's node list
  // (kSlotSkip: constrained or empty), the node-list offsets and outputs, and the
  // shared-node slots (as SimplexPatchArgs; sbuf is [slot][ncomp])
  const uint16_t *plmap = nullptr;
  const int32_t *pnptr = nullptr;
  const int32_t *pout = nullptr;
  T *psbuf = nullptr;
  int accumulate = 0;
};

// Q1 patch decomposition (full applies of degree-1 hex operators): patches of up to
// cap <= kPatchCells cells (a multiple of 64, the same for all patches of an
// operator) with at most kPatchNodes distinct nodes (the cells' vertices). Per-slot
// arrays are block-interleaved with cap slots per patch: entry e of slot s of patch
// p at ((p * cap / 64 + s / 64) * E + e) * 64 + s % 64; empty slots have local index
// kPatchEmpty. A patch node entry is the internal node id with flags: kPatchShared
// (another patch touches the node: written with a device atomic) and kPatchFixed
// (constrained: gathered as 0, never written; its coordinates are still needed).
// (The same scheme around the pencil stages for higher degrees measured slower than
// the atomic and coloured launches.)
constexpr int kPatchCells = 512, kPatchNodes = 1024, kPatchThreads = 256;
constexpr uint16_t kPatchEmpty = 0xFFFF;
constexpr int32_t kPatchShared = 1 << 30, kPatchFixed = 1 << 29, kPatchIdMask = kPatchFixed - 1;
template <typename T> struct HexPatchArgs {
  const int32_t *node_ptr;  // npatch + 1 offsets into nodes
  const int32_t *nodes;     // internal node ids with the kPatchShared / kPatchFixed flags
  const int32_t *gnodes;    // if set: gather positions of the nodes in x (else their ids)
  const uint16_t *lmap;     // per slot, 8 local node indices (local node v = vertex v)
  const double *xyz;        // FP64 operators: per internal node, 3 vertex coordinates
  const T *geo;             // FP32 operators: per slot, 24 geometry entries (c1..c7 x3, pad)
  const T *coef;            // per slot, 8 coefficient entries, or null
  const T *x;
  T *y;
  int npatch, max_nodes, ncomp, cap;
};
// N = 2 only (the lane-per-cell Q1 kernel).
template <typename T> int launch_hex_patches(int N, int kind, const HexPatchArgs<T> &a, hipStream_t s);
// N = 2, one colour's cells (no two share a node): the lane-per-cell kernel over the
// block-interleaved arrays (hex_q1_kernels.hip)
template <typename T> int launch_hex_q1_coloured(int kind, const HexArgs<T> &a, hipStream_t s);

// Kernel launchers (hex_kernels.hip)
// atomic: scatter with device-scope atomics (any cell set); otherwise plain
// read-modify-write, valid only when no two cells of [c0, c1) share a node.
// For N = 2 the non-atomic launch takes the block-interleaved arrays (q1map, q1geo,
// q1coef) and the atomic one the [cell][entry] arrays.
template <typename T>
int launch_hex_apply(int N, int kind, const HexArgs<T> &a, bool atomic, hipStream_t s);
template <typename T>
int launch_hex_diag(int N, int kind, const HexArgs<T> &a, hipStream_t s);
// Batched persistent launch over a device work list (see hex_kernels.hip for the
// layouts of the op and item records; degrees 1..5). stop (optional) is read at
// stop[op * stop_stride]; items of stopped operators are skipped.
template <typename T>
int launch_hex_batch(int kind, const void *ops, const void *items, int nitems, int grid, const int *stop,
                     int stop_stride, hipStream_t s);
size_t hex_batch_op_bytes(int precision);
size_t hex_batch_item_bytes();
int hex_cells_per_batch(int N);

// Tet elasticity (simplex_kernels.hip)
template <typename T> struct TetArgs {
  const int32_t *map;  // AoSoA: [ncells/64][D][64] node ids (negative: constrained)
  const T *geo;        // AoSoA: [ncells/64][10][64]: Kinv (9, row-major Kinv[b][a]) and w-free |det|
  const T *tab;        // [Q][D][3] reference gradients, then [Q] weights (device)
  const T *x;
  T *y;
  int64_t c0, c1;
  T lam, mu;
  const int32_t *cell_user;  // if set: only cells whose user index is in [ulo, uhi)
  int64_t ulo, uhi;
  // HYPERELASTIC (else null): the linearisation point (internal numbering, like x) and
  // the map it is gathered through (null: map; set when map flags constrained nodes)
  const T *u0;
  const int32_t *u0map;
  // scalar operators (MASS, POISSON): AoSoA [ncells/64][4][64] vertex coefficients, or null
  const T *coef;
};
// ELASTICITY, or HYPERELASTIC when a.u0 is set (k = 1, nq = 1 and k = 2, nq = 14)
template <typename T>
int launch_tet_elasticity(int k, int nq, const TetArgs<T> &a, bool atomic, hipStream_t s);
// one-component MASS, HELMHOLTZ, LAPLACIAN, POISSON on P1..P3 tets; tab holds phi
// [nq][D], the reference gradients [nq][D][3], the weights [nq] and the vertex
// basis [nq][4] at the points, then simplex_mfma_scalar_tables (matrix-core kernels)
template <typename T>
int launch_tet_scalar(int k, int nq, int kind, const TetArgs<T> &a, bool atomic, hipStream_t s);
// per-lane MFMA operands of the one-component simplex kernels (dim 2 or 3, D nodes)
int simplex_mfma_scalar_table_floats(int dim, int D, int nq);
void simplex_mfma_scalar_tables(int dim, int D, int nq, const double *phi, const double *dphi, double *out,
                                bool f64);
// the one-component forms on P1..P6 triangles on the matrix cores (TetArgs as a
// generic simplex argument block: geo [cell/64][5][64], coef [cell/64][3][64], tab phi
// [nq][D], gradients [nq][D][2], weights, vertex basis [nq][3], then
// simplex_mfma_scalar_tables), atomic or coloured
template <typename T>
int launch_tri_scalar_mfma(int k, int nq, int kind, const TetArgs<T> &a, bool atomic, hipStream_t s);
// 2D linear elasticity on P1..P6 triangles on the matrix cores (the same tables;
// two node-interleaved components, TetArgs lam and mu)
template <typename T>
int launch_tri_elasticity_mfma(int k, int nq, const TetArgs<T> &a, bool atomic, hipStream_t s);

template <typename T>
int launch_tet_elasticity_diag(int k, int nq, const TetArgs<T> &a, hipStream_t s);
// Degree >= 2: the action runs on MFMA and needs these per-lane operands of the
// tabulation appended to TetArgs::tab after the weights (host-built)
int tet_mfma_table_floats(int k, int nq);
void tet_mfma_tables(int k, int nq, const double *dphi, double *out, bool f64);

// Q1..Q6 on bilinear quadrilaterals (quad_kernels.hip): one-component MASS, HELMHOLTZ,
// LAPLACIAN, POISSON and two-component ELASTICITY, sum-factorised, nq = k+1 or k+2
// Gauss points per direction
template <typename T> struct QuadArgs {
  const int32_t *map;  // [ncells][(k+1)^2] node ids, dof i + (k+1) j (negative: constrained)
  const T *geo;        // [ncells][6]: bilinear map coefficients c1, c2, c3 as (x, y) pairs
  const T *coef;       // [ncells][4] vertex coefficients (MASS c, POISSON kappa), or null
  const T *tab;        // B [nq][k+1], B' [nq][k+1], weights [nq], points [nq]
  const T *x;          // ELASTICITY: two components per node, interleaved
  T *y;
  int64_t c0, c1;
  const int32_t *cell_user;  // if set: only cells whose user index is in [ulo, uhi)
  int64_t ulo, uhi;
  T lam, mu;  // ELASTICITY Lame parameters
};
// diag: accumulate diag(A) into a.y (a.x unused; always atomic)
template <typename T>
int launch_quad(int k, int nq, int kind, const QuadArgs<T> &a, bool atomic, hipStream_t s, bool diag = false);

// Scalar hex operators with k+2 Gauss points per direction on pencils
// (hex_kq_kernels.hip): rectangular interpolation to the k+2 points, the k+1 kernel's
// point stages, rectangular integration back. map and geo as HexElasArgs; coef: 8
// trilinear coefficients of the vertex coefficient per cell (or null); ncomp 1 or 3
// (node-interleaved). The 1D tables are compile-time constants.
template <typename T> struct HexQArgs {
  const int32_t *map;
  const T *geo;
  const T *coef;
  const T *x;
  T *y;
  int64_t c0, c1;
  const int32_t *cell_user;
  int64_t ulo, uhi;
  const int32_t *gmap;
  int ncomp;
};
template <typename T>
int launch_hex_kq(int k, int nq, int kind, const HexQArgs<T> &a, bool atomic, hipStream_t s);

// ELASTICITY on Q1..Q6 hexahedra (hex_elas_kernels.hip): three node-interleaved
// components, sum-factorised, nq = k+1 or k+2 Gauss points per direction (at most 7)
template <typename T> struct HexElasArgs {
  const int32_t *map;  // [ncells][(k+1)^3] node ids, internal numbering (negative: constrained)
  const T *geo;        // [ncells][24] trilinear coefficients c1..c7 per coordinate
  const T *tab;        // B [nq][k+1], B' [nq][k+1], weights [nq], points [nq]
  const T *x;
  T *y;
  int64_t c0, c1;
  const int32_t *cell_user;  // if set: only cells whose user index is in [ulo, uhi)
  int64_t ulo, uhi;
  T lam, mu;
  const int32_t *gmap;  // if set: x is gathered through it (fused permutation), y through map
  const T *u0 = nullptr;            // HYPERELASTIC: linearisation point, internal numbering
  const int32_t *u0map = nullptr;   // its map when `map` flags constrained nodes
};
template <typename T>
int launch_hex_elasticity(int k, int nq, const HexElasArgs<T> &a, bool atomic, hipStream_t s);

// Tri P1 mass with vertex coefficient (simplex_kernels.hip)
template <typename T> struct TriArgs {
  const int32_t *map;  // ncells x 3 (negative: constrained)
  const T *geo;        // ncells x 4: |T| c0, |T| c1, |T| c2, pad
  const T *x;
  T *y;
  int64_t c0, c1;
  const int32_t *cell_user;  // if set: only cells whose user index is in [ulo, uhi)
  int64_t ulo, uhi;
};
template <typename T> int launch_tri_mass(const TriArgs<T> &a, bool atomic, hipStream_t s);
template <typename T> int launch_tri_mass_diag(const TriArgs<T> &a, hipStream_t s);

// Vector kernels (vec_kernels.hip)
template <typename T> int launch_fill(T *y, T v, int64_t n, hipStream_t s);
template <typename T>
int launch_copy_constrained(const int32_t *dofs, int64_t n, const T *x, T *y, hipStream_t s);
template <typename T>
int launch_set_constrained(const int32_t *dofs, int64_t n, T v, T *y, hipStream_t s);
// x_int[i*nc + c] = x_user[uoi[i]*nc + c]
template <typename T>
int launch_to_internal(const int32_t *uoi, int64_t nnodes, int nc, const T *xu, T *xi, hipStream_t s);
// y_user[uoi[i]*nc + c] (+)= y_int[i*nc + c]
template <typename T>
int launch_from_internal(const int32_t *uoi, int64_t nnodes, int nc, const T *yi, T *yu, bool acc, hipStream_t s);
// out[i] = in[src[i]] (i < n nodes of nc values) in two stages through tmp, with the
// positions from permute2_positions(src): pos1[j] is the slot of source node j in the
// bucket of its destination, pos2[i] the slot holding destination i, which lies in
// bucket i / kPermBucket. One bucket of nc values must fit in LDS.
constexpr int kPermBucket = 2048;
template <typename T>
int launch_permute2(const int32_t *pos1, const int32_t *pos2, int64_t n, int nc, const T *in, T *tmp, T *out,
                    bool acc, hipStream_t s);
void permute2_positions(const int32_t *src, int64_t n, std::vector<int32_t> &pos1, std::vector<int32_t> &pos2);
// the first stage alone: tmp[pos1[j]] = in[j]
template <typename T>
int launch_permute_stage1(const int32_t *pos1, int64_t n, int nc, const T *in, T *tmp, hipStream_t s);
// the same with the inverse permutation iou (user node -> internal node), as a gather
template <typename T>
int launch_from_internal_gather(const int32_t *iou, int64_t nnodes, int nc, const T *yi, T *yu, bool acc,
                                hipStream_t s);

}  // namespace mf

namespace mf {
// Workgroups are dispatched round-robin over the 8 XCDs of an MI355X, each with its
// own L2. Mapping workgroup w to batch (w % 8) * ceil(nb / 8) + w / 8 gives every
// XCD one contiguous range of cell batches, so the nodes neighbouring cells share
// (and the cache lines around them) are fetched into one L2 instead of several.
// The grid must hold 8 * ceil(nb / 8) workgroups; results >= nb are idle.
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_batch(int64_t w, int64_t nb) {
  const int64_t per = (nb + kXcds - 1) / kXcds;
  return (w % kXcds) * per + w / kXcds;
}
inline int64_t xcd_grid(int64_t nb) { return ((nb + kXcds - 1) / kXcds) * kXcds; }

// Patch scatter of the simplex kernels (full applies). Cells are grouped into patches
// of at most cap slots (a multiple of 64) in a locality (Morton) order, each touching
// at most nmax distinct free nodes. A workgroup takes one patch: it sums the cells'
// local results into the patch's nodes in LDS, then writes each node once: a node of
// this patch alone straight into y, a node shared with other patches into its slot of
// sbuf; simplex_shared_reduce then sums each shared node's slots (in a fixed order)
// into y. Every free node is written once per apply, so overwrite applies need no
// clearing pass. Per-slot arrays are AoSoA blocks of 64 slots
// ([patch * cap / 64 + slot / 64][entry][slot % 64]); empty slots have map -1, local
// index kSlotSkip and zero geometry.
constexpr uint16_t kSlotSkip = 0xFFFF;      // constrained node or empty slot: no write
constexpr int32_t kSharedOut = 1 << 30;     // out entry: slot in sbuf rather than a node id
template <typename T> struct SimplexPatchArgs {
  const int32_t *map;    // [blocks][D][64] internal node ids (negative: constrained or empty)
  const T *geo;          // [blocks][G][64] the slot's cell geometry
  const uint16_t *lmap;  // [blocks][D][64] index of the node in the patch's node list
  const int32_t *nptr;   // [npatch + 1] node list offsets
  const int32_t *out;    // per patch node: internal node id, or kSharedOut | sbuf slot
  T *sbuf;               // [contributions][ncomp]
  int npatch, cap, nmax, accumulate;
};
template <typename T>
int launch_tet_elasticity_patches(int k, int nq, const TetArgs<T> &a, const SimplexPatchArgs<T> &p,
                                  hipStream_t s);
// the one-component triangle forms with the patch scatter (slot geometry: d xi / d x,
// |det| and, for MASS and POISSON, the three vertex coefficients: 5 or 8 entries)
template <typename T>
int launch_tri_scalar_patches(int k, int nq, int kind, const TetArgs<T> &a, const SimplexPatchArgs<T> &p,
                              hipStream_t s);
// 2D elasticity on triangles with the patch scatter (slot geometry as above, 5 entries;
// two components per node)
template <typename T>
int launch_tri_elasticity_patches(int k, int nq, const TetArgs<T> &a, const SimplexPatchArgs<T> &p, hipStream_t s);
// the one-component tet forms with the patch scatter (slot geometry: Kinv,
// |det| and, for MASS and POISSON, the four vertex coefficients: 10 or 14 entries)
template <typename T>
int launch_tet_scalar_patches(int k, int nq, int kind, const TetArgs<T> &a, const SimplexPatchArgs<T> &p,
                              hipStream_t s);
// hex pencil kernel with the patch scatter (degrees 2-6): a.map / gmap / geo / coef in
// patch-slot order (hex_cells_per_patch(N) slots per patch) and the patch fields set
template <typename T> int launch_hex_cell_patches(int N, int kind, const HexArgs<T> &a, int npatch, hipStream_t s);
int hex_cells_per_patch(int N);
// the closed-form P1 triangle mass (geometry: the three s_a = |T| c_a per slot)
template <typename T> int launch_tri_mass_patches(const T *x, T *y, const SimplexPatchArgs<T> &p, hipStream_t s);
// y[snode[i]] (+)= sum of sbuf slots sptr[i] .. sptr[i+1]-1, per component
template <typename T>
int launch_simplex_shared_reduce(const int32_t *sptr, const int32_t *snode, const T *sbuf, T *y, int64_t nshared,
                                 int ncomp, bool accumulate, hipStream_t s);

// Element matrices of tet operators (FP64 tables phi [nq][D], reference gradients
// [nq][D][3], weights [nq], vertex basis [nq][4]) added into CSR values (user numbering
// through unode [cell][D]); the closed-form P1 triangle mass likewise.
template <typename T>
int launch_simplex_element_csr(int dim, const int32_t *fmap, const int32_t *unode, const T *geo, const T *coef,
                               const double *tab, int64_t ncells, int D, int nq, int kind, int ncomp, double lam,
                               double mu, const int64_t *rowptr, const int32_t *col, T *vals, hipStream_t s);
template <typename T>
int launch_tensor_element_csr(int dim, const int32_t *map, const int32_t *unode, const T *geo, const T *coef,
                              const double *tab, int64_t ncells, int n, int nq, int kind, int ncomp, double lam,
                              double mu, const int64_t *rowptr, const int32_t *col, T *vals, hipStream_t s);
template <typename T>
int launch_tri_mass_element_csr(const int32_t *fmap, const int32_t *unode, const T *geo, int64_t ncells,
                                const int64_t *rowptr, const int32_t *col, T *vals, hipStream_t s);
template <typename T>
int launch_simplex_element_diag(int dim, const int32_t *fmap, const T *geo, const T *coef, const double *tab,
                                int64_t ncells, int D, int nq, int kind, int nc, double lam, double mu, T *d,
                                hipStream_t s);
template <typename T>
int launch_hex_element_diag(const int32_t *map, const T *geo, const T *coef, const double *tab, int64_t ncells,
                            int n, int nq, int kind, int nc, double lam, double mu, T *d, hipStream_t s);
bool element_diag_supported(const mf_op *op);
template <typename T> int element_diag(const mf_op *op, T *d, hipStream_t s);
template <typename T> int launch_set_at(const int64_t *pos, int64_t n, T v, T *vals, hipStream_t s);

// Internal-numbering entry points used by the solvers.
int op_apply_internal(const mf_op *op, const void *x, void *y, hipStream_t s);
// y += A x (internal numbering, y not cleared), then the constraint rows y_b = x_b
int op_apply_internal_acc(const mf_op *op, const void *x, void *y, hipStream_t s);
int op_diagonal_internal(const mf_op *op, void *d, hipStream_t s);
}  // namespace mf

struct mf_op {
  int cell_type = 0, kind = 0, precision = 0, degree = 0, ncomp = 0, nq1d = 0, nqp = 0, D = 0;
  int64_t ncells = 0, nnodes = 0, ndofs = 0;
  double lam = 1.0, mu = 0.5;
  bool has_coef = false;
  mf::DeviceBuffer map, geo, coef, tab, bc_dofs;  // map and bc_dofs in internal numbering
  mf::DeviceBuffer q1map, q1geo, q1coef;          // degree-1 hex: map, geometry, coefficient in
                                                  // blocks of 64 cells, [cell/64][entry][cell%64]
  mf::DeviceBuffer pt_nptr, pt_nodes, pt_lmap, pt_xyz, pt_geo, pt_coef;  // degree-1 hex patches
  // hex, user numbering: x is gathered straight from the first stage of the two-stage
  // permutation (positions to2 of the map's nodes), which saves the second stage
  mf::DeviceBuffer gmap, pt_gnodes;
  bool fused_gather = false;
  // first-touch thresholds (HexArgs::first) of a coloured pencil-kernel operator, and
  // whether every node without a constraint is first touched by some cell
  mf::DeviceBuffer first_lo;
  bool first_ok = false;
  int npatch = 0, pt_max_nodes = 0, pt_cap = 0;
  bool patched = false;  // full applies use the patch kernel
  // simplex patch scatter (SimplexPatchArgs): slot-ordered map, geometry and local
  // indices, node outputs, shared-node sums
  mf::DeviceBuffer sp_map, sp_geo, sp_lmap, sp_nptr, sp_out, sp_sbuf, sp_sptr, sp_snode;
  int sp_npatch = 0, sp_cap = 0, sp_nmax = 0;
  int64_t sp_nshared = 0;
  bool spatched = false;
  // hex pencil-kernel patch scatter (degrees 2-6): patch-slot-ordered cell arrays
  // (map, gather map, geometry, coefficient, local node indices) and node outputs; the
  // shared-node slots reuse sp_sbuf, sp_sptr, sp_snode, sp_nshared
  mf::DeviceBuffer hp_map, hp_gmap, hp_geo, hp_coef, hp_lmap, hp_nptr, hp_out;
  int hp_npatch = 0;
  bool hpatched = false;
  // matrix assembly (tets P1-P3 and the P1 triangle mass): per internal cell the user
  // node of each local node, the constrained user dofs, the quadrature degree of the
  // tet rule, and the CSR pattern once built
  std::vector<int32_t> h_bc_user;  // constrained dofs, user numbering
  int qdeg = 0;
  mutable std::vector<int64_t> csr_rowptr;
  mutable std::vector<int32_t> csr_col;
  mutable bool csr_built = false;
  mf::DeviceBuffer perm;                          // internal node -> user node (int32)
  mf::DeviceBuffer iperm;                         // user node -> internal node (int32)
  mf::DeviceBuffer to1, to2, from1, from2, wt;    // two-stage permutations (positions) and their buffer
  mf::DeviceBuffer u0, u0map;                    // HYPERELASTIC linearisation point and its gather map
  mf::DeviceBuffer cell_user;                     // internal cell -> user cell (int32)
  std::vector<int64_t> colour_ptr;                // colour ranges of the internal cell order
  mf::DeviceBuffer wx, wy;                        // user-numbering workspaces (ndofs, op precision)
  uint64_t numbering_id = 0;
  bool identity = false;
  bool coloured = true;  // full applies: one launch per colour with plain stores
  int64_t n_bc_dofs = 0;
  double flops = 0.0, bytes = 0.0;
};
