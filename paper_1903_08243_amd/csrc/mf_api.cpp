// C ABI entry points: mesh / space / operator setup and the operator action.
//
// Setup is host C++ in FP64: validation of the input maps (the paper's
// cell2dof and cell2vert maps, Section 2.2), cell geometry precompute, the
// constant tables of the element kernel, and the device layouts the kernels
// read. The action itself runs entirely in the HIP kernels.
#include <algorithm>
#include <type_traits>
#include <atomic>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>

#include "mf_internal.h"

namespace mf {

static thread_local std::string g_err;
void set_error(const std::string &m) { g_err = m; }
int fail(int code, const std::string &m) {
  g_err = m;
  return code;
}

int DeviceBuffer::alloc(size_t b) {
  if (ptr) (void)hipFree(ptr);
  ptr = nullptr;
  bytes = b;
  if (b == 0) return MF_OK;
  if (hipMalloc(&ptr, b) != hipSuccess) {
    ptr = nullptr;
    (void)hipGetLastError();
    return fail(MF_ENOMEM, "hipMalloc of " + std::to_string(b) + " bytes failed");
  }
  return MF_OK;
}

static int upload(DeviceBuffer &buf, const void *src, size_t bytes, hipStream_t s) {
  int rc = buf.alloc(bytes);
  if (rc) return rc;
  if (bytes) MF_HIP(hipMemcpyAsync(buf.ptr, src, bytes, hipMemcpyHostToDevice, s));
  return MF_OK;
}

template <typename T> static std::vector<T> cast_vec(const std::vector<double> &v) {
  return std::vector<T>(v.begin(), v.end());
}

static int nvc_of(int cell_type) {
  return cell_type == MF_CELL_TRI ? 3 : cell_type == MF_CELL_TET ? 4 : cell_type == MF_CELL_HEX ? 8
         : cell_type == MF_CELL_QUAD ? 4 : 0;
}

// Trilinear map x(xi) = c0 + c1 xi1 + c2 xi2 + c3 xi3 + c4 xi1 xi2 + c5 xi1 xi3 + c6 xi2 xi3
// + c7 xi1 xi2 xi3 from the 8 vertex values (vertex v at (v&1, v>>1&1, v>>2&1)).
static void trilinear_coeffs(const double X[8], double c[8]) {
  c[0] = X[0];
  c[1] = X[1] - X[0];
  c[2] = X[2] - X[0];
  c[3] = X[4] - X[0];
  c[4] = X[3] - X[1] - X[2] + X[0];
  c[5] = X[5] - X[1] - X[4] + X[0];
  c[6] = X[6] - X[2] - X[4] + X[0];
  c[7] = X[7] - X[3] - X[5] - X[6] + X[1] + X[2] + X[4] - X[0];
}

// 3 x 10-bit Morton code (bit i of x, y, z at bits 3i, 3i + 1, 3i + 2)
static uint32_t morton3(uint32_t x, uint32_t y, uint32_t z) {
  auto spread = [](uint32_t v) {
    v &= 1023u;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
  };
  return spread(x) | (spread(y) << 1) | (spread(z) << 2);
}

// Cells 0..nc-1 (vertex lists cv, nvc per cell) sorted by the Morton code of their
// centroids, each coordinate quantised to 1024 steps over the centroids' bounding
// box; ties by cell index.
static std::vector<int64_t> morton_cell_order(const std::vector<double> &coords, int gd, const int32_t *cv, int nvc,
                                              int64_t nc) {
  std::vector<double> cen((size_t)nc * 3, 0.0);
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t K = 0; K < nc; K++)
    for (int a = 0; a < gd; a++) {
      double c = 0.0;
      for (int v = 0; v < nvc; v++) c += coords[(int64_t)cv[K * nvc + v] * gd + a];
      c /= nvc;
      cen[K * 3 + a] = c;
      lo[a] = std::min(lo[a], c);
      hi[a] = std::max(hi[a], c);
    }
  std::vector<std::pair<uint32_t, int64_t>> key((size_t)nc);
  for (int64_t K = 0; K < nc; K++) {
    uint32_t q[3] = {0, 0, 0};
    for (int a = 0; a < gd; a++) {
      const double w = hi[a] - lo[a];
      const double f = w > 0.0 ? (cen[K * 3 + a] - lo[a]) / w * 1024.0 : 0.0;
      q[a] = (uint32_t)std::min(1023.0, std::max(0.0, f));
    }
    key[K] = {morton3(q[0], q[1], q[2]), K};
  }
  std::sort(key.begin(), key.end());
  std::vector<int64_t> order((size_t)nc);
  for (int64_t r = 0; r < nc; r++) order[r] = key[r].second;
  return order;
}

}  // namespace mf

using namespace mf;

extern "C" {

const char *mf_last_error(void) { return g_err.c_str(); }
const char *mf_version(void) { return "mf 0.1 (gfx950)"; }

int mf_mesh_create(int cell_type, int64_t nverts, const double *coords, int64_t ncells,
                   const int32_t *cell2vert, mf_mesh **out) {
  if (!out) return fail(MF_EINVAL, "mf_mesh_create: out is NULL");
  const int nvc = nvc_of(cell_type);
  if (!nvc) return fail(MF_EINVAL, "mf_mesh_create: unknown cell type");
  if (nverts <= 0 || ncells < 0 || !coords || (ncells > 0 && !cell2vert))
    return fail(MF_EINVAL, "mf_mesh_create: bad sizes or null arrays");
  if (nverts > INT32_MAX || ncells > INT32_MAX) return fail(MF_EINVAL, "mf_mesh_create: sizes exceed int32");
  const int g = (cell_type == MF_CELL_TRI || cell_type == MF_CELL_QUAD) ? 2 : 3;
  for (int64_t i = 0; i < ncells * nvc; i++)
    if (cell2vert[i] < 0 || cell2vert[i] >= nverts)
      return fail(MF_EINVAL, "mf_mesh_create: cell2vert entry " + std::to_string(i) + " out of range");
  // degenerate / inverted cells
  for (int64_t K = 0; K < ncells; K++) {
    const int32_t *cv = cell2vert + K * nvc;
    double L = 0.0;  // longest vertex offset from vertex 0
    for (int v = 1; v < nvc; v++) {
      double s = 0.0;
      for (int a = 0; a < g; a++) {
        const double d = coords[(int64_t)cv[v] * g + a] - coords[(int64_t)cv[0] * g + a];
        s += d * d;
      }
      L = std::max(L, std::sqrt(s));
    }
    const double tol = 1e-13 * std::pow(L, g);
    if (cell_type == MF_CELL_TRI) {
      const double *p0 = coords + (int64_t)cv[0] * 2, *p1 = coords + (int64_t)cv[1] * 2, *p2 = coords + (int64_t)cv[2] * 2;
      const double det = (p1[0] - p0[0]) * (p2[1] - p0[1]) - (p2[0] - p0[0]) * (p1[1] - p0[1]);
      if (!(std::fabs(det) > tol)) return fail(MF_EMESH, "degenerate triangle " + std::to_string(K));
    } else if (cell_type == MF_CELL_TET) {
      double J[3][3];
      for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) J[a][b] = coords[(int64_t)cv[b + 1] * 3 + a] - coords[(int64_t)cv[0] * 3 + a];
      const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                         J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                         J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
      if (!(std::fabs(det) > tol)) return fail(MF_EMESH, "degenerate tetrahedron " + std::to_string(K));
    } else if (cell_type == MF_CELL_QUAD) {
      // det J of a bilinear map is affine in (xi, eta) (the xi eta terms cancel), so
      // one sign at the 4 corners holds over the cell
      int sign = 0;
      for (int corner = 0; corner < 4; corner++) {
        const double xi = corner & 1, eta = corner >> 1;
        double j[2][2];
        for (int a = 0; a < 2; a++) {
          const double X0 = coords[(int64_t)cv[0] * 2 + a], X1 = coords[(int64_t)cv[1] * 2 + a],
                       X2 = coords[(int64_t)cv[2] * 2 + a], X3 = coords[(int64_t)cv[3] * 2 + a];
          j[a][0] = (X1 - X0) + (X3 - X1 - X2 + X0) * eta;
          j[a][1] = (X2 - X0) + (X3 - X1 - X2 + X0) * xi;
        }
        const double det = j[0][0] * j[1][1] - j[0][1] * j[1][0];
        const int sg = det > tol ? 1 : det < -tol ? -1 : 0;
        if (sg == 0 || (sign != 0 && sg != sign))
          return fail(MF_EMESH, "degenerate or tangled quadrilateral " + std::to_string(K));
        sign = sg;
      }
    } else {
      double c[3][8];
      for (int a = 0; a < 3; a++) {
        double X[8];
        for (int v = 0; v < 8; v++) X[v] = coords[(int64_t)cv[v] * 3 + a];
        trilinear_coeffs(X, c[a]);
      }
      int sign = 0;
      for (int corner = 0; corner < 8; corner++) {
        const double x1 = corner & 1, x2 = (corner >> 1) & 1, x3 = (corner >> 2) & 1;
        double j1[3], j2[3], j3[3];
        for (int a = 0; a < 3; a++) {
          j1[a] = c[a][1] + c[a][4] * x2 + c[a][5] * x3 + c[a][7] * x2 * x3;
          j2[a] = c[a][2] + c[a][4] * x1 + c[a][6] * x3 + c[a][7] * x1 * x3;
          j3[a] = c[a][3] + c[a][5] * x1 + c[a][6] * x2 + c[a][7] * x1 * x2;
        }
        const double det = j1[0] * (j2[1] * j3[2] - j2[2] * j3[1]) + j1[1] * (j2[2] * j3[0] - j2[0] * j3[2]) +
                           j1[2] * (j2[0] * j3[1] - j2[1] * j3[0]);
        const int sg = det > tol ? 1 : det < -tol ? -1 : 0;
        if (sg == 0 || (sign != 0 && sg != sign))
          return fail(MF_EMESH, "degenerate or tangled hexahedron " + std::to_string(K));
        sign = sg;
      }
    }
  }
  mf_mesh *m = new (std::nothrow) mf_mesh;
  if (!m) return fail(MF_ENOMEM, "mf_mesh_create: host allocation");
  m->cell_type = cell_type;
  m->gdim = g;
  m->nvc = nvc;
  m->nverts = nverts;
  m->ncells = ncells;
  m->coords.assign(coords, coords + nverts * g);
  m->cell2vert.assign(cell2vert, cell2vert + ncells * nvc);
  *out = m;
  return MF_OK;
}

void mf_mesh_destroy(mf_mesh *m) { delete m; }

int mf_space_create(const mf_mesh *mesh, int degree, int ncomp, const int32_t *cell2node, int64_t nnodes,
                    mf_space **out) {
  if (!mesh || !out || !cell2node) return fail(MF_EINVAL, "mf_space_create: null argument");
  if (ncomp < 1 || ncomp > 3) return fail(MF_EINVAL, "mf_space_create: ncomp must be 1..3");
  if (nnodes <= 0 || nnodes > INT32_MAX / 3) return fail(MF_EINVAL, "mf_space_create: nnodes out of range");
  int D = 0;
  if (mesh->cell_type == MF_CELL_HEX) {
    if (degree < 1 || degree > 6) return fail(MF_EUNSUPPORTED, "hex spaces support degree 1..6");
    D = (degree + 1) * (degree + 1) * (degree + 1);
  } else if (mesh->cell_type == MF_CELL_QUAD) {
    if (degree < 1 || degree > 6) return fail(MF_EUNSUPPORTED, "quad spaces support degree 1..6");
    D = (degree + 1) * (degree + 1);
  } else if (mesh->cell_type == MF_CELL_TET) {
    if (degree < 1 || degree > 6) return fail(MF_EUNSUPPORTED, "tet spaces support degree 1..6");
    D = tet_ndofs(degree);
  } else {
    if (degree < 1 || degree > 6) return fail(MF_EUNSUPPORTED, "tri spaces support degree 1..6");
    D = (degree + 1) * (degree + 2) / 2;
  }
  for (int64_t i = 0; i < mesh->ncells * D; i++)
    if (cell2node[i] < 0 || cell2node[i] >= nnodes)
      return fail(MF_EINVAL, "mf_space_create: cell2node entry " + std::to_string(i) + " out of range");
  mf_space *s = new (std::nothrow) mf_space;
  if (!s) return fail(MF_ENOMEM, "mf_space_create: host allocation");
  s->cell_type = mesh->cell_type;
  s->gdim = mesh->gdim;
  s->nvc = mesh->nvc;
  s->nverts = mesh->nverts;
  s->ncells = mesh->ncells;
  s->coords = mesh->coords;
  s->cell2vert = mesh->cell2vert;
  s->degree = degree;
  s->ncomp = ncomp;
  s->D = D;
  s->nnodes = nnodes;
  s->cell2node.assign(cell2node, cell2node + mesh->ncells * D);
  // colouring: greedy first-fit in user cell order over the cell-vertex graph
  // (for conforming Lagrange spaces two cells share a node iff they share a vertex)
  const int nvc = mesh->nvc;
  const int64_t nc = mesh->ncells;
  std::vector<int64_t> vptr(mesh->nverts + 1, 0);
  for (int64_t i = 0; i < nc * nvc; i++) vptr[mesh->cell2vert[i] + 1]++;
  for (int64_t v = 0; v < mesh->nverts; v++) vptr[v + 1] += vptr[v];
  std::vector<int32_t> vcells(nc * nvc);
  {
    std::vector<int64_t> fillp(vptr.begin(), vptr.end() - 1);
    for (int64_t K = 0; K < nc; K++)
      for (int v = 0; v < nvc; v++) vcells[fillp[mesh->cell2vert[K * nvc + v]]++] = (int32_t)K;
  }
  std::vector<int32_t> colour(nc, -1);
  std::vector<int64_t> stamp;  // stamp[c] == K + 1 marks colour c as used by a neighbour of K
  int ncol = 0;
  for (int64_t K = 0; K < nc; K++) {
    for (int v = 0; v < nvc; v++) {
      const int32_t vid = mesh->cell2vert[K * nvc + v];
      for (int64_t q = vptr[vid]; q < vptr[vid + 1]; q++) {
        const int32_t c = colour[vcells[q]];
        if (c >= 0) stamp[c] = K + 1;
      }
    }
    int c = 0;
    while (c < ncol && stamp[c] == K + 1) c++;
    if (c == ncol) {
      ncol++;
      stamp.push_back(0);
    }
    colour[K] = c;
  }
  s->colour_ptr.assign(ncol + 1, 0);
  for (int64_t K = 0; K < nc; K++) s->colour_ptr[colour[K] + 1]++;
  for (int c = 0; c < ncol; c++) s->colour_ptr[c + 1] += s->colour_ptr[c];
  s->cell_user_of_int.resize(nc);
  {
    std::vector<int64_t> fillp(s->colour_ptr.begin(), s->colour_ptr.end() - 1);
    for (int64_t K = 0; K < nc; K++) s->cell_user_of_int[fillp[colour[K]]++] = (int32_t)K;
  }
  s->cell2vert_int.resize(nc * nvc);
  for (int64_t ic = 0; ic < nc; ic++)
    for (int v = 0; v < nvc; v++) s->cell2vert_int[ic * nvc + v] = mesh->cell2vert[(int64_t)s->cell_user_of_int[ic] * nvc + v];
  // internal node numbering: first appearance when the cells are traversed in the
  // internal cell order (hexahedra, quadrilaterals: the coloured hex launches store a
  // node's first contribution without reading y, which needs this order) or, for
  // simplices, in the Morton order of their centroids (the patch scatter takes
  // Morton-ordered runs of cells, whose nodes then sit together in memory: tet P2
  // elasticity 86 -> 80 us, P3 384 -> 374 us at 48^3 x 6 cells; triangles at 1024^2 x 2,
  // P2 elasticity 175 -> 161 us, P3 Laplacian 191 -> 184 us, while the coloured and
  // atomic launches of degree 6 lost 3-7 %)
  s->int_of_user.assign((size_t)nnodes, -1);
  s->user_of_int.clear();
  s->user_of_int.reserve((size_t)nnodes);
  std::vector<int64_t> walk;
  if (mesh->cell_type == MF_CELL_TET || mesh->cell_type == MF_CELL_TRI) {
    walk = morton_cell_order(s->coords, s->gdim, s->cell2vert_int.data(), nvc, nc);
  } else {
    walk.resize((size_t)nc);
    for (int64_t ic = 0; ic < nc; ic++) walk[ic] = ic;
  }
  for (int64_t ic : walk) {
    const int32_t *row = cell2node + (int64_t)s->cell_user_of_int[ic] * D;
    for (int i = 0; i < D; i++) {
      const int32_t u = row[i];
      if (s->int_of_user[u] < 0) {
        s->int_of_user[u] = (int32_t)s->user_of_int.size();
        s->user_of_int.push_back(u);
      }
    }
  }
  s->cell2node_int.resize(s->cell2node.size());
  for (int64_t ic = 0; ic < nc; ic++) {
    const int32_t *row = cell2node + (int64_t)s->cell_user_of_int[ic] * D;
    for (int i = 0; i < D; i++) s->cell2node_int[ic * D + i] = s->int_of_user[row[i]];
  }
  for (int64_t u = 0; u < nnodes; u++)  // nodes in no cell keep their relative order at the end
    if (s->int_of_user[u] < 0) {
      s->int_of_user[u] = (int32_t)s->user_of_int.size();
      s->user_of_int.push_back((int32_t)u);
    }
  s->identity = true;
  for (int64_t i = 0; i < nnodes && s->identity; i++) s->identity = s->user_of_int[i] == i;
  static std::atomic<uint64_t> next_id{1};
  s->numbering_id = next_id++;
  *out = s;
  return MF_OK;
}

int mf_space_get_colouring(const mf_space *s, int32_t *internal_to_user_cell, int64_t *colour_ptr,
                           int *ncolours) {
  if (!s || !ncolours) return fail(MF_EINVAL, "mf_space_get_colouring: null argument");
  *ncolours = (int)s->colour_ptr.size() - 1;
  if (internal_to_user_cell)
    std::memcpy(internal_to_user_cell, s->cell_user_of_int.data(), s->cell_user_of_int.size() * sizeof(int32_t));
  if (colour_ptr) std::memcpy(colour_ptr, s->colour_ptr.data(), s->colour_ptr.size() * sizeof(int64_t));
  return MF_OK;
}

int mf_space_get_permutation(const mf_space *s, int32_t *internal_to_user) {
  if (!s || !internal_to_user) return fail(MF_EINVAL, "mf_space_get_permutation: null argument");
  std::memcpy(internal_to_user, s->user_of_int.data(), s->user_of_int.size() * sizeof(int32_t));
  return MF_OK;
}

void mf_space_destroy(mf_space *s) { delete s; }

}  // extern "C"

// ------------------------------------------------------------------ operator setup
namespace mf {

static bool default_coloured(const mf_op *op);


// Patches of the Q1 patch kernel: cells in Morton order of their centroids, cut
// greedily into runs of at most `cap` cells and kPatchNodes distinct free nodes. cap
// shrinks on small meshes so that there are about 1024 patches (several per compute
// unit). m: the flagged map ([cell][D], negative = constrained); to_pos2: gather
// positions after the first user -> internal permutation stage (empty when the
// numbering is the identity); geo, cf: the [cell][entry] geometry and coefficient.
template <typename T>
static int setup_hex_patches(mf_op *op, const mf_space *sp, const std::vector<int32_t> &m,
                             const std::vector<int32_t> &to_pos2, const std::vector<T> &geo,
                             const std::vector<T> &cf, bool required, hipStream_t s) {
  constexpr bool XYZ = sizeof(T) == 8;  // FP64: vertex coordinates; FP32: stored per-slot geometry
  auto not_patched = [&](const char *why) {
    if (required) return fail(MF_EUNSUPPORTED, std::string("mf_op_create: patch scatter: ") + why);
    op->patched = false;  // keep the default of the other scatters
    op->coloured = default_coloured(op);
    return (int)MF_OK;
  };
  if (sp->nnodes > kPatchIdMask) return not_patched("too many nodes for the patch node encoding");
  const int64_t nc = sp->ncells;
  constexpr int D = 8;
  std::vector<double> cen((size_t)nc * 3);
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t K = 0; K < nc; K++)
    for (int a = 0; a < 3; a++) {
      double c = 0.0;
      for (int v = 0; v < 8; v++) c += sp->coords[(int64_t)sp->cell2vert_int[K * 8 + v] * 3 + a];
      c *= 0.125;
      cen[K * 3 + a] = c;
      lo[a] = std::min(lo[a], c);
      hi[a] = std::max(hi[a], c);
    }
  std::vector<std::pair<uint32_t, int64_t>> key((size_t)nc);
  for (int64_t K = 0; K < nc; K++) {
    uint32_t q[3];
    for (int a = 0; a < 3; a++) {
      const double w = hi[a] - lo[a];
      const double f = w > 0.0 ? (cen[K * 3 + a] - lo[a]) / w * 1024.0 : 0.0;
      q[a] = (uint32_t)std::min(1023.0, std::max(0.0, f));
    }
    key[K] = {morton3(q[0], q[1], q[2]), K};
  }
  std::sort(key.begin(), key.end());

  // capacity: a multiple of 64 near ncells / 1024, at most kPatchCells
  const int cap = 64 * (int)std::min<int64_t>(kPatchCells / 64, std::max<int64_t>(1, (nc / 1024) / 64));
  auto at = [&](int64_t p, int sl, int E, int e) -> size_t {  // slot entry position
    return (((size_t)p * (cap / 64) + sl / 64) * E + e) * 64 + sl % 64;
  };
  // Vertex coordinates per internal node (a Q1 node is a vertex: local node v of a cell
  // is its vertex v); every cell must agree, else the patch path is not used.
  const std::vector<int32_t> &c2n = sp->cell2node_int;
  std::vector<double> xyz((size_t)sp->nnodes * 3, 0.0);
  std::vector<uint8_t> seen((size_t)sp->nnodes, 0);
  for (int64_t K = 0; K < nc; K++)
    for (int v = 0; v < D; v++) {
      const int64_t n = c2n[K * D + v];
      const double *X = &sp->coords[(int64_t)sp->cell2vert_int[K * 8 + v] * 3];
      if (!seen[n]) {
        seen[n] = 1;
        for (int a = 0; a < 3; a++) xyz[n * 3 + a] = X[a];
      } else if (xyz[n * 3] != X[0] || xyz[n * 3 + 1] != X[1] || xyz[n * 3 + 2] != X[2]) {
        return not_patched("the nodes are not the cells' vertices");
      }
    }
  std::vector<int32_t> stamp((size_t)sp->nnodes, -1), loc((size_t)sp->nnodes, 0);
  std::vector<int32_t> nptr{0}, nodes;
  std::vector<uint16_t> lmap;
  std::vector<T> pgeo, pcoef;
  int pid = -1, ncell = 0, nnode = 0;
  auto open_patch = [&]() {
    pid++;
    ncell = nnode = 0;
    lmap.resize((size_t)(pid + 1) * cap * D, kPatchEmpty);
    if (!XYZ) {
      pgeo.resize((size_t)(pid + 1) * cap * 24, T(0));
      for (int sl = 0; sl < cap; sl++)  // empty slots: the unit-cube map
        for (int j : {0, 4, 8}) pgeo[at(pid, sl, 24, j)] = T(1);
    }
    if (op->has_coef) pcoef.resize((size_t)(pid + 1) * cap * 8, T(0));
  };
  for (int64_t r = 0; r < nc; r++) {
    const int64_t K = key[r].second;
    int fresh = 0;
    for (int i = 0; i < D; i++)
      if (stamp[c2n[K * D + i]] != pid) fresh++;
    if (pid < 0 || ncell == cap || nnode + fresh > kPatchNodes) {
      if (pid >= 0) nptr.push_back((int32_t)nodes.size());
      open_patch();
    }
    const int sl = ncell++;
    for (int i = 0; i < D; i++) {
      const int32_t id = c2n[K * D + i];
      if (stamp[id] != pid) {
        stamp[id] = pid;
        loc[id] = nnode++;
        nodes.push_back(m[K * D + i] >= 0 ? id : (id | kPatchFixed));  // constrained: coordinates only
      }
      lmap[at(pid, sl, D, i)] = (uint16_t)loc[id];
    }
    if (!XYZ)
      for (int j = 0; j < 24; j++) pgeo[at(pid, sl, 24, j)] = geo[K * 24 + j];
    if (op->has_coef)
      for (int j = 0; j < 8; j++) pcoef[at(pid, sl, 8, j)] = cf[K * 8 + j];
  }
  if (pid >= 0) nptr.push_back((int32_t)nodes.size());
  const int np = pid + 1;
  // nodes that more than one patch touches are written with atomics
  std::vector<uint8_t> cnt((size_t)sp->nnodes, 0);
  for (int32_t e : nodes) cnt[e & kPatchIdMask] = (uint8_t)std::min(2, cnt[e & kPatchIdMask] + 1);
  int max_nodes = 0;
  for (int p = 0; p < np; p++) max_nodes = std::max(max_nodes, nptr[p + 1] - nptr[p]);
  for (int32_t &e : nodes)
    if (cnt[e & kPatchIdMask] > 1) e |= kPatchShared;
  op->npatch = np;
  op->pt_max_nodes = max_nodes;
  op->pt_cap = cap;
  int rc = upload(op->pt_nptr, nptr.data(), nptr.size() * sizeof(int32_t), s);
  if (!rc) rc = upload(op->pt_nodes, nodes.data(), nodes.size() * sizeof(int32_t), s);
  if (!rc) rc = upload(op->pt_lmap, lmap.data(), lmap.size() * sizeof(uint16_t), s);
  if (!rc && XYZ) rc = upload(op->pt_xyz, xyz.data(), xyz.size() * sizeof(double), s);
  if (!rc && !XYZ) rc = upload(op->pt_geo, pgeo.data(), pgeo.size() * sizeof(T), s);
  if (!rc && op->has_coef) rc = upload(op->pt_coef, pcoef.data(), pcoef.size() * sizeof(T), s);
  std::vector<int32_t> gn;
  if (!rc && !to_pos2.empty()) {  // gather positions after the first permutation stage
    gn.resize(nodes.size());
    for (size_t i = 0; i < nodes.size(); i++) gn[i] = to_pos2[nodes[i] & kPatchIdMask];
    rc = upload(op->pt_gnodes, gn.data(), gn.size() * sizeof(int32_t), s);
  }
  if (!rc) MF_HIP(hipStreamSynchronize(s));  // the host vectors go out of scope
  return rc;
}

// Patch scatter of the hex pencil kernel: patches are runs of EPB consecutive cells in
// the Morton order of the cell centroids (EPB: the kernel's cells per workgroup), the
// cell arrays are copied into patch-slot order, and each patch lists its free nodes;
// nodes of more than one patch get sbuf slots (as the simplex patches).
template <typename T>
static int setup_hex_cell_patches(mf_op *op, const mf_space *sp, const std::vector<int32_t> &m,
                                  const std::vector<int32_t> &gm, const std::vector<T> &geo,
                                  const std::vector<T> &cf, hipStream_t s) {
  const int64_t nc = sp->ncells;
  const int D = sp->D, N = sp->degree + 1, E = hex_cells_per_patch(N);
  if (E <= 0) return fail(MF_EUNSUPPORTED, "hex patch scatter: degree");
  std::vector<std::pair<uint32_t, int64_t>> key((size_t)nc);
  {
    std::vector<double> cen((size_t)nc * 3);
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t K = 0; K < nc; K++)
      for (int a = 0; a < 3; a++) {
        double c = 0.0;
        for (int v = 0; v < 8; v++) c += sp->coords[(int64_t)sp->cell2vert_int[K * 8 + v] * 3 + a];
        cen[K * 3 + a] = c * 0.125;
        lo[a] = std::min(lo[a], c * 0.125);
        hi[a] = std::max(hi[a], c * 0.125);
      }
    for (int64_t K = 0; K < nc; K++) {
      uint32_t q[3];
      for (int a = 0; a < 3; a++) {
        const double w = hi[a] - lo[a];
        const double f = w > 0.0 ? (cen[K * 3 + a] - lo[a]) / w * 1024.0 : 0.0;
        q[a] = (uint32_t)std::min(1023.0, std::max(0.0, f));
      }
      key[K] = {morton3(q[0], q[1], q[2]), K};
    }
    std::sort(key.begin(), key.end());
  }
  const int64_t np = (nc + E - 1) / E, ns = np * E;
  std::vector<int32_t> pmap((size_t)ns * D, -1), pgmap(gm.empty() ? 0 : (size_t)ns * D, -1), nptr{0}, nodes;
  std::vector<uint16_t> plmap((size_t)ns * D, kSlotSkip);
  std::vector<T> pgeo((size_t)ns * 24, T(0)), pcf(op->has_coef ? (size_t)ns * 8 : 0, T(0));
  std::vector<int32_t> stamp((size_t)sp->nnodes, -1), loc((size_t)sp->nnodes, 0);
  for (int64_t q = 0; q < ns; q++) {
    const int64_t p = q / E;
    if (q >= nc) {  // empty slot: the unit cube, coefficient 1, no nodes
      for (int j : {0, 4, 8}) pgeo[q * 24 + j] = T(1);
      if (op->has_coef) pcf[q * 8] = T(1);
      continue;
    }
    const int64_t K = key[q].second;
    for (int i = 0; i < D; i++) {
      const int32_t n = m[K * D + i];
      pmap[q * D + i] = n;
      if (!gm.empty()) pgmap[q * D + i] = gm[K * D + i];
      if (n < 0) continue;
      if (stamp[n] != (int32_t)p) {
        stamp[n] = (int32_t)p;
        loc[n] = (int32_t)nodes.size() - nptr[p];
        nodes.push_back(n);
      }
      plmap[q * D + i] = (uint16_t)loc[n];
    }
    for (int j = 0; j < 24; j++) pgeo[q * 24 + j] = geo[K * 24 + j];
    if (op->has_coef)
      for (int j = 0; j < 8; j++) pcf[q * 8 + j] = cf[K * 8 + j];
    if ((q + 1) % E == 0 || q + 1 == nc) nptr.push_back((int32_t)nodes.size());
  }
  while ((int64_t)nptr.size() < np + 1) nptr.push_back((int32_t)nodes.size());
  std::vector<int32_t> pc((size_t)sp->nnodes, 0);
  for (int32_t n : nodes) pc[n]++;
  std::vector<int32_t> sidx((size_t)sp->nnodes, -1), sptr{0}, snode;
  for (int64_t n = 0; n < sp->nnodes; n++)
    if (pc[n] > 1) {
      sidx[n] = (int32_t)snode.size();
      snode.push_back((int32_t)n);
      sptr.push_back(sptr.back() + pc[n]);
    }
  if ((int64_t)sptr.back() >= (int64_t)kSharedOut || (int64_t)sp->nnodes >= (int64_t)kSharedOut)
    return fail(MF_EUNSUPPORTED, "hex patch scatter: too many nodes");
  std::vector<int32_t> fill(snode.size(), 0), out(nodes.size());
  for (size_t e = 0; e < nodes.size(); e++) {
    const int32_t n = nodes[e];
    out[e] = sidx[n] < 0 ? n : (kSharedOut | (sptr[sidx[n]] + fill[sidx[n]]++));
  }
  op->hp_npatch = (int)np;
  op->sp_nshared = (int64_t)snode.size();
  int rc = upload(op->hp_map, pmap.data(), pmap.size() * sizeof(int32_t), s);
  if (!rc && !pgmap.empty()) rc = upload(op->hp_gmap, pgmap.data(), pgmap.size() * sizeof(int32_t), s);
  if (!rc) rc = upload(op->hp_lmap, plmap.data(), plmap.size() * sizeof(uint16_t), s);
  if (!rc) rc = upload(op->hp_geo, pgeo.data(), pgeo.size() * sizeof(T), s);
  if (!rc && op->has_coef) rc = upload(op->hp_coef, pcf.data(), pcf.size() * sizeof(T), s);
  if (!rc) rc = upload(op->hp_nptr, nptr.data(), nptr.size() * sizeof(int32_t), s);
  if (!rc) rc = upload(op->hp_out, out.data(), out.size() * sizeof(int32_t), s);
  if (!rc) rc = upload(op->sp_sptr, sptr.data(), sptr.size() * sizeof(int32_t), s);
  if (!rc && !snode.empty()) rc = upload(op->sp_snode, snode.data(), snode.size() * sizeof(int32_t), s);
  if (!rc) rc = op->sp_sbuf.alloc(std::max<size_t>(1, (size_t)sptr.back()) * sp->ncomp * sizeof(T));
  if (!rc) MF_HIP(hipStreamSynchronize(s));  // the host vectors go out of scope
  return rc;
}

template <typename T>
static int setup_hex(mf_op *op, const mf_space *sp, const mf_op_params *pr, const std::vector<int32_t> &m,
                     const std::vector<int32_t> &to_pos2, hipStream_t s) {
  const int k = sp->degree, N = k + 1;
  if (op->nq1d != N && op->nq1d != N + 1)
    return fail(MF_EUNSUPPORTED, "hex operators: nq1d must be k+1 or k+2");
  const int64_t nc = sp->ncells;
  std::vector<T> geo((size_t)nc * 24, T(0));
  for (int64_t K = 0; K < nc; K++) {
    for (int a = 0; a < 3; a++) {
      double X[8], c[8];
      for (int v = 0; v < 8; v++) X[v] = sp->coords[(int64_t)sp->cell2vert_int[K * 8 + v] * 3 + a];
      trilinear_coeffs(X, c);
      for (int m = 1; m < 8; m++) geo[K * 24 + 3 * (m - 1) + a] = (T)c[m];
    }
  }
  int rc = upload(op->geo, geo.data(), geo.size() * sizeof(T), s);
  if (rc) return rc;
  std::vector<T> cf;
  if (op->has_coef) {
    cf.resize((size_t)nc * 8);
    for (int64_t K = 0; K < nc; K++) {
      double X[8], c[8];
      for (int v = 0; v < 8; v++) X[v] = pr->vertex_coef[sp->cell2vert_int[K * 8 + v]];
      trilinear_coeffs(X, c);
      for (int m = 0; m < 8; m++) cf[K * 8 + m] = (T)c[m];
    }
    rc = upload(op->coef, cf.data(), cf.size() * sizeof(T), s);
    if (rc) return rc;
  }
  if (k == 1) {
    // block-interleaved copies for the degree-1 kernel; cells past the end get the
    // unit-cube map and coefficient 1
    const int64_t nb = (nc + 63) / 64;
    std::vector<T> g2((size_t)nb * 24 * 64, T(0)), k2;
    for (int64_t K = 0; K < nb * 64; K++)
      for (int j = 0; j < 24; j++)
        g2[((K / 64) * 24 + j) * 64 + K % 64] = K < nc ? geo[K * 24 + j] : T(j == 0 || j == 4 || j == 8 ? 1 : 0);
    rc = upload(op->q1geo, g2.data(), g2.size() * sizeof(T), s);
    if (!rc && op->has_coef) {
      k2.assign((size_t)nb * 8 * 64, T(0));
      for (int64_t K = 0; K < nb * 64; K++)
        for (int j = 0; j < 8; j++) k2[((K / 64) * 8 + j) * 64 + K % 64] = K < nc ? cf[K * 8 + j] : T(j == 0 ? 1 : 0);
      rc = upload(op->q1coef, k2.data(), k2.size() * sizeof(T), s);
    }
    if (!rc) MF_HIP(hipStreamSynchronize(s));  // the host vectors go out of scope
    if (rc) return rc;
  }
  if (op->kind == MF_OP_HYPERELASTIC) {
    // linearisation point in internal numbering (every node, constrained ones included);
    // with constrained nodes the map flags them, so u0 is gathered through an unflagged copy
    std::vector<T> u0((size_t)sp->nnodes * 3);
    for (int64_t n = 0; n < sp->nnodes; n++)
      for (int c = 0; c < 3; c++) u0[n * 3 + c] = (T)pr->u0[(int64_t)sp->user_of_int[n] * 3 + c];
    rc = upload(op->u0, u0.data(), u0.size() * sizeof(T), s);
    if (!rc && pr->dirichlet) rc = upload(op->u0map, sp->cell2node_int.data(), sp->cell2node_int.size() * 4, s);
    if (!rc) MF_HIP(hipStreamSynchronize(s));
    if (rc) return rc;
  }
  if (op->patched) return setup_hex_patches<T>(op, sp, m, to_pos2, geo, cf, pr->scatter == MF_SCATTER_PATCH, s);
  if (op->hpatched) {
    std::vector<int32_t> gm;
    if (op->fused_gather) {
      gm.resize(m.size());
      for (size_t i = 0; i < m.size(); i++) gm[i] = m[i] >= 0 ? to_pos2[m[i]] : m[i];
    }
    return setup_hex_cell_patches<T>(op, sp, m, gm, geo, cf, s);
  }
  return MF_OK;
}

// Simplex patch scatter (SimplexPatchArgs), built from the flagged internal map m
// (AoSoA [cell/64][D][64]) and the per-cell geometry gflat ([cell][G]): cells in Morton
// order of their centroids, greedy patches of at most cap cells and nmax free nodes.
template <typename T>
static int setup_simplex_patches(mf_op *op, const mf_space *sp, const std::vector<int32_t> &m, bool m_aosoa,
                                 const std::vector<T> &gflat, int G, int cap, int nmax, hipStream_t s) {
  const int64_t nc = sp->ncells;
  const int D = sp->D, nv = sp->nvc, gd = sp->gdim;
  auto mp = [&](int64_t K, int i) { return m_aosoa ? m[((K / 64) * D + i) * 64 + K % 64] : m[K * D + i]; };
  const std::vector<int64_t> order = morton_cell_order(sp->coords, gd, sp->cell2vert_int.data(), nv, nc);
  // greedy patches: slots (patch, slot) hold cells; node lists of free nodes
  std::vector<int32_t> stamp((size_t)sp->nnodes, -1), loc((size_t)sp->nnodes, 0);
  std::vector<int32_t> nptr{0}, nodes;
  std::vector<int64_t> slot_cell;  // per slot: cell or -1
  int pid = -1, ncell = 0, nnode = 0;
  for (int64_t r = 0; r < nc; r++) {
    const int64_t K = order[r];
    int fresh = 0;
    for (int i = 0; i < D; i++) {
      const int32_t n = mp(K, i);
      if (n >= 0 && stamp[n] != pid) fresh++;
    }
    if (pid < 0 || ncell == cap || nnode + fresh > nmax) {
      if (pid >= 0) {
        nptr.push_back((int32_t)nodes.size());
        slot_cell.resize((size_t)(pid + 1) * cap, -1);
      }
      pid++;
      ncell = nnode = 0;
    }
    slot_cell.resize((size_t)pid * cap + ncell + 1, -1);
    slot_cell[(size_t)pid * cap + ncell] = K;
    ncell++;
    for (int i = 0; i < D; i++) {
      const int32_t n = mp(K, i);
      if (n >= 0 && stamp[n] != pid) {
        stamp[n] = pid;
        loc[n] = nnode++;
        nodes.push_back(n);
      }
    }
  }
  const int np = pid + 1;
  nptr.push_back((int32_t)nodes.size());
  slot_cell.resize((size_t)np * cap, -1);
  int maxn = 0;
  for (int p = 0; p < np; p++) maxn = std::max(maxn, nptr[p + 1] - nptr[p]);
  // per-slot AoSoA arrays (local indices from each patch's own node list)
  const int64_t nblk = (int64_t)np * cap / 64;
  std::vector<int32_t> smap((size_t)nblk * D * 64, -1);
  std::vector<uint16_t> slmap((size_t)nblk * D * 64, kSlotSkip);
  std::vector<T> sgeo((size_t)nblk * G * 64, T(0));
  {
    std::vector<int32_t> lidx((size_t)sp->nnodes, -1);
    for (int p = 0; p < np; p++) {
      for (int e = nptr[p]; e < nptr[p + 1]; e++) lidx[nodes[e]] = e - nptr[p];
      for (int sl = 0; sl < cap; sl++) {
        const int64_t K = slot_cell[(size_t)p * cap + sl];
        if (K < 0) continue;
        const int64_t q = (int64_t)p * cap + sl, b = q / 64, l = q % 64;
        for (int i = 0; i < D; i++) {
          const int32_t n = mp(K, i);
          smap[(b * D + i) * 64 + l] = n;
          if (n >= 0) slmap[(b * D + i) * 64 + l] = (uint16_t)lidx[n];
        }
        for (int e = 0; e < G; e++) sgeo[(b * G + e) * 64 + l] = gflat[(size_t)K * G + e];
      }
    }
  }
  // nodes of more than one patch: their contributions go to sbuf slots, summed in
  // patch order by the shared-node reduction
  std::vector<int32_t> pc((size_t)sp->nnodes, 0);
  for (int32_t n : nodes) pc[n]++;
  std::vector<int32_t> sidx((size_t)sp->nnodes, -1), sptr{0}, snode;
  for (int64_t n = 0; n < sp->nnodes; n++)
    if (pc[n] > 1) {
      sidx[n] = (int32_t)snode.size();
      snode.push_back((int32_t)n);
      sptr.push_back(sptr.back() + pc[n]);
    }
  if ((int64_t)sptr.back() >= (int64_t)kSharedOut || (int64_t)sp->nnodes >= (int64_t)kSharedOut)
    return fail(MF_EUNSUPPORTED, "simplex patch scatter: too many nodes");
  std::vector<int32_t> fill(snode.size(), 0), out(nodes.size());
  for (size_t e = 0; e < nodes.size(); e++) {
    const int32_t n = nodes[e];
    out[e] = sidx[n] < 0 ? n : (kSharedOut | (sptr[sidx[n]] + fill[sidx[n]]++));
  }
  op->sp_npatch = np;
  op->sp_cap = cap;
  op->sp_nmax = maxn;
  op->sp_nshared = (int64_t)snode.size();
  int rc = upload(op->sp_map, smap.data(), smap.size() * sizeof(int32_t), s);
  if (!rc) rc = upload(op->sp_lmap, slmap.data(), slmap.size() * sizeof(uint16_t), s);
  if (!rc) rc = upload(op->sp_geo, sgeo.data(), sgeo.size() * sizeof(T), s);
  if (!rc) rc = upload(op->sp_nptr, nptr.data(), nptr.size() * sizeof(int32_t), s);
  if (!rc) rc = upload(op->sp_out, out.data(), out.size() * sizeof(int32_t), s);
  if (!rc) rc = upload(op->sp_sptr, sptr.data(), sptr.size() * sizeof(int32_t), s);
  if (!rc && !snode.empty()) rc = upload(op->sp_snode, snode.data(), snode.size() * sizeof(int32_t), s);
  if (!rc) rc = op->sp_sbuf.alloc(std::max<size_t>(1, (size_t)sptr.back()) * sp->ncomp * sizeof(T));
  if (!rc) MF_HIP(hipStreamSynchronize(s));  // the host vectors go out of scope
  return rc;
}

template <typename T>
static int setup_tet(mf_op *op, const mf_space *sp, const mf_op_params *pr, const std::vector<int32_t> &m,
                     hipStream_t s) {
  const int k = sp->degree, D = sp->D;
  std::vector<double> pts, w, phi, dphi;
  const bool hyper = op->kind == MF_OP_HYPERELASTIC;
  const bool scalar = sp->ncomp == 1;  // MASS, HELMHOLTZ, LAPLACIAN, POISSON
  // integrand degree on affine cells: grad u . grad v (the hyperelastic tangent adds
  // grad u0 three times: S is quadratic in it, then F S and F dS); u v for the value
  // terms; one more with a (linearly interpolated) vertex coefficient
  int deg = hyper ? 4 * (k - 1) : 2 * k - 2;
  if (scalar) {
    deg = (op->kind == MF_OP_MASS || op->kind == MF_OP_HELMHOLTZ) ? 2 * k : 2 * k - 2;
    if (op->has_coef) deg += 1;
  }
  if (!tet_rule(deg, pts, w)) return fail(MF_EUNSUPPORTED, "tet quadrature degree (the rules end at 21)");
  op->qdeg = deg;
  const int nq = (int)w.size();
  op->nqp = nq;
  tet_lagrange(k, pts, phi, dphi);
  std::vector<T> tab;
  if (scalar) {
    // phi [nq][D], reference gradients [nq][D][3], weights [nq], vertex basis [nq][4]
    for (double v : phi) tab.push_back((T)v);
    for (double v : dphi) tab.push_back((T)v);
    for (double v : w) tab.push_back((T)v);
    for (int q = 0; q < nq; q++) {
      const double *x = &pts[3 * q];
      tab.push_back((T)(1.0 - x[0] - x[1] - x[2]));
      for (int a = 0; a < 3; a++) tab.push_back((T)x[a]);
    }
    // per-lane operands of the MFMA contractions
    std::vector<double> mt((size_t)simplex_mfma_scalar_table_floats(3, D, nq));
    simplex_mfma_scalar_tables(3, D, nq, phi.data(), dphi.data(), mt.data(), sizeof(T) == 8);
    for (double v : mt) tab.push_back((T)v);
  } else {
    for (double v : dphi) tab.push_back((T)v);
    for (double v : w) tab.push_back((T)v);
  }
  if (!scalar && (k >= 2 || hyper)) {
    // per-lane operands of the MFMA contractions, appended after the weights (P1
    // elasticity keeps a lane-per-cell kernel; the hyperelastic tangent runs the MFMA
    // kernel at every degree)
    std::vector<double> mt((size_t)tet_mfma_table_floats(k, nq));
    tet_mfma_tables(k, nq, dphi.data(), mt.data(), sizeof(T) == 8);
    for (double v : mt) tab.push_back((T)v);
  }
  int rc = upload(op->tab, tab.data(), tab.size() * sizeof(T), s);
  if (rc) return rc;
  const int64_t nc = sp->ncells, nb = (nc + 63) / 64;
  if (scalar && op->has_coef) {
    // vertex coefficients per cell, AoSoA [cell/64][4][64]
    std::vector<T> cf((size_t)nb * 4 * 64, T(1));
    for (int64_t K = 0; K < nc; K++)
      for (int v = 0; v < 4; v++)
        cf[((K / 64) * 4 + v) * 64 + K % 64] = (T)pr->vertex_coef[sp->cell2vert_int[K * 4 + v]];
    rc = upload(op->coef, cf.data(), cf.size() * sizeof(T), s);
    if (!rc) MF_HIP(hipStreamSynchronize(s));
    if (rc) return rc;
  }
  if (hyper) {
    // linearisation point in internal numbering (every node, constrained ones included)
    std::vector<T> u0((size_t)sp->nnodes * 3);
    for (int64_t n = 0; n < sp->nnodes; n++)
      for (int c = 0; c < 3; c++) u0[n * 3 + c] = (T)pr->u0[(int64_t)sp->user_of_int[n] * 3 + c];
    rc = upload(op->u0, u0.data(), u0.size() * sizeof(T), s);
    if (!rc && pr->dirichlet) {
      // the map flags constrained nodes; u0 is gathered through an unflagged copy
      std::vector<int32_t> um((size_t)nb * D * 64, -1);
      for (int64_t K = 0; K < nc; K++)
        for (int i = 0; i < D; i++) um[((K / 64) * D + i) * 64 + K % 64] = sp->cell2node_int[K * D + i];
      rc = upload(op->u0map, um.data(), um.size() * sizeof(int32_t), s);
    }
    if (!rc) MF_HIP(hipStreamSynchronize(s));  // the host vectors go out of scope
    if (rc) return rc;
  }
  // patch slots carry the geometry and, for MASS and POISSON, the four vertex
  // coefficients (1 without one)
  const bool slot_coef = scalar && (op->kind == MF_OP_MASS || op->kind == MF_OP_POISSON);
  const int G = slot_coef ? 14 : 10;
  std::vector<T> geo((size_t)nb * 10 * 64, T(0)), gflat(op->spatched ? (size_t)nc * G : 0);
  for (int64_t K = 0; K < nc; K++) {
    const int32_t *cv = sp->cell2vert_int.data() + K * 4;
    double J[3][3];
    for (int a = 0; a < 3; a++)
      for (int b = 0; b < 3; b++) J[a][b] = sp->coords[(int64_t)cv[b + 1] * 3 + a] - sp->coords[(int64_t)cv[0] * 3 + a];
    // columns j_b = J[:, b]; rows of J^{-1}: (j2 x j3, j3 x j1, j1 x j2) / det
    double jc[3][3];
    for (int b = 0; b < 3; b++)
      for (int a = 0; a < 3; a++) jc[b][a] = J[a][b];
    auto cross = [](const double *u, const double *v, double *o) {
      o[0] = u[1] * v[2] - u[2] * v[1];
      o[1] = u[2] * v[0] - u[0] * v[2];
      o[2] = u[0] * v[1] - u[1] * v[0];
    };
    double R[3][3];
    cross(jc[1], jc[2], R[0]);
    cross(jc[2], jc[0], R[1]);
    cross(jc[0], jc[1], R[2]);
    const double det = jc[0][0] * R[0][0] + jc[0][1] * R[0][1] + jc[0][2] * R[0][2];
    const int64_t b = K / 64, l = K % 64;
    for (int bb = 0; bb < 3; bb++)
      for (int a = 0; a < 3; a++) geo[(b * 10 + 3 * bb + a) * 64 + l] = (T)(R[bb][a] / det);
    geo[(b * 10 + 9) * 64 + l] = (T)std::fabs(det);
    if (op->spatched) {
      for (int e = 0; e < 10; e++) gflat[(size_t)K * G + e] = geo[(b * 10 + e) * 64 + l];
      for (int v = 0; v < G - 10; v++)
        gflat[(size_t)K * G + 10 + v] = op->has_coef ? (T)pr->vertex_coef[cv[v]] : T(1);
    }
  }
  rc = upload(op->geo, geo.data(), geo.size() * sizeof(T), s);
  if (!rc && op->spatched) {
    // patch sizes measured best on 48^3 x 6 cells among 128..1024 cells and 1024..2700
    // nodes: P2 384 cells / 2048 nodes (FP64 72, FP32 57 us; 512 cells: 80, 74 us), P3
    // 384 / 2700 in FP64 (352 us; 256 / 2048: 366 us), 256 / 2048 in FP32 (210 us)
    const bool f64 = sizeof(T) == 8;
    int cap = k <= 2 ? 384 : (f64 ? 384 : 256), nmax = k <= 2 ? 2048 : (f64 ? 2700 : 2048);
    if (k == 1) cap = 1024;  // one-component P1: about 200 nodes per 1024 cells
    if (k >= 4) {  // one-component P4-P6: about k^3 / 6 nodes per cell. At 24^3 x 6 the
      // patches beat atomics in FP32 for P4 and P5 (Laplacian 147 -> 101 us, 291 -> 196 us)
      // and lost in FP64 (140 -> 174 us, 311 -> 263 us for P5 but 699 -> 1834 us for P6)
      cap = k == 4 ? 256 : 128;
      nmax = 4096;
    }
    rc = setup_simplex_patches<T>(op, sp, m, true, gflat, G, cap, nmax, s);
  }
  if (!rc) MF_HIP(hipStreamSynchronize(s));
  return rc;
}

// Triangles other than the closed-form P1 mass: tables (phi, reference gradients,
// weights, vertex basis at the points of a collapsed rule exact for the integrand),
// geometry [cell/64][5][64] (d xi_b / d x_a, |det J|), coefficients [cell/64][3][64].
template <typename T>
static int setup_tri_pk(mf_op *op, const mf_space *sp, const mf_op_params *pr, const std::vector<int32_t> &m,
                        hipStream_t s) {
  const int k = sp->degree;
  int deg = (op->kind == MF_OP_MASS || op->kind == MF_OP_HELMHOLTZ) ? 2 * k : 2 * k - 2;
  if (op->has_coef) deg += 1;
  op->qdeg = deg;
  std::vector<double> pts, w, phi, dphi;
  tri_rule(deg, pts, w);
  tri_lagrange(k, pts, phi, dphi);
  const int nq = (int)w.size();
  op->nqp = nq;
  // phi [nq][D], reference gradients [nq][D][2], weights [nq], vertex basis [nq][3],
  // then the per-lane operands of the matrix-core kernels
  std::vector<T> tab;
  for (double v : phi) tab.push_back((T)v);
  for (double v : dphi) tab.push_back((T)v);
  for (double v : w) tab.push_back((T)v);
  for (int q = 0; q < nq; q++) {
    tab.push_back((T)(1.0 - pts[2 * q] - pts[2 * q + 1]));
    tab.push_back((T)pts[2 * q]);
    tab.push_back((T)pts[2 * q + 1]);
  }
  {
    std::vector<double> mt((size_t)simplex_mfma_scalar_table_floats(2, sp->D, nq));
    simplex_mfma_scalar_tables(2, sp->D, nq, phi.data(), dphi.data(), mt.data(), sizeof(T) == 8);
    for (double v : mt) tab.push_back((T)v);
  }
  int rc = upload(op->tab, tab.data(), tab.size() * sizeof(T), s);
  if (rc) return rc;
  const int64_t nc = sp->ncells, nb = (nc + 63) / 64;
  std::vector<T> geo((size_t)nb * 5 * 64, T(0)), cf;
  if (op->has_coef) cf.assign((size_t)nb * 3 * 64, T(1));
  // patch slots: the geometry and, for MASS and POISSON, the three vertex coefficients
  const bool slot_coef = op->kind == MF_OP_MASS || op->kind == MF_OP_POISSON;
  const int nmax = op->kind == MF_OP_ELASTICITY ? 2048 : 4096;  // FP64 sums: 16 or 8 bytes per node
  const int G = slot_coef ? 8 : 5;
  std::vector<T> gflat(op->spatched ? (size_t)nc * G : 0);
  for (int64_t K = 0; K < nc; K++) {
    const int32_t *cv = sp->cell2vert_int.data() + K * 3;
    const double *p0 = &sp->coords[(int64_t)cv[0] * 2], *p1 = &sp->coords[(int64_t)cv[1] * 2],
                 *p2 = &sp->coords[(int64_t)cv[2] * 2];
    // J = [p1 - p0, p2 - p0] (columns); J^{-1}[b][a] = d xi_b / d x_a
    const double j00 = p1[0] - p0[0], j01 = p2[0] - p0[0], j10 = p1[1] - p0[1], j11 = p2[1] - p0[1];
    const double det = j00 * j11 - j01 * j10;
    const double inv[4] = {j11 / det, -j01 / det, -j10 / det, j00 / det};
    const int64_t b = K / 64, l = K % 64;
    for (int m = 0; m < 4; m++) geo[(b * 5 + m) * 64 + l] = (T)inv[m];
    geo[(b * 5 + 4) * 64 + l] = (T)std::fabs(det);
    if (op->has_coef)
      for (int v = 0; v < 3; v++) cf[(b * 3 + v) * 64 + l] = (T)pr->vertex_coef[cv[v]];
    if (op->spatched) {
      for (int e = 0; e < 5; e++) gflat[(size_t)K * G + e] = geo[(b * 5 + e) * 64 + l];
      for (int v = 0; v < G - 5; v++) gflat[(size_t)K * G + 5 + v] = op->has_coef ? (T)pr->vertex_coef[cv[v]] : T(1);
    }
  }
  rc = upload(op->geo, geo.data(), geo.size() * sizeof(T), s);
  if (!rc && op->has_coef) rc = upload(op->coef, cf.data(), cf.size() * sizeof(T), s);
  if (!rc && op->spatched) {
    // about k^2 / 2 nodes per cell: patches of at most 4096 nodes (elasticity 2048)
    const int cap = k <= 1 ? 2048 : k == 2 ? 1024 : k == 3 ? 512 : k == 4 ? 384 : 256;
    rc = setup_simplex_patches<T>(op, sp, m, true, gflat, G, cap, nmax, s);
  }
  if (!rc) MF_HIP(hipStreamSynchronize(s));
  return rc;
}

template <typename T>
static int setup_tri(mf_op *op, const mf_space *sp, const mf_op_params *pr, const std::vector<int32_t> &m,
                     hipStream_t s) {
  if (!(op->kind == MF_OP_MASS && sp->degree == 1)) return setup_tri_pk<T>(op, sp, pr, m, s);
  const int64_t nc = sp->ncells;
  std::vector<T> geo((size_t)nc * 4, T(0)), gflat(op->spatched ? (size_t)nc * 3 : 0);
  for (int64_t K = 0; K < nc; K++) {
    const int32_t *cv = sp->cell2vert_int.data() + K * 3;
    const double *p0 = &sp->coords[(int64_t)cv[0] * 2], *p1 = &sp->coords[(int64_t)cv[1] * 2],
                 *p2 = &sp->coords[(int64_t)cv[2] * 2];
    const double area = 0.5 * std::fabs((p1[0] - p0[0]) * (p2[1] - p0[1]) - (p2[0] - p0[0]) * (p1[1] - p0[1]));
    for (int i = 0; i < 3; i++) geo[K * 4 + i] = (T)(area * (op->has_coef ? pr->vertex_coef[cv[i]] : 1.0));
    if (op->spatched)
      for (int i = 0; i < 3; i++) gflat[K * 3 + i] = geo[K * 4 + i];
  }
  op->nqp = 0;
  int rc = upload(op->geo, geo.data(), geo.size() * sizeof(T), s);
  // patches of 2048 cells with at most 2048 nodes
  if (!rc && op->spatched) rc = setup_simplex_patches<T>(op, sp, m, false, gflat, 3, 2048, 2048, s);
  if (!rc) MF_HIP(hipStreamSynchronize(s));
  return rc;
}

// Quads: 1D tables (GLL Lagrange basis and its derivative at the Gauss points, the
// weights and the points), the bilinear map coefficients per cell [cell][6] and the
// vertex coefficients [cell][4], in internal cell order.
// 1D tables of the tensor-product kernels (quads, hex elasticity and hyperelasticity):
// the GLL Lagrange basis B[a][i] and its derivative at the nq1d Gauss points, the
// weights, the points
template <typename T> static int upload_tensor_tables(mf_op *op, hipStream_t s) {
  std::vector<double> g, w, V, dV;
  gauss_legendre(op->nq1d, g, w);
  lagrange_eval(gll_points(op->degree), g, V, dV);
  std::vector<T> tab;
  for (double v : V) tab.push_back((T)v);
  for (double v : dV) tab.push_back((T)v);
  for (double v : w) tab.push_back((T)v);
  for (double v : g) tab.push_back((T)v);
  int rc = upload(op->tab, tab.data(), tab.size() * sizeof(T), s);
  if (!rc) MF_HIP(hipStreamSynchronize(s));
  return rc;
}

template <typename T> static int setup_quad(mf_op *op, const mf_space *sp, const mf_op_params *pr, hipStream_t s) {
  int rc = upload_tensor_tables<T>(op, s);
  if (rc) return rc;
  const int64_t nc = sp->ncells;
  std::vector<T> geo((size_t)nc * 6), cf;
  if (op->has_coef) cf.resize((size_t)nc * 4);
  for (int64_t K = 0; K < nc; K++) {
    const int32_t *cv = sp->cell2vert_int.data() + K * 4;
    for (int a = 0; a < 2; a++) {
      const double X0 = sp->coords[(int64_t)cv[0] * 2 + a], X1 = sp->coords[(int64_t)cv[1] * 2 + a],
                   X2 = sp->coords[(int64_t)cv[2] * 2 + a], X3 = sp->coords[(int64_t)cv[3] * 2 + a];
      geo[K * 6 + 0 + a] = (T)(X1 - X0);
      geo[K * 6 + 2 + a] = (T)(X2 - X0);
      geo[K * 6 + 4 + a] = (T)(X3 - X1 - X2 + X0);
    }
    if (op->has_coef)
      for (int v = 0; v < 4; v++) cf[K * 4 + v] = (T)pr->vertex_coef[cv[v]];
  }
  rc = upload(op->geo, geo.data(), geo.size() * sizeof(T), s);
  if (!rc && op->has_coef) rc = upload(op->coef, cf.data(), cf.size() * sizeof(T), s);
  if (!rc) MF_HIP(hipStreamSynchronize(s));
  return rc;
}

static void count_work(mf_op *op) {
  const double s = op->precision == MF_F64 ? 8.0 : 4.0;
  const double nc = (double)op->ncells, nd = (double)op->ndofs;
  const int comps = op->ncomp;
  double fl = 0.0, by = 2.0 * nd * s + 4.0 * op->D * nc;
  if (op->cell_type == MF_CELL_HEX && (op->kind == MF_OP_ELASTICITY || op->kind == MF_OP_HYPERELASTIC)) {
    // per component, multiply-adds: x pass 2 q n^3, y pass 3 q^2 n^2, z pass 3 q^3 n and
    // the same backward (n = k+1, q points per direction); per point the Jacobian 36,
    // cofactors and det 50, gradients 54, stress 15, fluxes 54 and the weight 5 flops
    const double n = op->degree + 1, q = op->nq1d;
    const double fma = 3.0 * 2.0 * (2.0 * q * n * n * n + 3.0 * q * q * n * n + 3.0 * q * q * q * n);
    fl = nc * (2.0 * fma + q * q * q * 214.0);
    by += nc * 24.0 * s;
    if (op->kind == MF_OP_HYPERELASTIC) {
      // the forward passes again for u0, its push-forward (54) and F = I + grad u0 (3),
      // F^T F and dE (135), S and dS (30), grad u S + F dS (162) minus the linear stress
      // (15) per point; u0 read once
      fl += nc * (fma + q * q * q * 369.0);
      by += 3.0 * (double)op->nnodes * s;
    }
  } else if (op->cell_type == MF_CELL_HEX && op->nq1d != op->degree + 1) {
    // k+2 points on pencils (n = k+1 nodes, q points per direction), per component: the
    // rectangular even-odd passes n -> q over n^2, n q and q^2 pencils and back, plus,
    // with gradients, three collocation derivatives and their transposes over q^2 pencils
    // of length q (costed as in the k+1 count below); per point the k+1 kernel's
    // geometry and flux terms
    const int ni = op->degree + 1, nqi = op->nq1d;
    const double n = ni, q = nqi;
    const bool grad = op->kind != MF_OP_MASS, mass = op->kind == MF_OP_MASS || op->kind == MF_OP_HELMHOLTZ;
    // even-odd product of an no x nn matrix with reflection symmetry: the sums and
    // differences of the input, two half-size products per output pair (one middle
    // column when nn is odd), the pair itself, the middle row when no is odd
    auto rect = [](int nn, int no) {
      const int hi = nn / 2, ho = no / 2;
      return 2.0 * hi + ho * (4.0 * hi + 2.0 * (nn % 2) + 2.0) + (no % 2) * (2.0 * hi + 2.0 * (nn % 2));
    };
    const double pencil = q * q + 2.0 * q - (nqi % 2);
    const double contr = comps * ((n * n + n * q + q * q) * (rect(ni, nqi) + rect(nqi, ni)) +
                                  (grad ? 6.0 : 0.0) * q * q * pencil);
    const double geo = grad ? 39.0 : 24.0;
    const double pw = (grad ? 39.0 : 0.0) * comps + (mass ? 4.0 * comps : 0.0);
    fl = nc * (contr + q * q * q * (geo + pw));
    by += nc * 24.0 * s + (op->has_coef ? nc * 8.0 * s : 0.0);
  } else if (op->cell_type == MF_CELL_HEX) {
    const int ni = op->degree + 1;
    const double n = ni, q3 = n * n * n;
    const bool grad = op->kind != MF_OP_MASS, mass = op->kind == MF_OP_MASS || op->kind == MF_OP_HELMHOLTZ;
    // 1D contractions: 3 forward + 3 backward with B, plus 3 + 3 with the collocation
    // derivative when gradients are needed, each over n^2 pencils of length n. A pencil
    // costs 2 n^2 flops as a plain product (Q1) and, split into even and odd halves
    // (n >= 3), n^2 + 2n flops for even n and n^2 + 2n - 1 for odd n (multiply-adds
    // counted as two flops, as in the plain count).
    const double pencil = ni >= 3 ? n * n + 2.0 * n - (ni % 2) : 2.0 * n * n;
    const double contr = (grad ? 12.0 : 6.0) * n * n * pencil * comps;
    // per point: Jacobian 12, adjugate rows 18 (6 for the mass-only kernel), det 5,
    // weights/scale 4; per component: push-forward 18 + fluxes 21, mass term 4
    const double geo = grad ? 39.0 : 24.0;
    const double pw = (grad ? 39.0 : 0.0) * comps + (mass ? 4.0 * comps : 0.0);
    fl = nc * (contr + q3 * (geo + pw));
    // geometry: 24 stored values per cell, or (Q1 patch kernel in FP64) the FP64
    // coordinates of the vertices, once per vertex
    const bool xyz = op->patched && op->precision == MF_F64;
    by += (xyz ? 24.0 * (double)op->nnodes : nc * 24.0 * s) + (op->has_coef ? nc * 8.0 * s : 0.0);
  } else if (op->cell_type == MF_CELL_QUAD) {
    // sum factorisation in 2D, n = k+1 nodes and q points per direction; multiply-adds
    // per cell (two flops each): forward x pass q n^2 (twice with gradients), forward y
    // pass q^2 n per value or gradient component, backward passes the same in reverse;
    // per point: Jacobian and |det| w 14, coefficient 13, value 2, gradient push-forward
    // and flux 17
    // (per component; elasticity: two components, and its stress 10 flops per point)
    const double n = op->degree + 1, q = op->nq1d, C = comps;
    const bool val = op->kind == MF_OP_MASS || op->kind == MF_OP_HELMHOLTZ, grad = op->kind != MF_OP_MASS;
    const double g = grad ? 1.0 : 0.0, v = val ? 1.0 : 0.0;
    const double fma =
        C * (q * n * n * (1 + g) + q * q * n * (v + 2 * g) + q * q * n * (v + 2 * g) + q * n * n * (1 + g));
    const double pt = 14.0 + (op->has_coef ? 13.0 : 0.0) + 2.0 * v + 5.0 * g + 12.0 * g * C +
                      (op->kind == MF_OP_ELASTICITY ? 10.0 : 0.0);
    fl = nc * (2.0 * fma + q * q * pt);
    by += nc * 6.0 * s + (op->has_coef ? nc * 4.0 * s : 0.0);
  } else if (op->cell_type == MF_CELL_TET && op->ncomp == 1) {
    // scalar operators, dense tabulation, per point: value 2D and its test sum 2D;
    // reference gradient 6D, push-forward 18, the reference-direction flux 18 (and a
    // scale), test sum 6D; coefficient 8
    const double D = op->D, Q = op->nqp;
    const bool val = op->kind == MF_OP_MASS || op->kind == MF_OP_HELMHOLTZ, grad = op->kind != MF_OP_MASS;
    fl = nc * Q * ((val ? 4.0 * D + 3.0 : 0.0) + (grad ? 12.0 * D + 39.0 : 0.0) + (op->has_coef ? 8.0 : 0.0));
    by += nc * 10.0 * s + (op->has_coef ? nc * 4.0 * s : 0.0);
  } else if (op->cell_type == MF_CELL_TET) {
    const double D = op->D, Q = op->nqp;
    // per point per component: reference gradient 6D, its push-forward 18, stress 8,
    // P 20, test contraction 6D
    fl = nc * Q * 3.0 * (12.0 * D + 46.0);
    by += nc * 10.0 * s;
    if (op->kind == MF_OP_HYPERELASTIC) {
      // per point: the gradient of u0 (6D + 18 per component), F^T F and F^T dF (108),
      // E, S and dS (63), dF S + F dS (108), minus the linear stress it replaces (24)
      fl += nc * Q * (3.0 * (6.0 * D + 18.0) + 255.0);
      by += 3.0 * (double)op->nnodes * s;  // u0 read once
    }
  } else if (!(op->kind == MF_OP_MASS && op->degree == 1)) {
    // triangles of degree k: per point value 4D + 3, gradient 8D + 17, coefficient 6;
    // elasticity per component reference gradient 4D, push-forward and pull-back 12,
    // test sum 4D, plus the stress 9 and the weight
    const double D = op->D, Q = op->nqp;
    const bool val = op->kind == MF_OP_MASS || op->kind == MF_OP_HELMHOLTZ, grad = op->kind != MF_OP_MASS;
    if (op->kind == MF_OP_ELASTICITY)
      fl = nc * Q * (2.0 * (8.0 * D + 12.0) + 10.0);
    else
      fl = nc * Q * ((val ? 4.0 * D + 3.0 : 0.0) + (grad ? 8.0 * D + 17.0 : 0.0) + (op->has_coef ? 6.0 : 0.0));
    by += nc * 5.0 * s + (op->has_coef ? nc * 3.0 * s : 0.0);
  } else {
    fl = nc * 30.0;
    by += nc * 3.0 * s;
  }
  op->flops = fl;
  op->bytes = by;
}

// One launch of the cell kernel over internal cells [c0, c1). atomic: scatter with
// atomics (optionally only cells whose user index is in [ulo, uhi)); otherwise
// plain read-modify-write, which requires [c0, c1) to lie inside one colour.
// fused: x is the first-stage output of the user -> internal permutation, gathered
// through gmap (hex pencil kernel only).
template <typename T>
static int cell_launch(const mf_op *op, int64_t c0, int64_t c1, const T *x, T *y, bool atomic, const int32_t *filt,
                       int64_t ulo, int64_t uhi, hipStream_t s, bool fused = false, bool first = false) {
  if (op->cell_type == MF_CELL_HEX && (op->kind == MF_OP_ELASTICITY || op->kind == MF_OP_HYPERELASTIC)) {
    HexElasArgs<T> a{op->map.as<int32_t>(), op->geo.as<T>(), op->tab.as<T>(), x, y, c0, c1, filt, ulo, uhi,
                     (T)op->lam, (T)op->mu, fused ? op->gmap.as<int32_t>() : nullptr};
    if (op->kind == MF_OP_HYPERELASTIC) {
      a.u0 = op->u0.as<T>();
      a.u0map = op->u0map.ptr ? op->u0map.as<int32_t>() : nullptr;
    }
    return launch_hex_elasticity<T>(op->degree, op->nq1d, a, atomic, s);
  } else if (op->cell_type == MF_CELL_HEX && op->nq1d != op->degree + 1) {
    HexQArgs<T> a{op->map.as<int32_t>(), op->geo.as<T>(),
                  op->has_coef ? op->coef.as<T>() : nullptr, x, y, c0, c1, filt, ulo, uhi,
                  fused ? op->gmap.as<int32_t>() : nullptr, op->ncomp};
    return launch_hex_kq<T>(op->degree, op->nq1d, op->kind, a, atomic, s);
  } else if (op->cell_type == MF_CELL_HEX) {
    // the coloured degree-1 kernel reads the block-interleaved copies
    const bool q1 = op->degree == 1 && !atomic;
    if (fused && q1) return fail(MF_EINVAL, "internal: fused gather with the coloured Q1 kernel");
    HexArgs<T> a{(q1 ? op->q1map : op->map).as<int32_t>(), (q1 ? op->q1geo : op->geo).as<T>(),
                 op->has_coef ? (q1 ? op->q1coef : op->coef).as<T>() : nullptr, x, y, c0, c1, op->ncomp, filt, ulo,
                 uhi, fused ? op->gmap.as<int32_t>() : nullptr, first ? op->first_lo.as<int32_t>() : nullptr};
    return launch_hex_apply<T>(op->degree + 1, op->kind, a, atomic, s);
  } else if (op->cell_type == MF_CELL_QUAD) {
    QuadArgs<T> a{op->map.as<int32_t>(), op->geo.as<T>(), op->has_coef ? op->coef.as<T>() : nullptr,
                  op->tab.as<T>(), x, y, c0, c1, filt, ulo, uhi, (T)op->lam, (T)op->mu};
    return launch_quad<T>(op->degree, op->nq1d, op->kind, a, atomic, s);
  } else if (op->cell_type == MF_CELL_TET) {
    TetArgs<T> a{op->map.as<int32_t>(), op->geo.as<T>(), op->tab.as<T>(), x, y, c0, c1, (T)op->lam, (T)op->mu,
                 filt, ulo, uhi, op->u0.as<T>(), op->u0map.as<int32_t>(),
                 op->has_coef ? op->coef.as<T>() : nullptr};
    if (op->ncomp == 1) return launch_tet_scalar<T>(op->degree, op->nqp, op->kind, a, atomic, s);
    return launch_tet_elasticity<T>(op->degree, op->nqp, a, atomic, s);
  }
  if (!(op->kind == MF_OP_MASS && op->degree == 1)) {
    TetArgs<T> a{op->map.as<int32_t>(), op->geo.as<T>(), op->tab.as<T>(), x, y, c0, c1, (T)op->lam, (T)op->mu,
                 filt, ulo, uhi, nullptr, nullptr, op->has_coef ? op->coef.as<T>() : nullptr};
    if (op->ncomp == 1) return launch_tri_scalar_mfma<T>(op->degree, op->nqp, op->kind, a, atomic, s);
    return launch_tri_elasticity_mfma<T>(op->degree, op->nqp, a, atomic, s);
  }
  TriArgs<T> a{op->map.as<int32_t>(), op->geo.as<T>(), x, y, c0, c1, filt, ulo, uhi};
  return launch_tri_mass<T>(a, atomic, s);
}

// y (+)= A_[c0,c1) x in internal numbering; [c0, c1) is a range of user cells.
template <typename T> static int op_apply_t(const mf_op *op, int64_t c0, int64_t c1, const T *x, T *y, bool acc,
                                            bool bc, hipStream_t s, bool fused = false) {
  int rc = MF_OK;
  // A full colour-by-colour overwrite apply with first-touch thresholds writes every
  // free node and clears nothing; constrained rows are then written by the copy below.
  const bool first = !acc && c0 == 0 && c1 == op->ncells && op->coloured && !op->patched && op->first_ok &&
                     (op->n_bc_dofs == 0 || bc);
  // the simplex patch scatter writes every free node of a full apply once
  const bool self_written =
      !acc && c0 == 0 && c1 == op->ncells && (op->spatched || op->hpatched) && (op->n_bc_dofs == 0 || bc);
  if (!acc && !first && !self_written) {
    rc = launch_fill<T>(y, T(0), op->ndofs, s);
    if (rc) return rc;
  }
  if (c0 == 0 && c1 == op->ncells) {
    if (op->hpatched) {
      HexArgs<T> a{op->hp_map.as<int32_t>(), op->hp_geo.as<T>(), op->has_coef ? op->hp_coef.as<T>() : nullptr, x, y,
                   0, (int64_t)op->hp_npatch * hex_cells_per_patch(op->degree + 1), op->ncomp, nullptr, 0, 0,
                   fused ? op->hp_gmap.as<int32_t>() : nullptr, nullptr, op->hp_lmap.as<uint16_t>(),
                   op->hp_nptr.as<int32_t>(), op->hp_out.as<int32_t>(), op->sp_sbuf.as<T>(), acc ? 1 : 0};
      rc = launch_hex_cell_patches<T>(op->degree + 1, op->kind, a, op->hp_npatch, s);
      if (!rc)
        rc = launch_simplex_shared_reduce<T>(op->sp_sptr.as<int32_t>(), op->sp_snode.as<int32_t>(),
                                             op->sp_sbuf.as<T>(), y, op->sp_nshared, op->ncomp, acc, s);
    } else if (op->spatched) {
      SimplexPatchArgs<T> pa{op->sp_map.as<int32_t>(), op->sp_geo.as<T>(), op->sp_lmap.as<uint16_t>(),
                             op->sp_nptr.as<int32_t>(), op->sp_out.as<int32_t>(), op->sp_sbuf.as<T>(),
                             op->sp_npatch, op->sp_cap, op->sp_nmax, acc ? 1 : 0};
      if (op->cell_type == MF_CELL_TRI && op->kind == MF_OP_MASS && op->degree == 1) {
        rc = launch_tri_mass_patches<T>(x, y, pa, s);
      } else if (op->cell_type == MF_CELL_TRI) {
        TetArgs<T> a{op->map.as<int32_t>(), op->geo.as<T>(), op->tab.as<T>(), x, y, 0, op->ncells, (T)op->lam,
                     (T)op->mu, nullptr, 0, 0, nullptr, nullptr, nullptr};
        rc = op->ncomp == 1 ? launch_tri_scalar_patches<T>(op->degree, op->nqp, op->kind, a, pa, s)
                            : launch_tri_elasticity_patches<T>(op->degree, op->nqp, a, pa, s);
      } else {
        TetArgs<T> a{op->map.as<int32_t>(), op->geo.as<T>(), op->tab.as<T>(), x, y, 0, op->ncells, (T)op->lam,
                     (T)op->mu, nullptr, 0, 0, nullptr, nullptr, nullptr};
        rc = op->ncomp == 1 ? launch_tet_scalar_patches<T>(op->degree, op->nqp, op->kind, a, pa, s)
                            : launch_tet_elasticity_patches<T>(op->degree, op->nqp, a, pa, s);
      }
      if (!rc)
        rc = launch_simplex_shared_reduce<T>(op->sp_sptr.as<int32_t>(), op->sp_snode.as<int32_t>(),
                                             op->sp_sbuf.as<T>(), y, op->sp_nshared, op->ncomp, acc, s);
    } else if (op->patched) {
      HexPatchArgs<T> a{op->pt_nptr.as<int32_t>(), op->pt_nodes.as<int32_t>(),
                        fused ? op->pt_gnodes.as<int32_t>() : nullptr, op->pt_lmap.as<uint16_t>(),
                        op->pt_xyz.as<double>(), op->pt_geo.as<T>(), op->has_coef ? op->pt_coef.as<T>() : nullptr,
                        x, y, op->npatch,
                        op->pt_max_nodes, op->ncomp, op->pt_cap};
      rc = launch_hex_patches<T>(op->degree + 1, op->kind, a, s);
    } else if (op->coloured) {
      // one launch per colour: cells of a colour share no node, so no atomics
      for (size_t c = 0; c + 1 < op->colour_ptr.size() && !rc; c++)
        rc = cell_launch<T>(op, op->colour_ptr[c], op->colour_ptr[c + 1], x, y, false, nullptr, 0, 0, s, fused,
                            first);
    } else {
      rc = cell_launch<T>(op, 0, op->ncells, x, y, true, nullptr, 0, 0, s, fused);
    }
  } else if (c1 > c0) {
    rc = cell_launch<T>(op, 0, op->ncells, x, y, true, op->cell_user.as<int32_t>(), c0, c1, s, fused);
  }
  if (rc) return rc;
  if (bc && op->n_bc_dofs) rc = launch_copy_constrained<T>(op->bc_dofs.as<int32_t>(), op->n_bc_dofs, x, y, s);
  return rc;
}

// Coloured launches avoid device-scope float atomics but cost one launch per
// colour with 1/ncolours of the cells each. Measured on MI355X: for 32^3 hex the
// single atomic launch is faster for scalar operators and the coloured launches
// win for 3-component operators from Q2 up (three atomics per node otherwise). For
// scalar operators they break even at about 64^3 cells (Q1: 51 against 55 us, Q2:
// 142 against 127 us in FP64) and win above (Q1 at 128^3: 238 against 346 us, Q2 at
// 96^3: 364 against 458 us). For P2/P3 tet elasticity on 48^3 x 6 cells (31
// colours) the coloured launches are 1.1x (FP64) to 3.4x (FP32) faster. Quads (4
// colours): the two scatters are within a few percent for the one-component operators
// (atomic ahead at 256^2 cells), and the coloured launches win for elasticity (Q2 at
// 1024^2 cells: 390 against 527 us in FP64, 251 against 379 us in FP32).
// Triangles (lane-per-cell kernel): elasticity P1-P3 at 1024^2 x 2 cells 2.2-5x faster
// coloured (P2 FP64 943 -> 323 us), and mostly faster at 256^2 x 2; the one-component
// operators lose coloured at 256^2 x 2 cells (P2 Helmholtz 29 against 51 us) and win at
// 1024^2 x 2 (366 -> 173 us), so they switch at 2^20 cells (between the two measured
// sizes). The closed-form P1 mass keeps atomics (not measured).
static bool default_coloured(const mf_op *op) {
  if (op->ncells < 4096) return false;
  if (op->cell_type == MF_CELL_QUAD) return op->ncomp == 2;
  if (op->cell_type == MF_CELL_TRI) {
    if (op->kind == MF_OP_MASS && op->degree == 1) return false;
    return op->ncomp == 2 || op->ncells >= (1 << 20);
  }
  if (op->cell_type == MF_CELL_HEX) {
    // the hyperelastic tangent spends long enough per cell at Q6 (FP64 also Q5) that one
    // atomic launch beats 8 colour launches (32^3: FP64 Q5 610 against 632 us, Q6 1405
    // against 1467; FP32 Q6 665 against 704, but Q5 428 against 396)
    if (op->kind == MF_OP_HYPERELASTIC && op->degree >= (op->precision == MF_F64 ? 5 : 6)) return false;
    if (op->ncomp == 3 && op->degree >= 2) return true;
    return op->ncells >= (op->degree == 1 ? (1 << 19) : (1 << 18));
  }
  // tets of degree >= 4 (MFMA, 64-1331 points per cell) keep atomics: at 24^3 x 6 a
  // colour's 2,800 cells fill too little of the chip (FP64 P4 Laplacian 711 against
  // 146 us, P6 3700 against 677 us; P6 elasticity 7385 against 3952 us)
  return op->cell_type == MF_CELL_TET && op->degree >= 2 && op->degree <= 3;
}

template <typename T> static int op_diag_t(const mf_op *op, T *d, hipStream_t s) {
  if (op->kind == MF_OP_HYPERELASTIC) return fail(MF_EUNSUPPORTED, "diagonal: not built for HYPERELASTIC");
  int rc = launch_fill<T>(d, T(0), op->ndofs, s);
  if (rc) return rc;
  if (element_diag_supported(op)) {
    rc = element_diag<T>(op, d, s);
  } else if (op->cell_type == MF_CELL_HEX) {
    HexArgs<T> a{op->map.as<int32_t>(), op->geo.as<T>(), op->has_coef ? op->coef.as<T>() : nullptr, nullptr, d, 0,
                 op->ncells, op->ncomp, nullptr, 0, 0};
    rc = launch_hex_diag<T>(op->degree + 1, op->kind, a, s);
  } else if (op->cell_type == MF_CELL_QUAD) {
    QuadArgs<T> a{op->map.as<int32_t>(), op->geo.as<T>(), op->has_coef ? op->coef.as<T>() : nullptr,
                  op->tab.as<T>(), nullptr, d, 0, op->ncells, nullptr, 0, 0, (T)op->lam, (T)op->mu};
    rc = launch_quad<T>(op->degree, op->nq1d, op->kind, a, true, s, true);
  } else if (op->cell_type == MF_CELL_TET) {
    TetArgs<T> a{op->map.as<int32_t>(), op->geo.as<T>(), op->tab.as<T>(), nullptr, d, 0, op->ncells, (T)op->lam,
                 (T)op->mu, nullptr, 0, 0};
    rc = launch_tet_elasticity_diag<T>(op->degree, op->nqp, a, s);
  } else {
    TriArgs<T> a{op->map.as<int32_t>(), op->geo.as<T>(), nullptr, d, 0, op->ncells, nullptr, 0, 0};
    rc = launch_tri_mass_diag<T>(a, s);
  }
  if (rc) return rc;
  if (op->n_bc_dofs) rc = launch_set_constrained<T>(op->bc_dofs.as<int32_t>(), op->n_bc_dofs, T(1), d, s);
  return rc;
}

}  // namespace mf

extern "C" {

int mf_op_create(const mf_space *sp, int kind, int precision, int nq1d, const mf_op_params *params, void *stream,
                 mf_op **out) {
  if (!sp || !out) return fail(MF_EINVAL, "mf_op_create: null argument");
  if (precision != MF_F64 && precision != MF_F32) return fail(MF_EINVAL, "mf_op_create: precision");
  if (kind < MF_OP_MASS || kind > MF_OP_HYPERELASTIC) return fail(MF_EINVAL, "mf_op_create: operator kind");
  mf_op_params defaults{nullptr, 1.0, 0.5, nullptr, MF_SCATTER_AUTO, nullptr};
  const mf_op_params *pr = params ? params : &defaults;
  hipStream_t s = (hipStream_t)stream;
  const int ct = sp->cell_type;
  // supported combinations
  bool ok = false;
  if (ct == MF_CELL_HEX)
    ok = (kind == MF_OP_LAPLACIAN) ? (sp->ncomp == 1 || sp->ncomp == 3)
         : (kind == MF_OP_ELASTICITY || kind == MF_OP_HYPERELASTIC) ? sp->ncomp == 3
                                    : (kind <= MF_OP_POISSON && sp->ncomp == 1);
  else if (ct == MF_CELL_QUAD)
    ok = (kind <= MF_OP_POISSON && sp->ncomp == 1) || (kind == MF_OP_ELASTICITY && sp->ncomp == 2);
  else if (ct == MF_CELL_TET)
    ok = ((kind == MF_OP_ELASTICITY || kind == MF_OP_HYPERELASTIC) && sp->ncomp == 3) ||
         (kind <= MF_OP_POISSON && sp->ncomp == 1);
  else
    ok = (kind <= MF_OP_POISSON && sp->ncomp == 1) || (kind == MF_OP_ELASTICITY && sp->ncomp == 2);
  if (!ok) return fail(MF_EUNSUPPORTED, "mf_op_create: operator / cell / ncomp combination not built");
  if (kind == MF_OP_HYPERELASTIC && !pr->u0) return fail(MF_EINVAL, "HYPERELASTIC needs u0 (linearisation point)");
  if (kind == MF_OP_POISSON && !pr->vertex_coef) return fail(MF_EINVAL, "POISSON needs vertex_coef (kappa)");
  if (pr->scatter < MF_SCATTER_AUTO || pr->scatter > MF_SCATTER_PATCH)
    return fail(MF_EINVAL, "mf_op_create: unknown scatter mode");
  std::unique_ptr<mf_op> op(new (std::nothrow) mf_op);
  if (!op) return fail(MF_ENOMEM, "mf_op_create: host allocation");
  op->cell_type = ct;
  op->kind = kind;
  op->precision = precision;
  op->degree = sp->degree;
  op->ncomp = sp->ncomp;
  op->D = sp->D;
  op->ncells = sp->ncells;
  op->nnodes = sp->nnodes;
  op->ndofs = sp->nnodes * sp->ncomp;
  op->lam = pr->lambda;
  op->mu = pr->mu;
  op->has_coef = pr->vertex_coef != nullptr && (kind == MF_OP_MASS || kind == MF_OP_POISSON);
  const bool tensor = ct == MF_CELL_HEX || ct == MF_CELL_QUAD;
  op->nq1d = tensor ? (nq1d > 0 ? nq1d : sp->degree + 1) : 0;
  if (ct == MF_CELL_HEX) op->nqp = op->nq1d * op->nq1d * op->nq1d;
  if (ct == MF_CELL_HEX && (kind == MF_OP_ELASTICITY || kind == MF_OP_HYPERELASTIC) &&
      op->nq1d != sp->degree + 1 && op->nq1d != sp->degree + 2)
    return fail(MF_EUNSUPPORTED, "hex elasticity: nq1d must be k+1 or k+2");
  if (ct == MF_CELL_QUAD) {
    // one lane per point, and every dof needs a lane
    if (op->nq1d != sp->degree + 1 && op->nq1d != sp->degree + 2)
      return fail(MF_EUNSUPPORTED, "quad: nq1d must be k+1 or k+2");
    op->nqp = op->nq1d * op->nq1d;
  }

  // maps: constrained nodes are stored as -1 (gathered as 0, never scattered)
  const int64_t nc = sp->ncells;
  const int D = sp->D;
  std::vector<int32_t> m;
  // (internal node ids; the Dirichlet mask is given per user node)
  auto flag = [&](int32_t inode) { return (pr->dirichlet && pr->dirichlet[sp->user_of_int[inode]]) ? -1 : inode; };
  const std::vector<int32_t> &c2n = sp->cell2node_int;
  // the lane-per-cell simplex kernels read AoSoA maps (all but the closed-form P1
  // triangle mass)
  if (ct == MF_CELL_TET || (ct == MF_CELL_TRI && !(kind == MF_OP_MASS && sp->degree == 1))) {
    const int64_t nb = (nc + 63) / 64;
    m.assign((size_t)nb * D * 64, -1);
    for (int64_t K = 0; K < nc; K++)
      for (int i = 0; i < D; i++) m[((K / 64) * D + i) * 64 + K % 64] = flag(c2n[K * D + i]);
  } else {
    m.resize((size_t)nc * D);
    for (int64_t i = 0; i < nc * D; i++) m[i] = flag(c2n[i]);
  }
  int rc = upload(op->map, m.data(), m.size() * sizeof(int32_t), s);
  if (rc) return rc;
  std::vector<int32_t> m2;
  if (ct == MF_CELL_HEX && op->degree == 1) {
    const int64_t nb = (nc + 63) / 64;
    m2.assign((size_t)nb * 8 * 64, -1);
    for (int64_t K = 0; K < nc; K++)
      for (int i = 0; i < 8; i++) m2[((K / 64) * 8 + i) * 64 + K % 64] = m[K * 8 + i];
    rc = upload(op->q1map, m2.data(), m2.size() * sizeof(int32_t), s);
    if (rc) return rc;
  }
  // constrained dofs in user numbering (identity rows of the assembled matrix)
  if (pr->dirichlet)
    for (int64_t u = 0; u < sp->nnodes; u++)
      if (pr->dirichlet[u])
        for (int c = 0; c < sp->ncomp; c++) op->h_bc_user.push_back((int32_t)(u * sp->ncomp + c));
  if (pr->dirichlet) {
    std::vector<int32_t> bd;
    for (int64_t n = 0; n < sp->nnodes; n++)
      if (pr->dirichlet[sp->user_of_int[n]])
        for (int c = 0; c < sp->ncomp; c++) bd.push_back((int32_t)(n * sp->ncomp + c));
    op->n_bc_dofs = (int64_t)bd.size();
    rc = upload(op->bc_dofs, bd.data(), bd.size() * sizeof(int32_t), s);
    if (rc) return rc;
  }
  op->identity = sp->identity;
  op->numbering_id = sp->numbering_id;
  op->colour_ptr = sp->colour_ptr;
  rc = upload(op->cell_user, sp->cell_user_of_int.data(), sp->cell_user_of_int.size() * sizeof(int32_t), s);
  if (rc) return rc;
  op->coloured = pr->scatter == MF_SCATTER_COLOURED || (pr->scatter == MF_SCATTER_AUTO && default_coloured(op.get()));
  // P2/P3 tet elasticity, one-component tet operators and the triangle operators
  // (the MFMA kernels), the P1 triangle mass: patch scatter on request, and by default
  // from 2^15 cells (triangles up to degree 4: at 1024^2 x 2 cells, FP64, the patches took
  // P2 Helmholtz from 174 (coloured) to 115 us, P3 Laplacian from 306 to 191 us, P3
  // elasticity from 527 to 329 us; at degree 6 atomics ran the Helmholtz operator faster
  // in FP64, 395 against 447 us, and slower in FP32, 460 against 267 us, and the coloured
  // launches ran elasticity faster, 611 / 322 against 788 / 518 us)
  const bool tet_patchable = (ct == MF_CELL_TET && ((kind == MF_OP_ELASTICITY && sp->degree >= 2 && sp->degree <= 3) ||
                                                    (kind <= MF_OP_POISSON && sp->ncomp == 1))) ||
                             (ct == MF_CELL_TRI && ((kind <= MF_OP_POISSON && sp->ncomp == 1) || kind == MF_OP_ELASTICITY));
  // hex degrees 2-6 (the pencil kernel): patch scatter on request, and by default for
  // degrees 2-4 below 2^17 cells (Q2: 2^20). A patch is one workgroup's cells (7, 4 and
  // 2 cells for k = 2..4, 3 and 5 for k = 5, 6); at 32^3 it beat the coloured and atomic
  // scatters for k <= 4 (FP64 vector Laplacian Q2 63 -> 38 us, Q3 84 -> 65 us, Q4 157 ->
  // 138 us) and lost for k = 5, 6 (Q5 242 -> 309 us, Q6 390 -> 471 us), where most of a
  // patch's nodes are shared; on larger meshes the coloured launches win (FP64
  // Helmholtz at 64^3: Q2 98 against 125 us still for the patches, Q3 228 against 188,
  // Q4 496 against 421; at 128^3 Q2 874 against 773 us).
  const bool hex_patchable = ct == MF_CELL_HEX && kind <= MF_OP_POISSON && sp->degree >= 2 && sp->degree <= 6 &&
                             op->nq1d == sp->degree + 1;
  if (pr->scatter == MF_SCATTER_PATCH && tet_patchable) {
    op->spatched = true;
  } else if (pr->scatter == MF_SCATTER_AUTO && tet_patchable &&
             !(ct == MF_CELL_TRI && sp->degree >= 5 && (precision == MF_F64 || kind == MF_OP_ELASTICITY)) &&
             !(ct == MF_CELL_TET && sp->degree >= 4 && (precision == MF_F64 || sp->degree == 6)) &&
             nc >= (1 << 15)) {
    op->spatched = true;
  } else if (hex_patchable &&
             (pr->scatter == MF_SCATTER_PATCH ||
              (pr->scatter == MF_SCATTER_AUTO && nc < (sp->degree == 2 ? (1 << 20) : (1 << 17)) &&
               // measured at 32^3: patches win up to Q4 and, for one component, at Q5-Q6 in
               // FP32 (10-30 % over atomics); FP64 Q5 gains warm (3-10 %) but loses with cold
               // caches (125 against 96 us), FP64 Q6 does not gain
               (sp->degree <= 4 || (sp->ncomp == 1 && precision == MF_F32))))) {
    op->hpatched = true;
  } else if (pr->scatter == MF_SCATTER_PATCH) {
    if (ct != MF_CELL_HEX || op->degree != 1 || kind > MF_OP_POISSON || op->nq1d != 2)
      return fail(MF_EUNSUPPORTED, "mf_op_create: the patch scatter is built for the hex scalar operators, P2/P3 "
                                   "tet elasticity, one-component tet operators and the triangle operators");
    op->patched = true;
  } else if (pr->scatter == MF_SCATTER_AUTO && ct == MF_CELL_HEX && op->degree == 1 && nc >= (1 << 15) &&
             kind <= MF_OP_POISSON && op->nq1d == 2) {
    op->patched = true;
  }
  if (op->patched || op->spatched || op->hpatched) op->coloured = false;
  if (ct == MF_CELL_HEX && op->degree >= 2 && op->coloured && kind <= MF_OP_POISSON &&
      op->nq1d == op->degree + 1) {
    // First-touch thresholds for overwrite applies (HexArgs::first). Colours are
    // launched in internal cell order, so a node's first toucher is the first cell in
    // that order that lists it. The threshold form needs every later toucher to see the
    // node below its cell's threshold, and every free node needs a first toucher.
    std::vector<int32_t> lo((size_t)nc, INT32_MAX);
    std::vector<uint8_t> seen((size_t)sp->nnodes, 0);
    bool ok = true;
    for (int64_t K = 0; K < nc && ok; K++) {
      int32_t mn = INT32_MAX, old = -1;
      for (int i = 0; i < D; i++) {
        const int32_t n = m[K * D + i];
        if (n < 0) continue;
        if (!seen[n]) {
          seen[n] = 1;
          mn = std::min(mn, n);
        } else {
          old = std::max(old, n);
        }
      }
      lo[K] = mn;
      ok = old < mn;
    }
    for (int64_t n = 0; n < sp->nnodes && ok; n++) ok = seen[n] || flag((int32_t)n) < 0;
    if (ok) {
      rc = upload(op->first_lo, lo.data(), lo.size() * sizeof(int32_t), s);
      if (rc) return rc;
      MF_HIP(hipStreamSynchronize(s));
      op->first_ok = true;
    }
  }
  std::vector<int32_t> to_pos2, gm;  // second-stage positions of the user -> internal permutation
  if (!op->identity) {
    rc = upload(op->perm, sp->user_of_int.data(), sp->user_of_int.size() * sizeof(int32_t), s);
    if (!rc) rc = upload(op->iperm, sp->int_of_user.data(), sp->int_of_user.size() * sizeof(int32_t), s);
    const size_t vb = (size_t)op->ndofs * (precision == MF_F64 ? 8 : 4);
    if (!rc) rc = op->wx.alloc(vb);
    if (!rc) rc = op->wy.alloc(vb);
    if (!rc) rc = op->wt.alloc(vb);
    if (!rc) {
      // user -> internal: x_int[i] = x_user[user_of_int[i]]; back: y_user[u] = y_int[int_of_user[u]]
      std::vector<int32_t> p1, q1, q2;
      permute2_positions(sp->user_of_int.data(), sp->nnodes, p1, to_pos2);
      permute2_positions(sp->int_of_user.data(), sp->nnodes, q1, q2);
      rc = upload(op->to1, p1.data(), p1.size() * 4, s);
      if (!rc) rc = upload(op->to2, to_pos2.data(), to_pos2.size() * 4, s);
      if (!rc) rc = upload(op->from1, q1.data(), q1.size() * 4, s);
      if (!rc) rc = upload(op->from2, q2.data(), q2.size() * 4, s);
      if (!rc && ct == MF_CELL_HEX) {
        // x_int[i] sits at to_pos2[i] after the first stage: the map composed with it
        gm.resize(m.size());
        for (size_t i = 0; i < m.size(); i++) gm[i] = m[i] >= 0 ? to_pos2[m[i]] : m[i];
        rc = upload(op->gmap, gm.data(), gm.size() * 4, s);
        op->fused_gather = true;
      }
      if (!rc) MF_HIP(hipStreamSynchronize(s));  // the host vectors go out of scope
    }
    if (rc) return rc;
  }
  if (ct == MF_CELL_HEX) {
    rc = precision == MF_F64 ? setup_hex<double>(op.get(), sp, pr, m, to_pos2, s)
                             : setup_hex<float>(op.get(), sp, pr, m, to_pos2, s);
    if (!rc && (kind == MF_OP_ELASTICITY || kind == MF_OP_HYPERELASTIC))
      rc = precision == MF_F64 ? upload_tensor_tables<double>(op.get(), s) : upload_tensor_tables<float>(op.get(), s);
  }
  else if (ct == MF_CELL_QUAD)
    rc = precision == MF_F64 ? setup_quad<double>(op.get(), sp, pr, s) : setup_quad<float>(op.get(), sp, pr, s);
  else if (ct == MF_CELL_TET)
    rc = precision == MF_F64 ? setup_tet<double>(op.get(), sp, pr, m, s) : setup_tet<float>(op.get(), sp, pr, m, s);
  else
    rc = precision == MF_F64 ? setup_tri<double>(op.get(), sp, pr, m, s) : setup_tri<float>(op.get(), sp, pr, m, s);
  if (rc) return rc;
  MF_HIP(hipStreamSynchronize(s));
  count_work(op.get());
  *out = op.release();
  return MF_OK;
}

void mf_op_destroy(mf_op *op) {
  if (!op) return;
  (void)hipDeviceSynchronize();
  delete op;
}

}  // extern "C"

namespace mf {

// User-numbering wrappers: permute x into the internal numbering, run the
// internal-numbering kernels on the workspaces, permute the result back.
template <typename T>
static int user_apply(const mf_op *op, int64_t c0, int64_t c1, const T *x, T *y, bool acc, bool bc, hipStream_t s) {
  if (op->identity) return op_apply_t<T>(op, c0, c1, x, y, acc, bc, s);
  T *wx = op->wx.as<T>(), *wy = op->wy.as<T>(), *wt = op->wt.as<T>();
  int rc = MF_OK;
  // The kernels can gather x straight from the first stage of the permutation (the
  // composed map gmap), skipping its second stage, when no constrained rows need x in
  // internal numbering and the kernel is one that takes gmap.
  const bool fused = op->fused_gather && !(bc && op->n_bc_dofs) && !(op->degree == 1 && op->coloured);
  if (fused) {
    rc = launch_permute_stage1<T>(op->to1.as<int32_t>(), op->nnodes, op->ncomp, x, wt, s);
    if (!rc) rc = op_apply_t<T>(op, c0, c1, wt, wy, false, bc, s, true);
  } else {
    rc = launch_permute2<T>(op->to1.as<int32_t>(), op->to2.as<int32_t>(), op->nnodes, op->ncomp, x, wt, wx, false, s);
    if (!rc) rc = op_apply_t<T>(op, c0, c1, wx, wy, false, bc, s);
  }
  if (!rc)
    rc = launch_permute2<T>(op->from1.as<int32_t>(), op->from2.as<int32_t>(), op->nnodes, op->ncomp, wy, wt, y, acc,
                            s);
  return rc;
}

template <typename T> static int user_diag(const mf_op *op, T *d, hipStream_t s) {
  if (op->identity) return op_diag_t<T>(op, d, s);
  int rc = op_diag_t<T>(op, op->wy.as<T>(), s);
  if (!rc)
    rc = launch_from_internal_gather<T>(op->iperm.as<int32_t>(), op->nnodes, op->ncomp, op->wy.as<T>(), d, false, s);
  return rc;
}

int op_apply_internal(const mf_op *op, const void *x, void *y, hipStream_t s) {
  return op->precision == MF_F64
             ? op_apply_t<double>(op, 0, op->ncells, (const double *)x, (double *)y, false, true, s)
             : op_apply_t<float>(op, 0, op->ncells, (const float *)x, (float *)y, false, true, s);
}

int op_apply_internal_acc(const mf_op *op, const void *x, void *y, hipStream_t s) {
  return op->precision == MF_F64
             ? op_apply_t<double>(op, 0, op->ncells, (const double *)x, (double *)y, true, true, s)
             : op_apply_t<float>(op, 0, op->ncells, (const float *)x, (float *)y, true, true, s);
}

int op_diagonal_internal(const mf_op *op, void *d, hipStream_t s) {
  return op->precision == MF_F64 ? op_diag_t<double>(op, (double *)d, s) : op_diag_t<float>(op, (float *)d, s);
}

}  // namespace mf

extern "C" {

int mf_op_apply_range(const mf_op *op, int64_t start, int64_t end, const void *x, void *y, int accumulate,
                      void *stream) {
  if (!op || !x || !y) return fail(MF_EINVAL, "mf_op_apply_range: null argument");
  if (start < 0 || end > op->ncells || start > end) return fail(MF_EINVAL, "mf_op_apply_range: bad cell range");
  if (x == y) return fail(MF_EINVAL, "mf_op_apply_range: x and y alias");
  hipStream_t s = (hipStream_t)stream;
  return op->precision == MF_F64
             ? user_apply<double>(op, start, end, (const double *)x, (double *)y, accumulate != 0, false, s)
             : user_apply<float>(op, start, end, (const float *)x, (float *)y, accumulate != 0, false, s);
}

int mf_op_apply(const mf_op *op, const void *x, void *y, void *stream) {
  if (!op || !x || !y) return fail(MF_EINVAL, "mf_op_apply: null argument");
  if (x == y) return fail(MF_EINVAL, "mf_op_apply: x and y alias");
  hipStream_t s = (hipStream_t)stream;
  return op->precision == MF_F64
             ? user_apply<double>(op, 0, op->ncells, (const double *)x, (double *)y, false, true, s)
             : user_apply<float>(op, 0, op->ncells, (const float *)x, (float *)y, false, true, s);
}

int mf_op_apply_internal(const mf_op *op, const void *x, void *y, void *stream) {
  if (!op || !x || !y) return fail(MF_EINVAL, "mf_op_apply_internal: null argument");
  if (x == y) return fail(MF_EINVAL, "mf_op_apply_internal: x and y alias");
  return op_apply_internal(op, x, y, (hipStream_t)stream);
}

int mf_op_apply_range_internal(const mf_op *op, int64_t start, int64_t end, const void *x, void *y, int accumulate,
                               void *stream) {
  if (!op || !x || !y) return fail(MF_EINVAL, "mf_op_apply_range_internal: null argument");
  if (start < 0 || end > op->ncells || start > end) return fail(MF_EINVAL, "mf_op_apply_range_internal: bad range");
  if (x == y) return fail(MF_EINVAL, "mf_op_apply_range_internal: x and y alias");
  hipStream_t s = (hipStream_t)stream;
  return op->precision == MF_F64
             ? op_apply_t<double>(op, start, end, (const double *)x, (double *)y, accumulate != 0, false, s)
             : op_apply_t<float>(op, start, end, (const float *)x, (float *)y, accumulate != 0, false, s);
}

int mf_op_diagonal(const mf_op *op, void *d, void *stream) {
  if (!op || !d) return fail(MF_EINVAL, "mf_op_diagonal: null argument");
  hipStream_t s = (hipStream_t)stream;
  return op->precision == MF_F64 ? user_diag<double>(op, (double *)d, s) : user_diag<float>(op, (float *)d, s);
}

int mf_op_get_info(const mf_op *op, mf_op_info *info) {
  if (!op || !info) return fail(MF_EINVAL, "mf_op_get_info: null argument");
  info->ncells = op->ncells;
  info->nnodes = op->nnodes;
  info->ndofs = op->ndofs;
  info->cell_type = op->cell_type;
  info->kind = op->kind;
  info->precision = op->precision;
  info->degree = op->degree;
  info->ncomp = op->ncomp;
  info->nq1d = op->nq1d;
  info->nqp = op->nqp;
  info->dofs_per_cell = op->D;
  info->flops_per_apply = op->flops;
  info->bytes_per_apply = op->bytes;
  info->ncolours = (int)op->colour_ptr.size() - 1;
  info->cell_launches = op->coloured ? info->ncolours : 1;
  info->clears_output = (op->first_ok || op->spatched || op->hpatched) ? 0 : 1;
  info->scatter = (op->patched || op->spatched || op->hpatched) ? MF_SCATTER_PATCH
                  : op->coloured                                  ? MF_SCATTER_COLOURED
                                                                  : MF_SCATTER_ATOMIC;
  return MF_OK;
}

}  // extern "C"
