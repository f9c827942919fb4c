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
// 1D Gauss-Legendre rule on [0,1].
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w);
// k+1 Gauss-Lobatto-Legendre points on [0,1].
std::vector<double> gll_points(int k);
// Lagrange basis on `nodes` evaluated at `pts`: V[q*n+i], dV[q*n+i].
void lagrange_eval(const std::vector<double> &nodes, const std::vector<double> &pts,
                   std::vector<double> &V, std::vector<double> &dV);
// Simplex quadrature of the given exact degree on the reference tet: points (x,y,z) and weights
// (summing to 1/6). Returns false if no rule of that degree is built in.
bool tet_rule(int degree, std::vector<double> &pts, std::vector<double> &w);
// P_k Lagrange basis on the reference tet at pts: phi[q*D+i], dphi[(q*D+i)*3+d].
void tet_lagrange(int k, const std::vector<double> &pts, std::vector<double> &phi,
                  std::vector<double> &dphi);
int tet_ndofs(int k);

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
  std::vector<int32_t> cell2node;
};

namespace mf {

// Launch parameters of the hex sum-factorised kernel, per precision.
template <typename T> struct HexArgs {
  const int32_t *map;  // ncells x N^3 node ids (negative: constrained, -1-node)
  const T *geo;        // ncells x 24: trilinear coefficient vectors c1..c7 (x3), pad
  const T *coef;       // ncells x 8 monomial coefficients of the vertex coefficient, or null
  const T *x;
  T *y;
  int64_t c0, c1;      // cell range
  int ncomp;
};

// Hex tables for (T, N) are laid out contiguously as T B[N][N] (B[a][i] = l_i(g_a), GLL
// Lagrange basis at Gauss point a), T D[N][N] (D[a][b] = derivative of the Lagrange
// polynomial through the Gauss points, index b, at g_a), T g[N] (Gauss points on [0,1]),
// T w[N] (weights), T dB[N][N] (dB[a][i] = l_i'(g_a)); hex_table_bytes gives the size.
template <typename T> size_t hex_table_bytes(int N);

// Kernel launchers (hex_kernels.hip)
template <typename T>
int launch_hex_apply(int N, int kind, const HexArgs<T> &a, const void *tab, hipStream_t s);
template <typename T>
int launch_hex_diag(int N, int kind, const HexArgs<T> &a, const void *tab, hipStream_t s);

// Tet elasticity (simplex_kernels.hip)
template <typename T> struct TetArgs {
  const int32_t *map;  // AoSoA: [ncells/64][D][64] node ids (negative: constrained)
  const T *geo;        // AoSoA: [ncells/64][10][64]: Kinv (9, row-major Kinv[b][a]) and w-free |det|
  const T *tab;        // [Q][D][3] reference gradients, then [Q] weights (device)
  const T *x;
  T *y;
  int64_t c0, c1;
  T lam, mu;
};
template <typename T>
int launch_tet_elasticity(int k, int nq, const TetArgs<T> &a, hipStream_t s);
template <typename T>
int launch_tet_elasticity_diag(int k, int nq, const TetArgs<T> &a, hipStream_t s);

// Tri P1 mass with vertex coefficient (simplex_kernels.hip)
template <typename T> struct TriArgs {
  const int32_t *map;  // ncells x 3 (negative: constrained)
  const T *geo;        // ncells x 4: |T| c0, |T| c1, |T| c2, pad
  const T *x;
  T *y;
  int64_t c0, c1;
};
template <typename T> int launch_tri_mass(const TriArgs<T> &a, hipStream_t s);
template <typename T> int launch_tri_mass_diag(const TriArgs<T> &a, hipStream_t s);

// Vector kernels (vec_kernels.hip)
template <typename T> int launch_fill(T *y, T v, int64_t n, hipStream_t s);
template <typename T>
int launch_copy_constrained(const int32_t *dofs, int64_t n, const T *x, T *y, hipStream_t s);
template <typename T>
int launch_set_constrained(const int32_t *dofs, int64_t n, T v, T *y, hipStream_t s);

}  // namespace mf

struct mf_op {
  int cell_type = 0, kind = 0, precision = 0, degree = 0, ncomp = 0, nq1d = 0, nqp = 0, D = 0;
  int64_t ncells = 0, nnodes = 0, ndofs = 0;
  double lam = 1.0, mu = 0.5;
  bool has_coef = false;
  mf::DeviceBuffer map, geo, coef, tab, bc_dofs;
  int64_t n_bc_dofs = 0;
  std::vector<unsigned char> tab_host;  // hex tables passed by value to kernels
  double flops = 0.0, bytes = 0.0;
};
