// Host-side (FP64) quadrature rules and basis tabulations (no HIP dependency,
// so the build-time table generator links them with the host compiler alone).
#pragma once
#include <vector>

namespace mf {

// 1D Gauss-Legendre rule on [0,1], points ascending.
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w);
// k+1 Gauss-Lobatto-Legendre points on [0,1], ascending.
std::vector<double> gll_points(int k);
// Lagrange basis on `nodes` evaluated at `pts`: V[q*n+i], dV[q*n+i].
void lagrange_eval(const std::vector<double> &nodes, const std::vector<double> &pts,
                   std::vector<double> &V, std::vector<double> &dV);
// Simplex quadrature of the given exact degree on the reference tet: points (x,y,z) and
// weights (summing to 1/6). Returns false if no rule of that degree is built in.
bool tet_rule(int degree, std::vector<double> &pts, std::vector<double> &w);
// triangle: collapsed Gauss rule exact to `degree` (pts as (x, y) pairs) and the P_k
// equispaced Lagrange basis (a1 fastest) with reference gradients at given points
void tri_rule(int degree, std::vector<double> &pts, std::vector<double> &w);
void tri_lagrange(int k, const std::vector<double> &pts, std::vector<double> &phi, std::vector<double> &dphi);
// P_k Lagrange basis on the reference tet at pts: phi[q*D+i], dphi[(q*D+i)*3+d].
void tet_lagrange(int k, const std::vector<double> &pts, std::vector<double> &phi,
                  std::vector<double> &dphi);
int tet_ndofs(int k);

}  // namespace mf
