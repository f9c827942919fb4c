// Host-side (FP64) quadrature rules and basis tabulations used to build the
// constant tables of the device kernels.
//
// The element kernel needs, for every quadrature point, the weights and the
// values and derivatives of the basis functions -- the constant arrays shared
// by all cells in the paper's generated local kernel (Section 2.1, Listing 2).
// On hexahedra only the 1D factors are kept (sum factorisation, Section 3,
// "sum factorization" on tensor-product cells), so the tables are:
//   B[a][i] = l_i(g_a)   GLL Lagrange polynomial i at Gauss point a,
//   D[a][b] = L_b'(g_a)  derivative of the Lagrange polynomial through the
//                        Gauss points (collocation derivative).
#include <algorithm>
#include <cmath>

#include <cmath>

#include "tables.h"

namespace mf {

// Legendre P_n and P_n' at x via the three-term recurrence.
static void legendre(int n, double x, double &p, double &dp) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { p = 1.0; dp = 0.0; return; }
  for (int j = 1; j < n; j++) {
    double p2 = ((2 * j + 1) * x * p1 - j * p0) / (j + 1);
    p0 = p1;
    p1 = p2;
  }
  p = p1;
  // P_n' = n (x P_n - P_{n-1}) / (x^2 - 1), valid away from +-1
  dp = n * (x * p1 - p0) / (x * x - 1.0);
}

void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; i++) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; it++) {
      double p, dp;
      legendre(n, z, p, dp);
      double dz = p / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p, dp;
    legendre(n, z, p, dp);
    x[i] = 0.5 * (1.0 - z);  // ascending on [0,1]
    w[i] = 1.0 / ((1.0 - z * z) * dp * dp);  // 2/((1-z^2)P'^2), halved for [0,1]
  }
}

std::vector<double> gll_points(int k) {
  std::vector<double> r(k + 1);
  r[0] = 0.0;
  r[k] = 1.0;
  for (int i = 1; i < k; i++) {
    // interior points: roots of P_k', Newton with P_k'' from Legendre's equation
    double z = -std::cos(M_PI * i / k);
    for (int it = 0; it < 100; it++) {
      double p, dp;
      legendre(k, z, p, dp);
      double ddp = (2.0 * z * dp - k * (k + 1) * p) / (1.0 - z * z);
      double dz = dp / ddp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    r[i] = 0.5 * (z + 1.0);
  }
  std::sort(r.begin(), r.end());
  return r;
}

// Barycentric Lagrange interpolation (second form) and its derivative.
void lagrange_eval(const std::vector<double> &nodes, const std::vector<double> &pts,
                   std::vector<double> &V, std::vector<double> &dV) {
  const int n = (int)nodes.size(), nq = (int)pts.size();
  std::vector<double> lam(n, 1.0);
  for (int i = 0; i < n; i++)
    for (int j = 0; j < n; j++)
      if (j != i) lam[i] /= (nodes[i] - nodes[j]);
  V.assign((size_t)nq * n, 0.0);
  dV.assign((size_t)nq * n, 0.0);
  for (int q = 0; q < nq; q++) {
    const double x = pts[q];
    int hit = -1;
    for (int m = 0; m < n; m++)
      if (x == nodes[m]) hit = m;
    if (hit >= 0) {
      for (int i = 0; i < n; i++) {
        V[q * n + i] = (i == hit) ? 1.0 : 0.0;
        if (i != hit) {
          dV[q * n + i] = (lam[i] / lam[hit]) / (x - nodes[i]);
        } else {
          double s = 0.0;
          for (int j = 0; j < n; j++)
            if (j != hit) s += 1.0 / (x - nodes[j]);
          dV[q * n + i] = s;
        }
      }
      continue;
    }
    double den = 0.0;
    for (int j = 0; j < n; j++) den += lam[j] / (x - nodes[j]);
    double sinv = 0.0;
    for (int j = 0; j < n; j++) sinv += 1.0 / (x - nodes[j]);
    for (int i = 0; i < n; i++) {
      double li = lam[i] / (x - nodes[i]) / den;
      V[q * n + i] = li;
      // l_i'(x) = l_i(x) * sum_{j != i} 1/(x - x_j)
      dV[q * n + i] = li * (sinv - 1.0 / (x - nodes[i]));
    }
  }
}

int tet_ndofs(int k) { return (k + 1) * (k + 2) * (k + 3) / 6; }

// Fully symmetric tet rules, barycentric orbits; weights sum to 1/6.
//   degree 1: centroid;  degree 2: 4 points (a,a,a,1-3a) with a = (5 - sqrt 5)/20;
//   degree 5: 14 points -- two (a,a,a,1-3a) orbits and one (a,a,1/2-a,1/2-a) orbit
//   (the positive-weight 14-point rule of Walkington / Keast).
// Gauss-Jacobi rule on [0, 1] for the weight (1 - u)^alpha: the n nodes are the roots
// of the Jacobi polynomial P_n^(alpha, 0)(2u - 1), found by Newton's method with
// deflation against the roots already found; with s = 2u - 1 the weights on [-1, 1],
// 2^(alpha+1) / ((1 - s^2) P_n'(s)^2), shrink by 2^-(alpha+1) on [0, 1]. The three-term
// recurrence and the derivative identity
//   (2n + alpha)(1 - s^2) P_n' = n (alpha - (2n + alpha) s) P_n + 2 n (n + alpha) P_(n-1)
// are the standard ones for beta = 0.
static void gauss_jacobi01(int n, int alpha, std::vector<double> &x, std::vector<double> &w) {
  const double a = alpha;
  auto eval = [&](double s, double &pn, double &dpn) {
    double p0 = 1.0, p1 = 0.5 * ((a + 2.0) * s + a);
    if (n == 1) {
      pn = p1;
      p1 = p0;
    } else {
      for (int k = 2; k <= n; k++) {
        const double c = 2.0 * k + a;
        const double p2 = ((c - 1.0) * (c * (c - 2.0) * s + a * a) * p1 - 2.0 * (k + a - 1.0) * (k - 1.0) * c * p0) /
                          (2.0 * k * (k + a) * (c - 2.0));
        p0 = p1;
        p1 = p2;
      }
      pn = p1;
      p1 = p0;  // P_(n-1)
    }
    dpn = (n * (a - (2.0 * n + a) * s) * pn + 2.0 * n * (n + a) * p1) / ((2.0 * n + a) * (1.0 - s * s));
  };
  std::vector<double> r;
  for (int i = 0; i < n; i++) {
    double s = -std::cos((2.0 * i + 1.0) * M_PI / (2.0 * n));  // ascending start values
    for (int it = 0; it < 100; it++) {
      double p, dp;
      eval(s, p, dp);
      double defl = 0.0;
      for (double q : r) defl += 1.0 / (s - q);
      const double ds = p / (dp - p * defl);
      s -= ds;
      if (std::fabs(ds) < 1e-16) break;
    }
    r.push_back(s);
  }
  std::sort(r.begin(), r.end());
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; i++) {
    double p, dp;
    eval(r[i], p, dp);
    x[i] = 0.5 * (r[i] + 1.0);
    w[i] = 1.0 / ((1.0 - r[i] * r[i]) * dp * dp);
  }
}

bool tet_rule(int degree, std::vector<double> &pts, std::vector<double> &w) {
  pts.clear();
  w.clear();
  auto s31 = [&](double a, double wt) {
    const double b = 1.0 - 3.0 * a;
    for (int i = 0; i < 4; i++) {
      double l[4] = {a, a, a, a};
      l[i] = b;
      pts.push_back(l[1]); pts.push_back(l[2]); pts.push_back(l[3]);
      w.push_back(wt);
    }
  };
  auto s22 = [&](double a, double wt) {
    const double b = 0.5 - a;
    for (int i = 0; i < 4; i++)
      for (int j = i + 1; j < 4; j++) {
        double l[4] = {b, b, b, b};
        l[i] = a;
        l[j] = a;
        pts.push_back(l[1]); pts.push_back(l[2]); pts.push_back(l[3]);
        w.push_back(wt);
      }
  };
  if (degree <= 1) {
    pts = {0.25, 0.25, 0.25};
    w = {1.0 / 6.0};
  } else if (degree == 2) {
    s31((5.0 - std::sqrt(5.0)) / 20.0, 1.0 / 24.0);
  } else if (degree <= 5) {
    s31(0.0927352503108912, 0.0734930431163619 / 6.0);
    s31(0.3108859192633006, 0.1126879257180159 / 6.0);
    s22(0.0455037041256496, 0.0425460207770812 / 6.0);
  } else if (degree <= 21) {
    // conical product rule: x = u, y = v (1 - u), z = t (1 - u)(1 - v), Jacobian
    // (1 - u)^2 (1 - v). A degree-p monomial has degree at most p in each of u, v, t, so
    // Gauss-Jacobi rules for the weights (1 - u)^2 and (1 - v), which absorb the
    // Jacobian, and Gauss-Legendre in t, each with n points (exact to degree 2n - 1),
    // integrate it exactly: n = (degree + 2) / 2, 64 points for degrees 6-7 up to 1331
    // for degrees 20-21
    const int n = (degree + 2) / 2;
    std::vector<double> xu, wu, xv, wv, xt, wt;
    gauss_jacobi01(n, 2, xu, wu);
    gauss_jacobi01(n, 1, xv, wv);
    gauss_legendre(n, xt, wt);
    for (int i = 0; i < n; i++)
      for (int j = 0; j < n; j++)
        for (int l = 0; l < n; l++) {
          const double u = xu[i], v = xv[j], t = xt[l];
          pts.push_back(u);
          pts.push_back(v * (1.0 - u));
          pts.push_back(t * (1.0 - u) * (1.0 - v));
          w.push_back(wu[i] * wv[j] * wt[l]);
        }
  } else {
    return false;
  }
  return true;
}

// Equispaced P_k Lagrange basis on the reference simplex of dimension dim, in the
// library's local node order (lattice a1 fastest), from the barycentric product form:
// the node with lattice index a (alpha_0 = k - sum a, alpha_j = a_j) has
//   phi_a(x) = prod_j P_{alpha_j}(lambda_j),  P_m(l) = prod_{r<m} (k l - r) / (r + 1),
// with lambda_0 = 1 - sum x, lambda_j = x_j. It is 1 at its node and 0 at the others
// (one factor vanishes there), and needs no linear solve. pts: [nq][dim].
static void simplex_lagrange(int k, int dim, const std::vector<double> &pts, std::vector<double> &phi,
                             std::vector<double> &dphi) {
  std::vector<int> al;  // barycentric multi-indices, dim + 1 per node
  if (dim == 3) {
    for (int a3 = 0; a3 <= k; a3++)
      for (int a2 = 0; a2 + a3 <= k; a2++)
        for (int a1 = 0; a1 + a2 + a3 <= k; a1++) al.insert(al.end(), {k - a1 - a2 - a3, a1, a2, a3});
  } else {
    for (int a2 = 0; a2 <= k; a2++)
      for (int a1 = 0; a1 + a2 <= k; a1++) al.insert(al.end(), {k - a1 - a2, a1, a2});
  }
  const int nb = dim + 1, D = (int)al.size() / nb, nq = (int)pts.size() / dim;
  // P_m(l) and its derivative for m = 0..k
  auto pm = [k](int m, double l, double &v, double &dv) {
    v = 1.0;
    dv = 0.0;
    for (int r = 0; r < m; r++) {
      const double f = (k * l - r) / (r + 1.0), df = k / (r + 1.0);
      dv = dv * f + v * df;
      v *= f;
    }
  };
  phi.assign((size_t)nq * D, 0.0);
  dphi.assign((size_t)nq * D * dim, 0.0);
  for (int q = 0; q < nq; q++) {
    double lam[4];
    lam[0] = 1.0;
    for (int d = 0; d < dim; d++) {
      lam[d + 1] = pts[q * dim + d];
      lam[0] -= lam[d + 1];
    }
    for (int i = 0; i < D; i++) {
      double v[4], dv[4];
      for (int j = 0; j < nb; j++) pm(al[i * nb + j], lam[j], v[j], dv[j]);
      double val = 1.0;
      for (int j = 0; j < nb; j++) val *= v[j];
      phi[(size_t)q * D + i] = val;
      // d lambda_0 / d x_d = -1, d lambda_j / d x_d = [j = d + 1]
      for (int d = 0; d < dim; d++) {
        double g0 = dv[0], gd = dv[d + 1];
        for (int j = 0; j < nb; j++) {
          if (j != 0) g0 *= v[j];
          if (j != d + 1) gd *= v[j];
        }
        dphi[((size_t)q * D + i) * dim + d] = gd - g0;
      }
    }
  }
}

// P_k Lagrange basis (equispaced nodes) on the reference tet at pts [nq][3]:
// phi [nq][D], dphi [nq][D][3].
void tet_lagrange(int k, const std::vector<double> &pts, std::vector<double> &phi,
                  std::vector<double> &dphi) {
  simplex_lagrange(k, 3, pts, phi, dphi);
}

// Triangle rule exact to the given degree: the Gauss product rule on the square mapped
// by the collapse x = u, y = v (1 - u) (Jacobian 1 - u), n = ceil((degree + 2) / 2)
// points per direction (the u-integrand gains one degree from the Jacobian).
void tri_rule(int degree, std::vector<double> &pts, std::vector<double> &w) {
  const int n = (degree + 3) / 2;
  std::vector<double> x, wx;
  gauss_legendre(n, x, wx);
  pts.clear();
  w.clear();
  for (int i = 0; i < n; i++)
    for (int j = 0; j < n; j++) {
      pts.push_back(x[i]);
      pts.push_back(x[j] * (1.0 - x[i]));
      w.push_back(wx[i] * wx[j] * (1.0 - x[i]));
    }
}

// P_k Lagrange basis (equispaced nodes, a1 fastest) on the reference triangle at pts
// [nq][2]: phi [nq][D], dphi [nq][D][2] (the barycentric product form above).
void tri_lagrange(int k, const std::vector<double> &pts, std::vector<double> &phi, std::vector<double> &dphi) {
  simplex_lagrange(k, 2, pts, phi, dphi);
}

}  // namespace mf
