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
  } else if (degree <= 9) {
    // conical product rule: x = u, y = v (1 - u), z = t (1 - u)(1 - v), Jacobian
    // (1 - u)^2 (1 - v). A degree-p monomial has degree at most p in each of u, v, t, so
    // Gauss-Jacobi rules for the weights (1 - u)^2 and (1 - v), which absorb the
    // Jacobian, and Gauss-Legendre in t, each with n points (exact to degree 2n - 1),
    // integrate it exactly: n = 4 (64 points) for degrees 6-7, n = 5 (125 points) for
    // degrees 8-9
    const int n = degree <= 7 ? 4 : 5;
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

// P_k Lagrange basis on the reference tet by inverting the monomial
// Vandermonde matrix at the equispaced lattice points.
void tet_lagrange(int k, const std::vector<double> &pts, std::vector<double> &phi,
                  std::vector<double> &dphi) {
  const int D = tet_ndofs(k);
  std::vector<int> ex;  // monomial exponents (p,q,r)
  for (int p = 0; p <= k; p++)
    for (int q = 0; q + p <= k; q++)
      for (int r = 0; r + q + p <= k; r++) { ex.push_back(p); ex.push_back(q); ex.push_back(r); }
  std::vector<double> nodes;  // lattice in the library's local order: a1 fastest, a3 slowest
  for (int a3 = 0; a3 <= k; a3++)
    for (int a2 = 0; a2 + a3 <= k; a2++)
      for (int a1 = 0; a1 + a2 + a3 <= k; a1++) {
        nodes.push_back((double)a1 / k);
        nodes.push_back((double)a2 / k);
        nodes.push_back((double)a3 / k);
      }
  // Vandermonde V[n][m] = monomial m at node n; coefficients C = V^{-1} (column i -> phi_i)
  std::vector<double> A((size_t)D * 2 * D, 0.0);
  for (int n = 0; n < D; n++) {
    for (int m = 0; m < D; m++)
      A[n * 2 * D + m] = std::pow(nodes[3 * n], ex[3 * m]) * std::pow(nodes[3 * n + 1], ex[3 * m + 1]) *
                         std::pow(nodes[3 * n + 2], ex[3 * m + 2]);
    A[n * 2 * D + D + n] = 1.0;
  }
  for (int c = 0; c < D; c++) {  // Gauss-Jordan with partial pivoting
    int piv = c;
    for (int r = c + 1; r < D; r++)
      if (std::fabs(A[r * 2 * D + c]) > std::fabs(A[piv * 2 * D + c])) piv = r;
    for (int j = 0; j < 2 * D; j++) std::swap(A[c * 2 * D + j], A[piv * 2 * D + j]);
    double d = A[c * 2 * D + c];
    for (int j = 0; j < 2 * D; j++) A[c * 2 * D + j] /= d;
    for (int r = 0; r < D; r++)
      if (r != c) {
        double f = A[r * 2 * D + c];
        for (int j = 0; j < 2 * D; j++) A[r * 2 * D + j] -= f * A[c * 2 * D + j];
      }
  }
  // inverse: Vinv[m][n] = A[m][D+n]; phi_i(x) = sum_m Vinv[m][i] mono_m(x)
  const int nq = (int)pts.size() / 3;
  phi.assign((size_t)nq * D, 0.0);
  dphi.assign((size_t)nq * D * 3, 0.0);
  auto pw = [](double b, int e) { return e <= 0 ? 1.0 : std::pow(b, e); };
  for (int q = 0; q < nq; q++) {
    const double x = pts[3 * q], y = pts[3 * q + 1], z = pts[3 * q + 2];
    for (int m = 0; m < D; m++) {
      const int p = ex[3 * m], r1 = ex[3 * m + 1], r2 = ex[3 * m + 2];
      const double val = pw(x, p) * pw(y, r1) * pw(z, r2);
      const double dx = p ? p * pw(x, p - 1) * pw(y, r1) * pw(z, r2) : 0.0;
      const double dy = r1 ? r1 * pw(x, p) * pw(y, r1 - 1) * pw(z, r2) : 0.0;
      const double dz = r2 ? r2 * pw(x, p) * pw(y, r1) * pw(z, r2 - 1) : 0.0;
      for (int i = 0; i < D; i++) {
        const double c = A[m * 2 * D + D + i];
        phi[q * D + i] += c * val;
        dphi[(q * D + i) * 3 + 0] += c * dx;
        dphi[(q * D + i) * 3 + 1] += c * dy;
        dphi[(q * D + i) * 3 + 2] += c * dz;
      }
    }
  }
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

// P_k Lagrange basis on the reference triangle (equispaced lattice, a1 fastest) by
// inverting the monomial Vandermonde matrix, as tet_lagrange in two dimensions.
void tri_lagrange(int k, const std::vector<double> &pts, std::vector<double> &phi, std::vector<double> &dphi) {
  const int D = (k + 1) * (k + 2) / 2;
  std::vector<int> ex;  // monomial exponents (p, q)
  for (int p = 0; p <= k; p++)
    for (int q = 0; q + p <= k; q++) { ex.push_back(p); ex.push_back(q); }
  std::vector<double> nodes;
  for (int a2 = 0; a2 <= k; a2++)
    for (int a1 = 0; a1 + a2 <= k; a1++) {
      nodes.push_back((double)a1 / k);
      nodes.push_back((double)a2 / k);
    }
  auto pw = [](double b, int e) { return e <= 0 ? 1.0 : std::pow(b, e); };
  std::vector<double> A((size_t)D * 2 * D, 0.0);
  for (int n = 0; n < D; n++) {
    for (int m = 0; m < D; m++) A[n * 2 * D + m] = pw(nodes[2 * n], ex[2 * m]) * pw(nodes[2 * n + 1], ex[2 * m + 1]);
    A[n * 2 * D + D + n] = 1.0;
  }
  for (int c = 0; c < D; c++) {  // Gauss-Jordan with partial pivoting
    int piv = c;
    for (int r = c + 1; r < D; r++)
      if (std::fabs(A[r * 2 * D + c]) > std::fabs(A[piv * 2 * D + c])) piv = r;
    for (int j = 0; j < 2 * D; j++) std::swap(A[c * 2 * D + j], A[piv * 2 * D + j]);
    const double d = A[c * 2 * D + c];
    for (int j = 0; j < 2 * D; j++) A[c * 2 * D + j] /= d;
    for (int r = 0; r < D; r++)
      if (r != c) {
        const double f = A[r * 2 * D + c];
        for (int j = 0; j < 2 * D; j++) A[r * 2 * D + j] -= f * A[c * 2 * D + j];
      }
  }
  const int nq = (int)pts.size() / 2;
  phi.assign((size_t)nq * D, 0.0);
  dphi.assign((size_t)nq * D * 2, 0.0);
  for (int q = 0; q < nq; q++) {
    const double x = pts[2 * q], y = pts[2 * q + 1];
    for (int m = 0; m < D; m++) {
      const int p = ex[2 * m], r = ex[2 * m + 1];
      const double val = pw(x, p) * pw(y, r);
      const double dx = p ? p * pw(x, p - 1) * pw(y, r) : 0.0;
      const double dy = r ? r * pw(x, p) * pw(y, r - 1) : 0.0;
      for (int i = 0; i < D; i++) {
        const double c = A[m * 2 * D + D + i];
        phi[q * D + i] += c * val;
        dphi[(q * D + i) * 2 + 0] += c * dx;
        dphi[(q * D + i) * 2 + 1] += c * dy;
      }
    }
  }
}

}  // namespace mf
