// Build-time generator of the hex kernels' 1D tables as compile-time constants.
//
// The sum-factorised kernels contract every pencil with the same small
// matrices; as constexpr values the compiler materialises them with scalar
// moves at the point of use instead of keeping ~100 doubles live in scalar
// registers (which spills). The values come from the library's host table
// code (tables.cpp), printed as exact hexadecimal floating-point literals.
//   B[a][i]  = l_i(g_a)   GLL Lagrange basis i at Gauss point a
//   D[a][b]  = L_b'(g_a)  collocation derivative on the Gauss points
//   dB[a][i] = l_i'(g_a)
//   g[a], w[a]            Gauss points and weights on [0,1]
//   HexR<n>::B[a][i]      l_i at the n+1 Gauss points (the paper's k+2 rule)
#include <cstdio>
#include <vector>

#include "tables.h"

static void mat(const char *name, const std::vector<double> &v, int n) {
  std::printf("  static constexpr double %s[%d][%d] = {", name, n, n);
  for (int a = 0; a < n; a++) {
    std::printf("{");
    for (int i = 0; i < n; i++) std::printf("%a%s", v[a * n + i], i + 1 < n ? ", " : "");
    std::printf("}%s", a + 1 < n ? ", " : "");
  }
  std::printf("};\n");
}

static void vec(const char *name, const std::vector<double> &v) {
  std::printf("  static constexpr double %s[%zu] = {", name, v.size());
  for (size_t a = 0; a < v.size(); a++) std::printf("%a%s", v[a], a + 1 < v.size() ? ", " : "");
  std::printf("};\n");
}

int main() {
  std::printf("// generated at build time by gen_hex_tables.cpp -- do not edit\n#pragma once\n");
  std::printf("namespace mf {\ntemplate <int N> struct HexC;\n");
  // k = 1..6; k = 7 only for the 8-point rule (points, weights, collocation derivative)
  // of the Q6 operators with k+2 points
  for (int k = 1; k <= 7; k++) {
    const int n = k + 1;
    std::vector<double> g, w, V, dV, Vg, dVg;
    mf::gauss_legendre(n, g, w);
    mf::lagrange_eval(mf::gll_points(k), g, V, dV);
    mf::lagrange_eval(g, g, Vg, dVg);
    std::printf("template <> struct HexC<%d> {\n", n);
    mat("B", V, n);
    mat("D", dVg, n);
    mat("dB", dV, n);
    vec("g", g);
    vec("w", w);
    std::printf("};\n");
  }
  // the paper's k+2 points: B[a][i] = l_i(g_a) on the n+1 Gauss points (k = 1..6); the
  // collocation derivative and the points and weights are HexC<n+1>'s
  std::printf("template <int N> struct HexR;\n");
  for (int k = 1; k <= 6; k++) {
    const int n = k + 1, q = n + 1;
    std::vector<double> g, w, V, dV;
    mf::gauss_legendre(q, g, w);
    mf::lagrange_eval(mf::gll_points(k), g, V, dV);
    std::printf("template <> struct HexR<%d> {\n  static constexpr double B[%d][%d] = {", n, q, n);
    for (int a = 0; a < q; a++) {
      std::printf("{");
      for (int i = 0; i < n; i++) std::printf("%a%s", V[a * n + i], i + 1 < n ? ", " : "");
      std::printf("}%s", a + 1 < q ? ", " : "");
    }
    std::printf("};\n};\n");
  }
  std::printf("}  // namespace mf\n");
  return 0;
}
