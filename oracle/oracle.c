/*
 * CPU FP64 oracle for the matrix-free finite element operator action.
 *
 * TEST INFRASTRUCTURE. Only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark may load this library. It shares no code with the GPU path.
 *
 * What it computes is the paper's global assembly of a linear form (Section 2,
 * eq. 1: v_i = L(u; phi_i)) done the plain way of Section 2.2 (Listing 3's
 * gather / zero / local kernel / scatter loop) with the local kernel written as
 * in Section 2.1 (Listing 2: Jacobian, its inverse and |det| from the vertex
 * coordinates, a loop over quadrature points that evaluates the trial function
 * from densely tabulated basis values, then accumulation against every test
 * function). Here the Jacobian is evaluated at every quadrature point (the
 * general case the paper states for multilinear quad/hex maps; for affine
 * simplices it is the same at every point). There is no sum factorisation, no
 * hoisting and no blocking.
 *
 * Pointwise integrands (supplementary material "operators"): for a trial field
 * u with value u_c and physical gradient G_ca = d u_c / d x_a at a point, the
 * bilinear form is written as  sum_c f0_c v_c + sum_{c,a} f1_ca d v_c / d x_a:
 *   MASS        f0 = coef * u                                 (int c u v)
 *   HELMHOLTZ   f0 = u,          f1 = grad u                   (eq. 2)
 *   LAPLACIAN   f1_c = grad u_c  for each component            (int grad u : grad v)
 *   POISSON     f1 = coef * grad u                             (int kappa grad u . grad v)
 *   ELASTICITY  f1 = lambda tr(G) I + mu (G + G^T)             (int sigma(u) : grad v)
 *   HYPERELASTIC  the St-Venant-Kirchhoff model of the supplementary operator list
 *               (F = I + grad u0, E = (F^T F - I)/2, Psi = lambda/2 tr(E)^2 + mu tr(E^2),
 *               S = dPsi/dE = lambda tr(E) I + 2 mu E, P = F S) linearised at a given
 *               field u0: the directional derivative of P in the direction of the
 *               trial field, f1 = dF S + F dS with dF = G, dE = (dF^T F + F^T dF)/2,
 *               dS = lambda tr(dE) I + 2 mu dE
 *   HYPER_RESIDUAL  the nonlinear form itself at u = x: f1 = P(I + G)   (int P : grad v)
 * The coefficient is a per-vertex field interpolated with the coordinate map's
 * vertex basis (linear on simplices, trilinear on hexahedra).
 *
 * Parallelism: OpenMP over cells, each thread accumulating into its own copy of
 * the output vector, summed at the end (so the result equals the sequential
 * scatter up to summation order).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { OP_MASS = 0, OP_HELMHOLTZ = 1, OP_LAPLACIAN = 2, OP_POISSON = 3, OP_ELASTICITY = 4,
       OP_HYPERELASTIC = 5, OP_HYPER_RESIDUAL = 6 };
enum { MODE_ACTION = 0, MODE_DIAG = 1 };

#define MAXV 8
#define MAXC 3

typedef struct {
  int gdim, nvc, D, ncomp, nq, op;
  double lam, mu;
  const double *coords, *qw, *vN, *vdN, *phi, *dphi, *vcoef;
  const int *c2v, *c2n;
  const double *u0; /* linearisation point of HYPERELASTIC (node-interleaved like x) */
} problem;

/* Jacobian J[a][b] = d x_a / d xi_b at quadrature point q; returns det J and
 * fills the inverse K[b][a] = d xi_b / d x_a by cofactors. */
static double jacobian(const problem *P, const double *X, int q, double J[3][3], double K[3][3]) {
  const int g = P->gdim;
  for (int a = 0; a < g; a++)
    for (int b = 0; b < g; b++) {
      double s = 0.0;
      for (int v = 0; v < P->nvc; v++) s += X[v * g + a] * P->vdN[(q * P->nvc + v) * g + b];
      J[a][b] = s;
    }
  double det;
  if (g == 2) {
    det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    K[0][0] = J[1][1] / det;
    K[0][1] = -J[0][1] / det;
    K[1][0] = -J[1][0] / det;
    K[1][1] = J[0][0] / det;
  } else {
    double C[3][3]; /* cofactor matrix */
    C[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    C[0][1] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    C[0][2] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    C[1][0] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    C[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    C[1][2] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    C[2][0] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    C[2][1] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    C[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    det = J[0][0] * C[0][0] + J[0][1] * C[0][1] + J[0][2] * C[0][2];
    /* inverse = adjugate / det, adjugate = C^T */
    for (int b = 0; b < 3; b++)
      for (int a = 0; a < 3; a++) K[b][a] = C[a][b] / det;
  }
  return det;
}

/* Second Piola-Kirchhoff stress of the St-Venant-Kirchhoff model for a strain E. */
static void svk_stress(const problem *P, double E[3][3], double S[3][3]) {
  const double tr = E[0][0] + E[1][1] + E[2][2];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) S[i][j] = 2.0 * P->mu * E[i][j] + (i == j ? P->lam * tr : 0.0);
}

/* Pointwise fluxes (f0, f1) of the bilinear form for trial value u and gradient G;
 * G0 is the gradient of the linearisation point u0 (HYPERELASTIC only). */
static void pointwise(const problem *P, double coef, const double *u, double G[MAXC][3],
                      double G0[MAXC][3], double *f0, double f1[MAXC][3]) {
  const int g = P->gdim, nc = P->ncomp;
  for (int c = 0; c < nc; c++) {
    f0[c] = 0.0;
    for (int a = 0; a < 3; a++) f1[c][a] = 0.0;
  }
  switch (P->op) {
    case OP_MASS:
      for (int c = 0; c < nc; c++) f0[c] = coef * u[c];
      break;
    case OP_HELMHOLTZ:
      for (int c = 0; c < nc; c++) {
        f0[c] = u[c];
        for (int a = 0; a < g; a++) f1[c][a] = G[c][a];
      }
      break;
    case OP_LAPLACIAN:
      for (int c = 0; c < nc; c++)
        for (int a = 0; a < g; a++) f1[c][a] = G[c][a];
      break;
    case OP_POISSON:
      for (int c = 0; c < nc; c++)
        for (int a = 0; a < g; a++) f1[c][a] = coef * G[c][a];
      break;
    case OP_ELASTICITY: {
      double tr = 0.0;
      for (int a = 0; a < g; a++) tr += G[a][a];
      for (int c = 0; c < g; c++)
        for (int a = 0; a < g; a++)
          f1[c][a] = P->mu * (G[c][a] + G[a][c]) + (c == a ? P->lam * tr : 0.0);
      break;
    }
    case OP_HYPERELASTIC: {
      /* F = I + grad u0; E = (F^T F - I)/2; S(E); dF = G; dE = (dF^T F + F^T dF)/2; dS(dE);
       * f1 = dF S + F dS */
      double F[3][3], E[3][3], S[3][3], dE[3][3], dS[3][3];
      for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) F[i][j] = (i == j ? 1.0 : 0.0) + G0[i][j];
      for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
          double c = 0.0, d = 0.0;
          for (int k = 0; k < 3; k++) {
            c += F[k][i] * F[k][j];
            d += G[k][i] * F[k][j] + F[k][i] * G[k][j];
          }
          E[i][j] = 0.5 * (c - (i == j ? 1.0 : 0.0));
          dE[i][j] = 0.5 * d;
        }
      svk_stress(P, E, S);
      svk_stress(P, dE, dS);
      for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
          double s = 0.0;
          for (int k = 0; k < 3; k++) s += G[i][k] * S[k][j] + F[i][k] * dS[k][j];
          f1[i][j] = s;
        }
      break;
    }
    case OP_HYPER_RESIDUAL: {
      /* P = F S(E) with F = I + grad u, u = the trial field itself */
      double F[3][3], E[3][3], S[3][3];
      for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) F[i][j] = (i == j ? 1.0 : 0.0) + G[i][j];
      for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
          double c = 0.0;
          for (int k = 0; k < 3; k++) c += F[k][i] * F[k][j];
          E[i][j] = 0.5 * (c - (i == j ? 1.0 : 0.0));
        }
      svk_stress(P, E, S);
      for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
          double s = 0.0;
          for (int k = 0; k < 3; k++) s += F[i][k] * S[k][j];
          f1[i][j] = s;
        }
      break;
    }
  }
}

/* Gradient of the linearisation point u0 at one point (zero when there is none). */
static void grad_u0(const problem *P, long cell, const double *gphi, double G0[MAXC][3]) {
  for (int c = 0; c < MAXC; c++)
    for (int a = 0; a < 3; a++) G0[c][a] = 0.0;
  if (!P->u0) return;
  const int D = P->D, nc = P->ncomp;
  for (int i = 0; i < D; i++) {
    const long n = P->c2n[cell * D + i];
    for (int c = 0; c < nc; c++)
      for (int a = 0; a < P->gdim; a++) G0[c][a] += gphi[i * 3 + a] * P->u0[n * nc + c];
  }
}

/* One cell: gather, local kernel, scatter into out (action) or diagonal. */
static void cell_kernel(const problem *P, long cell, const double *x, double *out, int mode,
                        double *xe, double *ye, double *gphi) {
  const int g = P->gdim, nvc = P->nvc, D = P->D, nc = P->ncomp;
  double X[MAXV * 3], cv[MAXV];
  for (int v = 0; v < nvc; v++) {
    int vid = P->c2v[cell * nvc + v];
    for (int a = 0; a < g; a++) X[v * g + a] = P->coords[(long)vid * g + a];
    cv[v] = P->vcoef ? P->vcoef[vid] : 1.0;
  }
  if (mode == MODE_ACTION)
    for (int i = 0; i < D; i++)
      for (int c = 0; c < nc; c++) xe[i * nc + c] = x[(long)P->c2n[cell * D + i] * nc + c];
  for (int i = 0; i < D * nc; i++) ye[i] = 0.0;

  for (int q = 0; q < P->nq; q++) {
    double J[3][3], K[3][3];
    double det = jacobian(P, X, q, J, K);
    double wdet = P->qw[q] * fabs(det);
    double coef = 0.0;
    for (int v = 0; v < nvc; v++) coef += P->vN[q * nvc + v] * cv[v];
    /* physical gradients of every basis function: grad phi_i = J^{-T} grad_ref phi_i */
    for (int i = 0; i < D; i++)
      for (int a = 0; a < g; a++) {
        double s = 0.0;
        for (int b = 0; b < g; b++) s += K[b][a] * P->dphi[(q * D + i) * g + b];
        gphi[i * 3 + a] = s;
      }
    const double *ph = P->phi + (long)q * D;
    double G0[MAXC][3];
    grad_u0(P, cell, gphi, G0);
    if (mode == MODE_ACTION) {
      double u[MAXC] = {0}, G[MAXC][3] = {{0}}, f0[MAXC], f1[MAXC][3];
      for (int i = 0; i < D; i++)
        for (int c = 0; c < nc; c++) {
          u[c] += ph[i] * xe[i * nc + c];
          for (int a = 0; a < g; a++) G[c][a] += gphi[i * 3 + a] * xe[i * nc + c];
        }
      pointwise(P, coef, u, G, G0, f0, f1);
      for (int i = 0; i < D; i++)
        for (int c = 0; c < nc; c++) {
          double s = f0[c] * ph[i];
          for (int a = 0; a < g; a++) s += f1[c][a] * gphi[i * 3 + a];
          ye[i * nc + c] += wdet * s;
        }
    } else {
      /* diagonal entry a(phi_i e_c, phi_i e_c) */
      for (int i = 0; i < D; i++)
        for (int c = 0; c < nc; c++) {
          double u[MAXC] = {0}, G[MAXC][3] = {{0}}, f0[MAXC], f1[MAXC][3];
          u[c] = ph[i];
          for (int a = 0; a < g; a++) G[c][a] = gphi[i * 3 + a];
          pointwise(P, coef, u, G, G0, f0, f1);
          double s = f0[c] * ph[i];
          for (int a = 0; a < g; a++) s += f1[c][a] * gphi[i * 3 + a];
          ye[i * nc + c] += wdet * s;
        }
    }
  }
  for (int i = 0; i < D; i++)
    for (int c = 0; c < nc; c++) out[(long)P->c2n[cell * D + i] * nc + c] += ye[i * nc + c];
}

static int run(const problem *P, long c0, long c1, long ndofs, const double *x, double *y,
               int mode, int nthreads) {
  if (nthreads < 1) nthreads = 1;
  double *part = (double *)calloc((size_t)ndofs * nthreads, sizeof(double));
  if (!part) return -1;
  const int D = P->D, nc = P->ncomp;
#pragma omp parallel num_threads(nthreads)
  {
    int t = 0;
#ifdef _OPENMP
    t = omp_get_thread_num();
#endif
    double *xe = (double *)malloc(sizeof(double) * D * nc);
    double *ye = (double *)malloc(sizeof(double) * D * nc);
    double *gphi = (double *)malloc(sizeof(double) * D * 3);
    double *mine = part + (size_t)t * ndofs;
#pragma omp for schedule(static)
    for (long cell = c0; cell < c1; cell++) cell_kernel(P, cell, x, mine, mode, xe, ye, gphi);
    free(xe);
    free(ye);
    free(gphi);
  }
  for (long i = 0; i < ndofs; i++) {
    double s = 0.0;
    for (int t = 0; t < nthreads; t++) s += part[(size_t)t * ndofs + i];
    y[i] = s;
  }
  free(part);
  return 0;
}

#define PROBLEM_ARGS                                                                         \
  int gdim, int nvc, const double *coords, const int *c2v, int D, const int *c2n, int ncomp, \
      int nq, const double *qw, const double *vN, const double *vdN, const double *phi,     \
      const double *dphi, int op, double lam, double mu, const double *vcoef, const double *u0

#define FILL_PROBLEM                                                                        \
  problem P = {gdim, nvc, D, ncomp, nq, op, lam, mu, coords, qw, vN, vdN, phi, dphi, vcoef, \
               c2v, c2n, u0}

/* y = A x over cells [c0, c1); y (ndofs) is overwritten. */
int oracle_apply(PROBLEM_ARGS, long c0, long c1, long ndofs, const double *x, double *y,
                 int nthreads) {
  FILL_PROBLEM;
  return run(&P, c0, c1, ndofs, x, y, MODE_ACTION, nthreads);
}

/* d = diag(A); d (ndofs) is overwritten. */
int oracle_diagonal(PROBLEM_ARGS, long ncells, long ndofs, double *d, int nthreads) {
  FILL_PROBLEM;
  return run(&P, 0, ncells, ndofs, NULL, d, MODE_DIAG, nthreads);
}

/* Element matrices A_K[(i,c),(j,d)] = a(phi_j e_d, phi_i e_c), for tiny meshes:
 * out has ncells * (D*ncomp)^2 entries, row (test) index first. */
int oracle_element_matrices(PROBLEM_ARGS, long ncells, double *out) {
  FILL_PROBLEM;
  const int nc = ncomp, n = D * nc, g = gdim;
  double *gphi = (double *)malloc(sizeof(double) * D * 3);
  for (long cell = 0; cell < ncells; cell++) {
    double X[MAXV * 3], cv[MAXV];
    for (int v = 0; v < nvc; v++) {
      int vid = c2v[cell * nvc + v];
      for (int a = 0; a < g; a++) X[v * g + a] = coords[(long)vid * g + a];
      cv[v] = vcoef ? vcoef[vid] : 1.0;
    }
    double *A = out + cell * (long)n * n;
    memset(A, 0, sizeof(double) * n * n);
    for (int q = 0; q < nq; q++) {
      double J[3][3], K[3][3];
      double wdet = qw[q] * fabs(jacobian(&P, X, q, J, K));
      double coef = 0.0;
      for (int v = 0; v < nvc; v++) coef += vN[q * nvc + v] * cv[v];
      for (int i = 0; i < D; i++)
        for (int a = 0; a < g; a++) {
          double s = 0.0;
          for (int b = 0; b < g; b++) s += K[b][a] * dphi[(q * D + i) * g + b];
          gphi[i * 3 + a] = s;
        }
      const double *ph = phi + (long)q * D;
      double G0[MAXC][3];
      grad_u0(&P, cell, gphi, G0);
      for (int j = 0; j < D; j++)
        for (int d = 0; d < nc; d++) {
          double u[MAXC] = {0}, G[MAXC][3] = {{0}}, f0[MAXC], f1[MAXC][3];
          u[d] = ph[j];
          for (int a = 0; a < g; a++) G[d][a] = gphi[j * 3 + a];
          pointwise(&P, coef, u, G, G0, f0, f1);
          for (int i = 0; i < D; i++)
            for (int c = 0; c < nc; c++) {
              double s = f0[c] * ph[i];
              for (int a = 0; a < g; a++) s += f1[c][a] * gphi[i * 3 + a];
              A[(i * nc + c) * n + (j * nc + d)] += wdet * s;
            }
        }
    }
  }
  free(gphi);
  return 0;
}

/* Signed Jacobian determinant at every quadrature point of every cell (for
 * mesh validity checks); out has ncells * nq entries. */
int oracle_detj(PROBLEM_ARGS, long ncells, double *out) {
  FILL_PROBLEM;
  for (long cell = 0; cell < ncells; cell++) {
    double X[MAXV * 3];
    for (int v = 0; v < nvc; v++)
      for (int a = 0; a < gdim; a++) X[v * gdim + a] = coords[(long)c2v[cell * nvc + v] * gdim + a];
    for (int q = 0; q < nq; q++) {
      double J[3][3], K[3][3];
      out[cell * nq + q] = jacobian(&P, X, q, J, K);
    }
  }
  return 0;
}
