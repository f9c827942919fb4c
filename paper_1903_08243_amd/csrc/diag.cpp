// Jacobi diagonal of the operators without a fused diagonal kernel, from the diagonals
// of their element matrices (diag_kernels.hip): one-component tet operators, triangle
// operators of degree 1-3 (other than the closed-form P1 mass), hex elasticity and the
// hex scalar operators with k+2 points. The FP64 tables are those of the operator's own
// quadrature rule, built here and freed when the call returns.
#include "mf_internal.h"

namespace mf {

bool element_diag_supported(const mf_op *op) {
  if (op->kind == MF_OP_HYPERELASTIC) return false;
  if (op->cell_type == MF_CELL_TET) return op->ncomp == 1 || op->degree >= 4;
  if (op->cell_type == MF_CELL_TRI) return !(op->kind == MF_OP_MASS && op->degree == 1);
  if (op->cell_type == MF_CELL_HEX) return op->kind == MF_OP_ELASTICITY || op->nq1d != op->degree + 1;
  return false;
}

template <typename T> int element_diag(const mf_op *op, T *d, hipStream_t s) {
  std::vector<double> tab, pts, w, phi, dphi;
  const int ct = op->cell_type;
  if (ct == MF_CELL_HEX) {
    std::vector<double> V, dV;
    gauss_legendre(op->nq1d, pts, w);
    lagrange_eval(gll_points(op->degree), pts, V, dV);
    tab = V;
    tab.insert(tab.end(), dV.begin(), dV.end());
    tab.insert(tab.end(), w.begin(), w.end());
    tab.insert(tab.end(), pts.begin(), pts.end());
  } else {
    const int dim = ct == MF_CELL_TET ? 3 : 2;
    if (ct == MF_CELL_TET) {
      if (!tet_rule(op->qdeg, pts, w)) return fail(MF_EUNSUPPORTED, "diagonal: tet rule");
      tet_lagrange(op->degree, pts, phi, dphi);
    } else {
      tri_rule(op->qdeg, pts, w);
      tri_lagrange(op->degree, pts, phi, dphi);
    }
    tab = phi;
    tab.insert(tab.end(), dphi.begin(), dphi.end());
    tab.insert(tab.end(), w.begin(), w.end());
    for (size_t q = 0; q < w.size(); q++) {
      const double *x = &pts[dim * q];
      double s0 = 1.0;
      for (int a = 0; a < dim; a++) s0 -= x[a];
      tab.push_back(s0);
      for (int a = 0; a < dim; a++) tab.push_back(x[a]);
    }
  }
  DeviceBuffer dtab;
  int rc = dtab.alloc(tab.size() * sizeof(double));
  if (rc) return rc;
  MF_HIP(hipMemcpyAsync(dtab.ptr, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice, s));
  const T *coef = op->has_coef ? op->coef.as<T>() : nullptr;
  if (ct == MF_CELL_HEX)
    rc = launch_hex_element_diag<T>(op->map.as<int32_t>(), op->geo.as<T>(), coef, dtab.as<double>(), op->ncells,
                                    op->degree + 1, op->nq1d, op->kind, op->ncomp, op->lam, op->mu, d, s);
  else
    rc = launch_simplex_element_diag<T>(ct == MF_CELL_TET ? 3 : 2, op->map.as<int32_t>(), op->geo.as<T>(), coef,
                                        dtab.as<double>(), op->ncells, op->D, (int)w.size(), op->kind, op->ncomp,
                                        op->lam, op->mu, d, s);
  if (rc) return rc;
  MF_HIP(hipStreamSynchronize(s));  // the table is freed on return
  return MF_OK;
}

template int element_diag<double>(const mf_op *, double *, hipStream_t);
template int element_diag<float>(const mf_op *, float *, hipStream_t);

}  // namespace mf
