// Assembly of the global sparse matrix of an operator (CSR, user numbering): the
// paper's matrix assembly (Section 5) beside the matrix-free action. The pattern is
// built on the host from the space's cell-to-node map (entry (r, c) exists when the
// nodes of dofs r and c share a cell); the values are the element matrices computed on
// the device and added at their CSR positions (csr_kernels.hip).
#include <algorithm>

#include "mf_internal.h"

namespace mf {

static const char *kCsrScope =
    "assembly is built for tet and triangle operators of degree 1-6, quadrilaterals of degree 1-6 and hexahedra of "
    "degree 1-4 (not HYPERELASTIC)";

static bool csr_supported(const mf_op *op) {
  if (op->kind == MF_OP_HYPERELASTIC) return false;
  switch (op->cell_type) {
    case MF_CELL_TET:
    case MF_CELL_TRI: return op->degree <= 6;
    case MF_CELL_QUAD: return op->degree <= 6;
    case MF_CELL_HEX: return op->degree <= 4;
  }
  return false;
}

static int csr_check(const mf_op *op, const mf_space *sp, const char *who) {
  if (!op || !sp) return fail(MF_EINVAL, std::string(who) + ": null argument");
  if (sp->numbering_id != op->numbering_id || sp->ncells != op->ncells || sp->D != op->D)
    return fail(MF_EINVAL, std::string(who) + ": the operator was not created on this space");
  if (!csr_supported(op)) return fail(MF_EUNSUPPORTED, std::string(who) + ": " + kCsrScope);
  return MF_OK;
}

static void build_pattern(const mf_op *op, const mf_space *sp) {
  if (op->csr_built) return;
  const int D = sp->D, nc = sp->ncomp;
  std::vector<std::vector<int32_t>> nbr((size_t)sp->nnodes);
  for (int64_t K = 0; K < sp->ncells; K++) {
    const int32_t *u = sp->cell2node.data() + K * D;
    for (int a = 0; a < D; a++)
      for (int b = 0; b < D; b++) nbr[u[a]].push_back(u[b]);
  }
  op->csr_rowptr.assign((size_t)sp->nnodes * nc + 1, 0);
  op->csr_col.clear();
  for (int64_t n = 0; n < sp->nnodes; n++) {
    auto &v = nbr[n];
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    for (int c = 0; c < nc; c++) {
      for (int32_t m : v)
        for (int d = 0; d < nc; d++) op->csr_col.push_back(m * nc + d);
      op->csr_rowptr[(size_t)n * nc + c + 1] = (int64_t)op->csr_col.size();
    }
    std::vector<int32_t>().swap(v);
  }
  op->csr_built = true;
}

// FP64 tables of the operator's own rule: simplices phi [nq][D], reference gradients
// [nq][D][dim], weights [nq], vertex basis [nq][dim+1]; tensor cells B [q][n],
// B' [q][n], weights, points
static int csr_tables(const mf_op *op, std::vector<double> &tab, int &nq) {
  std::vector<double> pts, w, phi, dphi;
  const int ct = op->cell_type;
  if (ct == MF_CELL_HEX || ct == MF_CELL_QUAD) {
    std::vector<double> V, dV;
    gauss_legendre(op->nq1d, pts, w);
    lagrange_eval(gll_points(op->degree), pts, V, dV);
    tab = V;
    tab.insert(tab.end(), dV.begin(), dV.end());
    tab.insert(tab.end(), w.begin(), w.end());
    tab.insert(tab.end(), pts.begin(), pts.end());
    nq = op->nq1d;
    return MF_OK;
  }
  const int dim = ct == MF_CELL_TET ? 3 : 2;
  if (ct == MF_CELL_TET) {
    if (!tet_rule(op->qdeg, pts, w)) return fail(MF_EUNSUPPORTED, "assembly: tet rule");
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
  nq = (int)w.size();
  return MF_OK;
}

template <typename T> static int assemble(const mf_op *op, const mf_space *sp, T *vals, hipStream_t s) {
  build_pattern(op, sp);
  const int64_t nnz = (int64_t)op->csr_col.size();
  int rc = launch_fill<T>(vals, T(0), nnz, s);
  if (rc || op->ncells == 0) return rc;
  // user node of each (internal cell, local node)
  const int D = sp->D;
  std::vector<int32_t> unode((size_t)sp->ncells * D);
  for (int64_t ic = 0; ic < sp->ncells; ic++)
    for (int i = 0; i < D; i++) unode[ic * D + i] = sp->cell2node[(int64_t)sp->cell_user_of_int[ic] * D + i];
  std::vector<double> tab;
  int nq = 0;
  const bool p1mass = op->cell_type == MF_CELL_TRI && op->kind == MF_OP_MASS && op->degree == 1;
  if (!p1mass) {
    rc = csr_tables(op, tab, nq);
    if (rc) return rc;
  }
  DeviceBuffer drow, dcol, dun, dtab, dpos;
  rc = drow.alloc(op->csr_rowptr.size() * sizeof(int64_t));
  if (!rc) rc = dcol.alloc(std::max<size_t>(1, (size_t)nnz) * sizeof(int32_t));
  if (!rc) rc = dun.alloc(unode.size() * sizeof(int32_t));
  if (!rc && !p1mass) rc = dtab.alloc(tab.size() * sizeof(double));
  if (rc) return rc;
  MF_HIP(hipMemcpyAsync(drow.ptr, op->csr_rowptr.data(), op->csr_rowptr.size() * sizeof(int64_t),
                        hipMemcpyHostToDevice, s));
  if (nnz) MF_HIP(hipMemcpyAsync(dcol.ptr, op->csr_col.data(), (size_t)nnz * 4, hipMemcpyHostToDevice, s));
  MF_HIP(hipMemcpyAsync(dun.ptr, unode.data(), unode.size() * 4, hipMemcpyHostToDevice, s));
  if (!p1mass) MF_HIP(hipMemcpyAsync(dtab.ptr, tab.data(), tab.size() * 8, hipMemcpyHostToDevice, s));
  const T *coef = op->has_coef ? op->coef.as<T>() : nullptr;
  const int32_t *map = op->map.as<int32_t>();
  if (p1mass) {
    rc = launch_tri_mass_element_csr<T>(map, dun.as<int32_t>(), op->geo.as<T>(), op->ncells, drow.as<int64_t>(),
                                        dcol.as<int32_t>(), vals, s);
  } else if (op->cell_type == MF_CELL_TET || op->cell_type == MF_CELL_TRI) {
    rc = launch_simplex_element_csr<T>(op->cell_type == MF_CELL_TET ? 3 : 2, map, dun.as<int32_t>(), op->geo.as<T>(),
                                       coef, dtab.as<double>(), op->ncells, D, nq, op->kind, op->ncomp, op->lam,
                                       op->mu, drow.as<int64_t>(), dcol.as<int32_t>(), vals, s);
  } else {
    rc = launch_tensor_element_csr<T>(op->cell_type == MF_CELL_HEX ? 3 : 2, map, dun.as<int32_t>(), op->geo.as<T>(),
                                      coef, dtab.as<double>(), op->ncells, op->degree + 1, nq, op->kind, op->ncomp,
                                      op->lam, op->mu, drow.as<int64_t>(), dcol.as<int32_t>(), vals, s);
  }
  if (rc) return rc;
  // constrained dofs: identity rows (their other entries and columns stay 0)
  if (!op->h_bc_user.empty()) {
    std::vector<int64_t> pos;
    for (int32_t r : op->h_bc_user) {
      const auto b = op->csr_col.begin() + op->csr_rowptr[r], e = op->csr_col.begin() + op->csr_rowptr[r + 1];
      const auto it = std::lower_bound(b, e, r);
      if (it == e || *it != r) return fail(MF_EINVAL, "assembly: diagonal missing from the pattern");
      pos.push_back(it - op->csr_col.begin());
    }
    rc = dpos.alloc(pos.size() * sizeof(int64_t));
    if (rc) return rc;
    MF_HIP(hipMemcpyAsync(dpos.ptr, pos.data(), pos.size() * 8, hipMemcpyHostToDevice, s));
    rc = launch_set_at<T>(dpos.as<int64_t>(), (int64_t)pos.size(), T(1), vals, s);
    if (rc) return rc;
  }
  MF_HIP(hipStreamSynchronize(s));  // the temporary buffers are freed on return
  return MF_OK;
}

}  // namespace mf

using namespace mf;

extern "C" {

int mf_op_csr_pattern(const mf_op *op, const mf_space *space, int64_t *rowptr, int32_t *col, int64_t *nnz) {
  int rc = csr_check(op, space, "mf_op_csr_pattern");
  if (rc) return rc;
  build_pattern(op, space);
  if (nnz) *nnz = (int64_t)op->csr_col.size();
  if (rowptr) std::copy(op->csr_rowptr.begin(), op->csr_rowptr.end(), rowptr);
  if (col) std::copy(op->csr_col.begin(), op->csr_col.end(), col);
  return MF_OK;
}

int mf_op_assemble_csr(const mf_op *op, const mf_space *space, void *vals, void *stream) {
  int rc = csr_check(op, space, "mf_op_assemble_csr");
  if (rc) return rc;
  if (!vals) return fail(MF_EINVAL, "mf_op_assemble_csr: null vals");
  hipStream_t s = (hipStream_t)stream;
  return op->precision == MF_F64 ? assemble<double>(op, space, (double *)vals, s)
                                 : assemble<float>(op, space, (float *)vals, s);
}

}  // extern "C"
