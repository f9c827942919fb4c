// Assembly of the global sparse matrix of an operator (CSR, user numbering): the
// paper's matrix assembly (Section 5) beside the matrix-free action. The pattern is
// built on the host from the cell-to-node map (entry (r, c) exists when the nodes of
// dofs r and c share a cell); the values are the element matrices computed on the
// device and added at their CSR positions (csr_kernels.hip).
#include <algorithm>

#include "mf_internal.h"

namespace mf {

static bool csr_supported(const mf_op *op) {
  return (op->cell_type == MF_CELL_TET && op->kind != MF_OP_HYPERELASTIC && op->degree <= 3) ||
         (op->cell_type == MF_CELL_TRI && op->kind == MF_OP_MASS && op->degree == 1);
}

static void build_pattern(const mf_op *op) {
  if (op->csr_built) return;
  const int D = op->D, nc = op->ncomp;
  std::vector<std::vector<int32_t>> nbr((size_t)op->nnodes);
  for (int64_t K = 0; K < op->ncells; K++) {
    const int32_t *u = op->h_unode.data() + K * D;
    for (int a = 0; a < D; a++)
      for (int b = 0; b < D; b++) nbr[u[a]].push_back(u[b]);
  }
  op->csr_rowptr.assign((size_t)op->ndofs + 1, 0);
  op->csr_col.clear();
  for (int64_t n = 0; n < op->nnodes; n++) {
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

template <typename T> static int assemble(const mf_op *op, T *vals, hipStream_t s) {
  build_pattern(op);
  const int64_t nnz = (int64_t)op->csr_col.size();
  if (op->ncells == 0) return launch_fill<T>(vals, T(0), nnz, s);
  DeviceBuffer drow, dcol, dun, dtab, dpos;
  int rc = drow.alloc(op->csr_rowptr.size() * sizeof(int64_t));
  if (!rc) rc = dcol.alloc(std::max<size_t>(1, (size_t)nnz) * sizeof(int32_t));
  if (!rc) rc = dun.alloc(op->h_unode.size() * sizeof(int32_t));
  if (rc) return rc;
  MF_HIP(hipMemcpyAsync(drow.ptr, op->csr_rowptr.data(), op->csr_rowptr.size() * sizeof(int64_t),
                        hipMemcpyHostToDevice, s));
  if (nnz) MF_HIP(hipMemcpyAsync(dcol.ptr, op->csr_col.data(), (size_t)nnz * 4, hipMemcpyHostToDevice, s));
  MF_HIP(hipMemcpyAsync(dun.ptr, op->h_unode.data(), op->h_unode.size() * 4, hipMemcpyHostToDevice, s));
  rc = launch_fill<T>(vals, T(0), nnz, s);
  if (rc) return rc;
  std::vector<double> tab;
  if (op->cell_type == MF_CELL_TET) {
    // the operator's own rule: phi [nq][D], reference gradients [nq][D][3], weights,
    // vertex basis [nq][4]
    std::vector<double> pts, w, phi, dphi;
    if (!tet_rule(op->qdeg, pts, w)) return fail(MF_EUNSUPPORTED, "assembly: tet rule");
    tet_lagrange(op->degree, pts, phi, dphi);
    tab = phi;
    tab.insert(tab.end(), dphi.begin(), dphi.end());
    tab.insert(tab.end(), w.begin(), w.end());
    for (size_t q = 0; q < w.size(); q++) {
      const double *x = &pts[3 * q];
      tab.push_back(1.0 - x[0] - x[1] - x[2]);
      for (int a = 0; a < 3; a++) tab.push_back(x[a]);
    }
    rc = dtab.alloc(tab.size() * sizeof(double));
    if (rc) return rc;
    MF_HIP(hipMemcpyAsync(dtab.ptr, tab.data(), tab.size() * 8, hipMemcpyHostToDevice, s));
    rc = launch_tet_element_csr<T>(op->map.as<int32_t>(), dun.as<int32_t>(), op->geo.as<T>(),
                                   op->has_coef ? op->coef.as<T>() : nullptr, dtab.as<double>(), op->ncells, op->D,
                                   (int)w.size(), op->kind, op->ncomp, op->lam, op->mu, drow.as<int64_t>(),
                                   dcol.as<int32_t>(), vals, s);
  } else {
    rc = launch_tri_mass_element_csr<T>(op->map.as<int32_t>(), dun.as<int32_t>(), op->geo.as<T>(), op->ncells,
                                        drow.as<int64_t>(), dcol.as<int32_t>(), vals, s);
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

int mf_op_csr_pattern(const mf_op *op, int64_t *rowptr, int32_t *col, int64_t *nnz) {
  if (!op) return fail(MF_EINVAL, "mf_op_csr_pattern: null operator");
  if (!csr_supported(op))
    return fail(MF_EUNSUPPORTED, "mf_op_csr_pattern: assembly is built for tet operators of degree 1-3 (not "
                                 "HYPERELASTIC) and the P1 triangle mass");
  build_pattern(op);
  if (nnz) *nnz = (int64_t)op->csr_col.size();
  if (rowptr) std::copy(op->csr_rowptr.begin(), op->csr_rowptr.end(), rowptr);
  if (col) std::copy(op->csr_col.begin(), op->csr_col.end(), col);
  return MF_OK;
}

int mf_op_assemble_csr(const mf_op *op, void *vals, void *stream) {
  if (!op || !vals) return fail(MF_EINVAL, "mf_op_assemble_csr: null argument");
  if (!csr_supported(op))
    return fail(MF_EUNSUPPORTED, "mf_op_assemble_csr: assembly is built for tet operators of degree 1-3 (not "
                                 "HYPERELASTIC) and the P1 triangle mass");
  hipStream_t s = (hipStream_t)stream;
  return op->precision == MF_F64 ? assemble<double>(op, (double *)vals, s) : assemble<float>(op, (float *)vals, s);
}

}  // extern "C"
