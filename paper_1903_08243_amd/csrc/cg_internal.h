// Conjugate-gradient internals shared by the solver driver and its kernels.
#pragma once
#include "mf_internal.h"

namespace mf {

constexpr int CG_NPART = 1024;  // per-block partial sums of one reduction (fixed order)

enum { CG_STAGE_RESIDUAL = 0, CG_STAGE_INIT = 1, CG_STAGE_PAP = 2, CG_STAGE_UPDATE = 3 };

// Device-resident iteration state.
struct CgState {
  double rz, pAp, alpha, beta, rr;
  double tol2;     // stop when r'r <= tol2
  int iters, maxit;
  int stop, breakdown;
};

int cg_residual(const double *b, const void *Ax, bool ax32, double *r, int64_t n, double *part, CgState *st,
                hipStream_t s);
// z = M^-1 r, p = z (+ FP32 copy), r'z and r'r; ap_zero (nullable, FP32 when p32 is set)
// is cleared for the next accumulating action
int cg_init(const double *r, const double *dinv, double *p, float *p32, int64_t n, double *part, CgState *st,
            hipStream_t s, void *ap_zero);
// after Ap = A p: alpha, x += alpha p, r -= alpha Ap, beta, p = z + beta p; Ap is cleared
// for the next accumulating action
int cg_step_after_apply(double *x, double *r, double *p, float *p32, void *Ap, bool ap32, const double *dinv,
                        int64_t n, double *part, CgState *st, hipStream_t s);
int cg_axpy(double *x, const double *d, int64_t n, hipStream_t s);
int cg_recip(const void *d, bool d32, double *dinv, int64_t n, hipStream_t s);
int cg_cast(const double *a, float *b, int64_t n, hipStream_t s);

}  // namespace mf

struct mf_precond {
  int kind = 0;  // 0 Jacobi, 1 learned
  int64_t n = 0;
  uint64_t numbering_id = 0;  // internal numbering of the operator it was built from
  mf::DeviceBuffer dinv;      // FP64 inverse diagonal, internal numbering
};
