// Conjugate-gradient internals shared by the solver driver and its kernels.
#pragma once
#include "cnn_internal.h"
#include "mf_internal.h"

namespace mf {

constexpr int CG_NPART = 1024;  // per-block partial sums of one reduction (fixed order)

enum {
  CG_STAGE_RESIDUAL = 0,
  CG_STAGE_INIT = 1,
  CG_STAGE_PAP = 2,
  CG_STAGE_UPDATE = 3,
  // flexible CG (non-linear preconditioner)
  CG_STAGE_FUPDATE = 4,  // r'r after x, r update
  CG_STAGE_FZ = 5,       // z'r, z'Ap, non-finite count of z: accept z or flag the Jacobi fallback
  CG_STAGE_FZFIX = 6,    // after the fallback pass: beta (Polak-Ribiere) and r'z
  CG_STAGE_FINIT = 7,    // first z: r'r, z'r, non-finite count
  CG_STAGE_RELIABLE = 8  // after r was replaced by the true residual: r'z, r'r (iterations kept)
};

// Device-resident iteration state.
struct CgState {
  double rz, pAp, alpha, beta, rr;
  double tol2;     // stop when r'r <= tol2
  int iters, maxit;
  int stop, breakdown;
  int fallback;   // flexible CG: this iteration's z is replaced by the Jacobi z
  int nfallback;  // flexible CG: iterations that used the fallback
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
// reliable update: r'z and r'r of the replaced residual r (z = M^{-1} r); the search
// direction and the iteration count are kept, stop is re-evaluated
int cg_reliable(const double *r, const double *dinv, int64_t n, double *part, CgState *st, hipStream_t s);
int cg_recip(const void *d, bool d32, double *dinv, int64_t n, hipStream_t s);
int cg_cast(const double *a, float *b, int64_t n, hipStream_t s);
int cg_sqrt(const double *a, double *b, int64_t n, hipStream_t s);
int cg_scale(const double *d, const double *a, double *b, int64_t n, hipStream_t s);  // b = d a

// Flexible PCG pieces (z produced by a preconditioner between the calls).
// Before the loop: z = M r computed; fcg_init sets r'r, r'z (Jacobi z if M's z is
// unusable) and p = z (+ FP32 copy), clearing ap_zero.
int fcg_init(const double *r, double *z, const double *dinv, double *p, float *p32, int64_t n, double *part,
             CgState *st, hipStream_t s, void *ap_zero);
// After Ap = A p: alpha, x += alpha p, r -= alpha Ap, r'r.
int fcg_update(double *x, double *r, const double *p, const void *Ap, bool ap32, int64_t n, double *part,
               CgState *st, hipStream_t s);
// After z = M r: checks z, Jacobi fallback, beta = -alpha z'Ap / r'z_old, p = z + beta p, Ap cleared.
int fcg_direction(const double *r, double *z, const double *dinv, double *p, float *p32, void *Ap, bool ap32,
                  int64_t n, double *part, CgState *st, hipStream_t s);
int precond_cnn_apply_internal(const mf_precond *P, const double *r, double *z, hipStream_t s);

// Device workspace (bytes) that a solve of (A64, A32, M) needs: every vector of the
// solve, each rounded up to 256 bytes.
size_t cg_workspace_bytes(const mf_op *A64, const mf_op *A32, const mf_precond *M);
// mf_cg_solve on the caller's stream with its vectors carved from ws (ws_bytes
// long): creates no stream, event, graph or pinned buffer and allocates no device
// memory (learned preconditioners are rejected). MF_EINVAL when the solve needs more
// than ws_bytes.
int cg_solve_in(void *ws, size_t ws_bytes, const mf_op *A64, const mf_op *A32, const mf_precond *M,
                const double *b, double *x, double rtol, double inner_rtol, int maxit, mf_cg_info *info,
                hipStream_t s);

}  // namespace mf

struct mf_precond {
  int kind = 0;  // 0 Jacobi, 1 learned
  int64_t n = 0;
  uint64_t numbering_id = 0;  // internal numbering of the operator it was built from
  mf::DeviceBuffer dinv;      // FP64 inverse diagonal, internal numbering
  // numbering of the operator (for applies to user-numbered vectors)
  int64_t nnodes = 0;
  int ncomp = 1;
  bool identity = true;
  mf::DeviceBuffer perm;  // internal node -> user node (int32), empty if identity
  mutable mf::DeviceBuffer wr, wz;  // user-numbering workspaces (grown on first use)
  // learned preconditioner (kind 1): network borrowed from the caller, lattice of
  // gz x gy x gx points, grid index and D^{-1/2} per internal dof, Dirichlet mask
  const mf_cnn *net = nullptr;
  int gz = 0, gy = 0, gx = 0;
  mf::DeviceBuffer gidx, sd, bc, gin, gaux;
  mutable mf::CnnActs acts;
};
