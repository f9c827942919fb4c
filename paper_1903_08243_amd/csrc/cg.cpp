// Conjugate-gradient driver: plain FP64 PCG, and FP32-action iterative
// refinement (FP64 outer residual, FP64 inner vectors, dots and updates).
//
// The operator action is the paper's matrix-free residual evaluation
// (Section 1: a matrix-vector product is the assembly of a linear form);
// CG is the textbook consumer of that action and is not part of the paper.
//
// The iteration body (operator action + dot + finalize + update + finalize +
// search-direction update) is a fixed launch sequence with device-resident
// scalars. A chunk of CHUNK iterations is captured once into a hipGraph on a
// private stream and replayed; the host reads the 64-byte state after each
// replay to test convergence. Iterations after convergence are no-ops
// (alpha = beta = 0), so a partially used chunk is harmless.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>

#include "cg_internal.h"

namespace mf {

static constexpr int CHUNK = 8;

struct CgWork {
  int64_t n = 0;
  // device vectors of one solve: owned by `own` (mf_cg_solve) or carved from a
  // caller-provided workspace (cg_solve_in); null when the solve does not need them
  double *r = nullptr, *p = nullptr, *Ap = nullptr, *part = nullptr, *d = nullptr, *bi = nullptr, *xi = nullptr,
         *z = nullptr;
  float *p32 = nullptr, *Ap32 = nullptr;
  CgState *st = nullptr;
  DeviceBuffer own[11];
  const mf_precond *M = nullptr;  // learned preconditioner (flexible CG), or null
  hipStream_t s = nullptr;
  bool own_stream = false;
  bool graphs = true;  // replay captured chunks (false: launch each chunk directly)
  hipEvent_t ev = nullptr;
  CgState *host_st = nullptr;  // pinned (mf_cg_solve) or host_local
  bool pinned = false;
  CgState host_local{};
  hipGraphExec_t exec[2] = {nullptr, nullptr};  // [0] FP64 operator chunk, [1] FP32 operator chunk
  ~CgWork() {
    for (auto &e : exec)
      if (e) (void)hipGraphExecDestroy(e);
    if (pinned && host_st) (void)hipHostFree(host_st);
    if (ev) (void)hipEventDestroy(ev);
    if (own_stream && s) (void)hipStreamDestroy(s);
  }
};

// The device vectors a solve of (A64, A32, M) needs, in a fixed order: one entry
// per vector with its size in bytes (0 when unused).
struct CgNeed {
  void **slot[11];
  size_t bytes[11];
};
static CgNeed cg_need(CgWork &w, const mf_op *A64, const mf_op *A32, const mf_precond *M) {
  const size_t n = (size_t)A64->ndofs;
  const bool learned = M && M->kind == 1, perm = !A64->identity;
  return CgNeed{{(void **)&w.r, (void **)&w.p, (void **)&w.Ap, (void **)&w.part, (void **)&w.st, (void **)&w.z,
                 (void **)&w.p32, (void **)&w.Ap32, (void **)&w.d, (void **)&w.bi, (void **)&w.xi},
                {n * 8, n * 8, n * 8, (size_t)4 * CG_NPART * 8, sizeof(CgState), learned ? n * 8 : 0,
                 A32 ? n * 4 : 0, A32 ? n * 4 : 0, A32 ? n * 8 : 0, perm ? n * 8 : 0, perm ? n * 8 : 0}};
}
static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// all solver vectors live in the operators' internal numbering; the output was
// cleared by the preceding vector kernel, so the action accumulates
static int apply_any(const mf_op *A, const void *x, void *y, hipStream_t s) { return op_apply_internal_acc(A, x, y, s); }

// One chunk of PCG iterations on operator A (FP64 or FP32 action), recorded on w.s.
static int record_chunk(const mf_op *A, const double *dinv, double *x, CgWork &w) {
  const bool a32 = A->precision == MF_F32;
  if (w.M) {
    // flexible CG: z = M r from the learned preconditioner, Polak-Ribiere beta
    for (int j = 0; j < CHUNK; j++) {
      void *Ap = a32 ? (void *)w.Ap32 : (void *)w.Ap;
      int rc = a32 ? apply_any(A, w.p32, Ap, w.s) : apply_any(A, w.p, Ap, w.s);
      if (!rc) rc = fcg_update(x, w.r, w.p, Ap, a32, w.n, w.part,
                               w.st, w.s);
      if (!rc) rc = precond_cnn_apply_internal(w.M, w.r, w.z, w.s);
      if (!rc) rc = fcg_direction(w.r, w.z, dinv, w.p,
                                  a32 ? w.p32 : nullptr, Ap, a32, w.n, w.part,
                                  w.st, w.s);
      if (rc) return rc;
    }
    return MF_OK;
  }
  for (int j = 0; j < CHUNK; j++) {
    int rc = a32 ? apply_any(A, w.p32, w.Ap32, w.s) : apply_any(A, w.p, w.Ap, w.s);
    if (rc) return rc;
    rc = cg_step_after_apply(x, w.r, w.p, a32 ? w.p32 : nullptr,
                             a32 ? (void *)w.Ap32 : (void *)w.Ap, a32, dinv, w.n, w.part, w.st,
                             w.s);
    if (rc) return rc;
  }
  return MF_OK;
}

static int chunk_graph(const mf_op *A, const double *dinv, double *x, CgWork &w, hipGraphExec_t &exec) {
  if (exec) return MF_OK;
  hipGraph_t g = nullptr;
  MF_HIP(hipStreamBeginCapture(w.s, hipStreamCaptureModeThreadLocal));
  int rc = record_chunk(A, dinv, x, w);
  hipError_t e = hipStreamEndCapture(w.s, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(MF_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    exec = nullptr;
    return fail(MF_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  return MF_OK;
}

static int read_state(CgWork &w, CgState &out) {
  MF_HIP(hipMemcpyAsync(w.host_st, w.st, sizeof(CgState), hipMemcpyDeviceToHost, w.s));
  MF_HIP(hipStreamSynchronize(w.s));
  out = *w.host_st;
  return MF_OK;
}

// PCG from the residual already stored in w.r (for iterate x); x is updated in place.
static int pcg_core(const mf_op *A, const double *dinv, double *x, double tol2, int maxit, CgWork &w,
                    CgState &out) {
  const bool a32 = A->precision == MF_F32;
  CgState init{};
  init.tol2 = tol2;
  init.maxit = maxit;
  *w.host_st = init;
  MF_HIP(hipMemcpyAsync(w.st, w.host_st, sizeof(CgState), hipMemcpyHostToDevice, w.s));
  int rc;
  if (w.M) {
    rc = precond_cnn_apply_internal(w.M, w.r, w.z, w.s);
    if (!rc) rc = fcg_init(w.r, w.z, dinv, w.p,
                           a32 ? w.p32 : nullptr, w.n, w.part, w.st, w.s,
                           a32 ? (void *)w.Ap32 : (void *)w.Ap);
  } else {
    rc = cg_init(w.r, dinv, w.p, a32 ? w.p32 : nullptr, w.n,
                 w.part, w.st, w.s, a32 ? (void *)w.Ap32 : (void *)w.Ap);
  }
  if (rc) return rc;
  rc = read_state(w, out);
  if (rc || out.stop || maxit <= 0) return rc;
  hipGraphExec_t &exec = w.exec[a32 ? 1 : 0];
  if (w.graphs) {
    rc = chunk_graph(A, dinv, x, w, exec);
    if (rc) return rc;
  }
  while (true) {
    if (w.graphs) {
      MF_HIP(hipGraphLaunch(exec, w.s));
    } else {
      rc = record_chunk(A, dinv, x, w);
      if (rc) return rc;
    }
    rc = read_state(w, out);
    if (rc) return rc;
    if (out.stop) break;
  }
  return MF_OK;
}

// FP32-action PCG with reliable updates: one Krylov sequence on A32 with FP64 vectors,
// dots and updates; whenever the recursively updated residual has dropped by `delta`
// since the last true one (and when it meets the target), r is replaced by the true
// residual b - A64 x and r'z recomputed, keeping the search direction (the reliable
// updates of van der Vorst and Ye, 2000). The FP32 rounding of the action then only
// perturbs the search directions and x converges to the FP64 solution, without the
// restarts of outer-inner refinement. w.r holds b - A64 x on entry; rr returns the
// last true r'r.
static int pcg_reliable(const mf_op *A32, const mf_op *A64, const double *b, const double *dinv, double *x,
                        double tol2, int maxit, double delta, CgWork &w, mf_cg_info &inf, double &rr) {
  CgState init{};
  init.tol2 = tol2;
  init.maxit = maxit;
  *w.host_st = init;
  MF_HIP(hipMemcpyAsync(w.st, w.host_st, sizeof(CgState), hipMemcpyHostToDevice, w.s));
  int rc = cg_init(w.r, dinv, w.p, w.p32, w.n, w.part, w.st, w.s, w.Ap32);
  CgState st{};
  if (!rc) rc = read_state(w, st);
  if (rc || st.stop || maxit <= 0) return rc;
  double rr_ref = st.rr;
  hipGraphExec_t &exec = w.exec[1];
  if (w.graphs) {
    rc = chunk_graph(A32, dinv, x, w, exec);
    if (rc) return rc;
  }
  while (true) {
    if (w.graphs) {
      MF_HIP(hipGraphLaunch(exec, w.s));
    } else {
      rc = record_chunk(A32, dinv, x, w);
      if (rc) return rc;
    }
    rc = read_state(w, st);
    if (rc) return rc;
    inf.inner_iterations = st.iters;
    if (st.breakdown) return fail(MF_EBREAKDOWN, "CG breakdown (non-finite value or p'Ap <= 0)");
    if (!st.stop && st.rr > delta * rr_ref) continue;
    // reliable update: r = b - A64 x, then r'z, r'r
    rc = op_apply_internal(A64, x, w.Ap, w.s);
    if (!rc) rc = cg_residual(b, w.Ap, false, w.r, w.n, w.part, w.st, w.s);
    if (!rc) rc = cg_reliable(w.r, dinv, w.n, w.part, w.st, w.s);
    if (!rc) rc = read_state(w, st);
    if (rc) return rc;
    inf.outer_iterations++;
    rr = st.rr;
    rr_ref = st.rr;
    if (st.breakdown) return fail(MF_EBREAKDOWN, "CG breakdown (non-finite residual)");
    if (st.stop) return MF_OK;  // converged on the true residual, or maxit
  }
}

static int residual(const mf_op *A64, const double *b, const double *x, CgWork &w, double &rr) {
  int rc = op_apply_internal(A64, x, w.Ap, w.s);
  if (rc) return rc;
  rc = cg_residual(b, w.Ap, false, w.r, w.n, w.part, w.st, w.s);
  if (rc) return rc;
  CgState st;
  rc = read_state(w, st);
  rr = st.rr;
  return rc;
}

}  // namespace mf

using namespace mf;

extern "C" {

int mf_precond_create_jacobi(const mf_op *A, void *stream, mf_precond **out) {
  if (!A || !out) return fail(MF_EINVAL, "mf_precond_create_jacobi: null argument");
  hipStream_t s = (hipStream_t)stream;
  std::unique_ptr<mf_precond> P(new (std::nothrow) mf_precond);
  if (!P) return fail(MF_ENOMEM, "mf_precond_create_jacobi: host allocation");
  P->kind = 0;
  P->n = A->ndofs;
  P->numbering_id = A->numbering_id;
  P->nnodes = A->nnodes;
  P->ncomp = A->ncomp;
  P->identity = A->identity;
  DeviceBuffer d;
  int rc = d.alloc((size_t)A->ndofs * (A->precision == MF_F64 ? 8 : 4));
  if (!rc && !A->identity) {
    rc = P->perm.alloc((size_t)A->nnodes * 4);
    if (!rc) MF_HIP(hipMemcpyAsync(P->perm.ptr, A->perm.ptr, (size_t)A->nnodes * 4, hipMemcpyDeviceToDevice, s));
  }
  if (!rc) rc = P->dinv.alloc((size_t)A->ndofs * 8);
  if (!rc) rc = op_diagonal_internal(A, d.ptr, s);
  if (!rc) rc = cg_recip(d.ptr, A->precision == MF_F32, P->dinv.as<double>(), A->ndofs, s);
  if (rc) return rc;
  MF_HIP(hipStreamSynchronize(s));
  *out = P.release();
  return MF_OK;
}

void mf_precond_destroy(mf_precond *p) {
  if (!p) return;
  (void)hipDeviceSynchronize();
  delete p;
}

}  // extern "C"

namespace mf {

static int cg_check(const mf_op *A64, const mf_op *A32, const mf_precond *M, const double *b, double *x, double rtol,
                    int maxit, const char *who) {
  const std::string f(who);
  if (!A64 || !b || !x) return fail(MF_EINVAL, f + ": null argument");
  if (A64->precision != MF_F64) return fail(MF_EINVAL, f + ": A64 must be an FP64 operator");
  if (A32 && (A32->ndofs != A64->ndofs || A32->precision != MF_F32))
    return fail(MF_EINVAL, f + ": A32 must be an FP32 operator of the same size");
  if (A32 && A32->numbering_id != A64->numbering_id)
    return fail(MF_EINVAL, f + ": A32 and A64 must be built on the same space");
  if (M && (M->n != A64->ndofs || M->numbering_id != A64->numbering_id))
    return fail(MF_EINVAL, f + ": preconditioner built for another space");
  if (!(rtol > 0.0) || maxit < 0) return fail(MF_EINVAL, f + ": rtol / maxit");
  return MF_OK;
}

// The solve proper, on w.s with w's vectors bound: the outer loop, the inner PCG
// chunks and the moves between the user and the internal numbering.
static int cg_core(CgWork &w, const mf_op *A64, const mf_op *A32, const mf_precond *M, const double *b, double *x,
                   double rtol, double inner_rtol, int maxit, mf_cg_info *info) {
  const int64_t n = A64->ndofs;
  const double *dinv = M ? M->dinv.as<double>() : nullptr;
  // move b and x into the internal numbering (once per solve)
  double *x_user = x;
  int rc = MF_OK;
  if (!A64->identity) {
    const int32_t *uoi = A64->perm.as<int32_t>();
    rc = launch_to_internal<double>(uoi, A64->nnodes, A64->ncomp, b, w.bi, w.s);
    if (!rc) rc = launch_to_internal<double>(uoi, A64->nnodes, A64->ncomp, x, w.xi, w.s);
    if (rc) return rc;
    b = w.bi;
    x = w.xi;
  }

  // ||b||^2 via the residual kernel with Ax = 0 is avoided: r = b - A*0 costs an apply; use r = b - Ap with Ap = 0
  rc = launch_fill<double>(w.Ap, 0.0, n, w.s);
  if (!rc) rc = cg_residual(b, w.Ap, false, w.r, n, w.part, w.st, w.s);
  CgState st{};
  if (!rc) rc = read_state(w, st);
  if (rc) return rc;
  const double bb = st.rr;
  mf_cg_info inf{0, 0, 0, 0.0};
  if (bb == 0.0) {
    rc = launch_fill<double>(x_user, 0.0, n, w.s);
    if (!rc) rc = read_state(w, st);
    if (info) *info = inf;
    return rc;
  }
  const double tol2 = rtol * rtol * bb;
  double rr = 0.0;
  int status = MF_OK;
  if (!A32) {
    // plain PCG with the FP64 action; restart from the true residual if the recurrence drifted
    for (int restart = 0; restart < 5; restart++) {
      rc = residual(A64, b, x, w, rr);
      if (rc) return rc;
      inf.outer_iterations++;
      if (rr <= tol2 || inf.inner_iterations >= maxit) break;
      rc = pcg_core(A64, dinv, x, tol2, maxit - inf.inner_iterations, w, st);
      if (rc) return rc;
      inf.inner_iterations += st.iters;
      inf.fallbacks += st.nfallback;
      if (st.breakdown) {
        status = fail(MF_EBREAKDOWN, "CG breakdown (non-finite value or p'Ap <= 0)");
        break;
      }
    }
    if (status == MF_OK) {
      rc = residual(A64, b, x, w, rr);
      if (rc) return rc;
    }
  } else if (!w.M) {
    // FP32 action with a reliable update every `delta` of residual reduction
    // (inner_rtol; default 1e-3, measured best among 0.3 .. 1e-4: Helmholtz Q3 at 32^3
    // 49.2 ms against 51.9 ms in FP64, Q5 at 24^3 101.5 against 119.1 ms, Q2 at 64^3
    // 113.8 against 137.5 ms)
    const double delta = inner_rtol > 0.0 ? std::min(inner_rtol, 0.5) : 1e-3;
    rc = residual(A64, b, x, w, rr);
    if (rc) return rc;
    inf.outer_iterations = 1;
    if (rr > tol2 && maxit > 0) {
      status = pcg_reliable(A32, A64, b, dinv, x, tol2, maxit, delta, w, inf, rr);
      if (status == MF_EDEVICE) return status;
    }
  } else {
    // learned preconditioner (flexible CG) with the FP32 action: outer-inner
    // refinement. Inner tolerance: aim straight at the final target, but not below the FP32
    // action's accuracy floor (inner_rtol, default 1e-6): the first inner solve
    // then removes six orders of magnitude and the next one the rest, so little
    // Krylov information is lost to restarts.
    const double floor_rt = inner_rtol > 0.0 ? inner_rtol : 1e-6;
    for (int outer = 0; outer < 100; outer++) {
      rc = residual(A64, b, x, w, rr);
      if (rc) return rc;
      inf.outer_iterations++;
      if (rr <= tol2 || !(rr == rr) || inf.inner_iterations >= maxit) break;
      const double irt = std::max(floor_rt, std::sqrt(tol2 / rr));
      // inner: A32 d = r from d = 0, FP64 vectors
      rc = launch_fill<double>(w.d, 0.0, n, w.s);
      if (rc) return rc;
      rc = pcg_core(A32, dinv, w.d, irt * irt * rr, maxit - inf.inner_iterations, w, st);
      if (rc) return rc;
      inf.inner_iterations += st.iters;
      inf.fallbacks += st.nfallback;
      if (st.breakdown) {
        status = fail(MF_EBREAKDOWN, "inner CG breakdown (non-finite value or p'Ap <= 0)");
        break;
      }
      rc = cg_axpy(x, w.d, n, w.s);
      if (rc) return rc;
    }
  }
  if (x != x_user) {
    rc = launch_from_internal<double>(A64->perm.as<int32_t>(), A64->nnodes, A64->ncomp, x, x_user, false, w.s);
    if (rc) return rc;
  }
  inf.rel_residual = std::sqrt(rr / bb);
  if (status == MF_OK && !(rr == rr)) status = fail(MF_EBREAKDOWN, "non-finite residual");
  if (status == MF_OK && rr > tol2)
    status = fail(MF_ENOTCONV, "CG did not reach the tolerance within maxit iterations");
  MF_HIP(hipStreamSynchronize(w.s));
  if (info) *info = inf;
  return status;
}

size_t cg_workspace_bytes(const mf_op *A64, const mf_op *A32, const mf_precond *M) {
  CgWork w;
  const CgNeed need = cg_need(w, A64, A32, M);
  size_t tot = 0;
  for (int i = 0; i < 11; i++) tot += align256(need.bytes[i]);
  return tot;
}

int cg_solve_in(void *ws, size_t ws_bytes, const mf_op *A64, const mf_op *A32, const mf_precond *M,
                const double *b, double *x, double rtol, double inner_rtol, int maxit, mf_cg_info *info,
                hipStream_t s) {
  int rc = cg_check(A64, A32, M, b, x, rtol, maxit, "mf_cg_solve_noalloc");
  if (rc) return rc;
  if (M && M->kind != 0)
    return fail(MF_EUNSUPPORTED, "mf_cg_solve_noalloc: only the Jacobi preconditioner (or none) is supported");
  const size_t need_bytes = cg_workspace_bytes(A64, A32, M);
  if (need_bytes > ws_bytes)
    return fail(MF_EINVAL, "mf_cg_solve_noalloc: the solve needs " + std::to_string(need_bytes) +
                               " bytes of workspace, more than the " + std::to_string(ws_bytes) + " available");
  CgWork w;
  w.n = A64->ndofs;
  w.s = s;
  w.graphs = false;  // graph instantiation allocates; the chunks are launched directly
  w.host_st = &w.host_local;
  const CgNeed need = cg_need(w, A64, A32, M);
  char *base = (char *)ws;
  for (int i = 0; i < 11; i++) {
    *need.slot[i] = need.bytes[i] ? (void *)base : nullptr;
    base += align256(need.bytes[i]);
  }
  return cg_core(w, A64, A32, M, b, x, rtol, inner_rtol, maxit, info);
}

}  // namespace mf

using namespace mf;

extern "C" {

int mf_cg_solve(const mf_op *A64, const mf_op *A32, const mf_precond *M, const double *b, double *x, double rtol,
                double inner_rtol, int maxit, mf_cg_info *info, void *stream) {
  int rc = cg_check(A64, A32, M, b, x, rtol, maxit, "mf_cg_solve");
  if (rc) return rc;
  hipStream_t caller = (hipStream_t)stream;
  CgWork w;
  w.n = A64->ndofs;
  MF_HIP(hipStreamCreateWithFlags(&w.s, hipStreamNonBlocking));
  w.own_stream = true;
  MF_HIP(hipEventCreateWithFlags(&w.ev, hipEventDisableTiming));
  MF_HIP(hipHostMalloc((void **)&w.host_st, sizeof(CgState), hipHostMallocDefault));
  w.pinned = true;
  // order the solve after the caller's pending work on its stream
  MF_HIP(hipEventRecord(w.ev, caller));
  MF_HIP(hipStreamWaitEvent(w.s, w.ev, 0));
  if (M && M->kind == 1) w.M = M;
  const CgNeed need = cg_need(w, A64, A32, M);
  for (int i = 0; i < 11 && !rc; i++)
    if (need.bytes[i]) {
      rc = w.own[i].alloc(need.bytes[i]);
      *need.slot[i] = w.own[i].ptr;
    }
  if (rc) return rc;
  return cg_core(w, A64, A32, M, b, x, rtol, inner_rtol, maxit, info);
}

}  // extern "C"
