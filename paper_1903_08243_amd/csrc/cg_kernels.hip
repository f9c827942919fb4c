// Device kernels of the conjugate-gradient solver (FP64 vectors).
//
// The scalars of the iteration (alpha, beta, r'z, r'r) live in device memory
// and are produced by one-block "finalize" kernels from fixed-size per-block
// partial sums, so the whole iteration is a fixed launch sequence (graph
// capturable, no host round trip) and every reduction is summed in the same
// order on every run (bit-reproducible). The operator output Ap may be FP32
// (inner solves of iterative refinement) and is widened on load.
#include "mf_internal.h"
#include "cg_internal.h"

namespace mf {

constexpr int RB = 256;  // threads per reduction block

__device__ __forceinline__ double block_sum(double v, double *sh) {
  // wavefront reduction by shuffles, then across the 4 wavefronts through LDS
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < RB / 64; i++) s += sh[i];
  __syncthreads();
  return s;
}

template <typename TA>
__global__ void __launch_bounds__(RB) residual_kernel(const double *__restrict__ b, const TA *__restrict__ Ax,
                                                      double *__restrict__ r, int64_t n, double *__restrict__ part) {
  __shared__ double sh[RB / 64];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB) {
    const double v = b[i] - (double)Ax[i];
    r[i] = v;
    s += v * v;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// z = M^{-1} r (dinv == null: identity), p = z (and its FP32 copy), partials r'z and r'r.
__global__ void __launch_bounds__(RB) init_p_kernel(const double *__restrict__ r, const double *__restrict__ dinv,
                                                    double *__restrict__ p, float *__restrict__ p32, int64_t n,
                                                    double *__restrict__ part, void *__restrict__ ap_zero) {
  __shared__ double sh[RB / 64];
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB) {
    const double ri = r[i];
    const double z = dinv ? dinv[i] * ri : ri;
    p[i] = z;
    if (p32) {
      p32[i] = (float)z;
      if (ap_zero) ((float *)ap_zero)[i] = 0.0f;
    } else if (ap_zero) {
      ((double *)ap_zero)[i] = 0.0;
    }
    s1 += ri * z;
    s2 += ri * ri;
  }
  s1 = block_sum(s1, sh);
  s2 = block_sum(s2, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s1;
    part[gridDim.x + blockIdx.x] = s2;
  }
}

// partials of r'z (z = M^{-1} r) and r'r
__global__ void __launch_bounds__(RB) rz_kernel(const double *__restrict__ r, const double *__restrict__ dinv, int64_t n,
                                                double *__restrict__ part) {
  __shared__ double sh[RB / 64];
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB) {
    const double ri = r[i];
    s1 += ri * (dinv ? dinv[i] * ri : ri);
    s2 += ri * ri;
  }
  s1 = block_sum(s1, sh);
  s2 = block_sum(s2, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s1;
    part[gridDim.x + blockIdx.x] = s2;
  }
}

template <typename TA>
__global__ void __launch_bounds__(RB) dot_kernel(const double *__restrict__ a, const TA *__restrict__ b, int64_t n,
                                                 double *__restrict__ part) {
  __shared__ double sh[RB / 64];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB)
    s += a[i] * (double)b[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// x += alpha p; r -= alpha Ap; partial sums of r'z and r'r with z = M^{-1} r.
template <typename TA>
__global__ void __launch_bounds__(RB) update_kernel(double *__restrict__ x, double *__restrict__ r,
                                                    const double *__restrict__ p, const TA *__restrict__ Ap,
                                                    const double *__restrict__ dinv, const CgState *__restrict__ st,
                                                    int64_t n, double *__restrict__ part) {
  __shared__ double sh[RB / 64];
  const double alpha = st->alpha;
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB) {
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * (double)Ap[i];
    r[i] = ri;
    const double zi = dinv ? dinv[i] * ri : ri;
    s1 += ri * zi;
    s2 += ri * ri;
  }
  s1 = block_sum(s1, sh);
  s2 = block_sum(s2, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s1;
    part[gridDim.x + blockIdx.x] = s2;
  }
}

// p = M^{-1} r + beta p (and the FP32 copy for the next FP32 action); the output of
// the next (accumulating) action is cleared in the same pass
__global__ void __launch_bounds__(RB) p_update_kernel(double *__restrict__ p, float *__restrict__ p32,
                                                      const double *__restrict__ r, const double *__restrict__ dinv,
                                                      const CgState *__restrict__ st, int64_t n,
                                                      void *__restrict__ ap_zero) {
  const double beta = st->beta;
  for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB) {
    const double z = dinv ? dinv[i] * r[i] : r[i];
    const double v = z + beta * p[i];
    p[i] = v;
    if (p32) {
      p32[i] = (float)v;
      ((float *)ap_zero)[i] = 0.0f;
    } else {
      ((double *)ap_zero)[i] = 0.0;
    }
  }
}

__global__ void axpy_kernel(double *__restrict__ x, const double *__restrict__ d, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB) x[i] += d[i];
}

template <typename TS>
__global__ void recip_kernel(const TS *__restrict__ d, double *__restrict__ dinv, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB)
    dinv[i] = 1.0 / (double)d[i];
}

__global__ void cast_kernel(const double *__restrict__ a, float *__restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB) b[i] = (float)a[i];
}

__global__ void sqrt_kernel(const double *__restrict__ a, double *__restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB) b[i] = sqrt(a[i]);
}

__global__ void scale_kernel(const double *__restrict__ d, const double *__restrict__ a, double *__restrict__ b,
                             int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB) b[i] = d[i] * a[i];
}

// ---- flexible CG
// x += alpha p; r -= alpha Ap; partial r'r
template <typename TA>
__global__ void __launch_bounds__(RB) fupdate_kernel(double *__restrict__ x, double *__restrict__ r,
                                                     const double *__restrict__ p, const TA *__restrict__ Ap,
                                                     const CgState *__restrict__ st, int64_t n,
                                                     double *__restrict__ part) {
  __shared__ double sh[RB / 64];
  if (st->stop) return;  // uniform; p may hold an unused direction after convergence
  const double alpha = st->alpha;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB) {
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * (double)Ap[i];
    r[i] = ri;
    s += ri * ri;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// partials of z'r, z'Ap (0 without Ap), the number of non-finite z, and r'r
template <typename TA>
__global__ void __launch_bounds__(RB) zdot_kernel(const double *__restrict__ z, const double *__restrict__ r,
                                                  const TA *__restrict__ Ap, int64_t n, double *__restrict__ part) {
  __shared__ double sh[RB / 64];
  double s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB) {
    const double zi = z[i], ri = r[i];
    const bool fin = zi - zi == 0.0;
    s3 += fin ? 0.0 : 1.0;
    const double zf = fin ? zi : 0.0;
    s1 += zf * ri;
    if (Ap) s2 += zf * (double)Ap[i];
    s4 += ri * ri;
  }
  s1 = block_sum(s1, sh);
  s2 = block_sum(s2, sh);
  s3 = block_sum(s3, sh);
  s4 = block_sum(s4, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s1;
    part[gridDim.x + blockIdx.x] = s2;
    part[2 * gridDim.x + blockIdx.x] = s3;
    part[3 * gridDim.x + blockIdx.x] = s4;
  }
}

// when the state flags a fallback: z = D^{-1} r and partials of z'r, z'Ap; otherwise nothing
template <typename TA>
__global__ void __launch_bounds__(RB) zfix_kernel(double *__restrict__ z, const double *__restrict__ r,
                                                  const double *__restrict__ dinv, const TA *__restrict__ Ap,
                                                  const CgState *__restrict__ st, int64_t n,
                                                  double *__restrict__ part) {
  __shared__ double sh[RB / 64];
  if (!st->fallback || st->stop) return;  // uniform over the grid
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB) {
    const double ri = r[i];
    const double zi = dinv ? dinv[i] * ri : ri;
    z[i] = zi;
    s1 += zi * ri;
    if (Ap) s2 += zi * (double)Ap[i];
  }
  s1 = block_sum(s1, sh);
  s2 = block_sum(s2, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s1;
    part[gridDim.x + blockIdx.x] = s2;
  }
}

// p = z + beta p (first direction: p = z), FP32 copy, next action's output cleared
__global__ void __launch_bounds__(RB) fp_update_kernel(double *__restrict__ p, float *__restrict__ p32,
                                                       const double *__restrict__ z, const CgState *__restrict__ st,
                                                       int64_t n, void *__restrict__ ap_zero, int first) {
  if (!first && st->stop) return;  // uniform: keep the last direction once converged
  const double beta = st->beta;
  for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB) {
    const double v = first ? z[i] : z[i] + beta * p[i];
    p[i] = v;
    if (p32) {
      p32[i] = (float)v;
      if (ap_zero) ((float *)ap_zero)[i] = 0.0f;
    } else if (ap_zero) {
      ((double *)ap_zero)[i] = 0.0;
    }
  }
}

// One-block finalize: sums the partials in a fixed order and advances the state.
__global__ void __launch_bounds__(RB) finalize_kernel(const double *__restrict__ part, int nparts, CgState *st,
                                                      int stage) {
  __shared__ double sh[RB / 64];
  const int nsum = (stage == CG_STAGE_FZ || stage == CG_STAGE_FINIT)                               ? 4
                   : (stage == CG_STAGE_UPDATE || stage == CG_STAGE_INIT || stage == CG_STAGE_FZFIX ||
                      stage == CG_STAGE_RELIABLE)                                                   ? 2
                                                                                                     : 1;
  CgState S;
  if (threadIdx.x == 0) S = *st;  // issued together with the partial loads below
  double tot[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = 0; k < nsum; k++) {
    double s = 0.0;
    for (int i = threadIdx.x; i < nparts; i += RB) s += part[k * nparts + i];
    tot[k] = block_sum(s, sh);
  }
  if (threadIdx.x != 0) return;
  switch (stage) {
    case CG_STAGE_RESIDUAL:  // tot0 = r'r
      S.rr = tot[0];
      break;
    case CG_STAGE_INIT:  // tot0 = r'z, tot1 = r'r
      S.rz = tot[0];
      S.rr = tot[1];
      S.iters = 0;
      S.stop = (S.rr <= S.tol2) ? 1 : 0;
      S.breakdown = 0;
      if (!(S.rr == S.rr) || !(S.rz == S.rz) || S.rz < 0.0) S.stop = S.breakdown = 1;
      break;
    case CG_STAGE_RELIABLE:  // tot0 = r'z, tot1 = r'r of the true residual; p and iters kept
      S.rz = tot[0];
      S.rr = tot[1];
      S.breakdown = 0;
      S.stop = (S.rr <= S.tol2 || S.iters >= S.maxit) ? 1 : 0;
      if (!(S.rr == S.rr) || !(S.rz == S.rz) || S.rz < 0.0) S.stop = S.breakdown = 1;
      break;
    case CG_STAGE_PAP: {  // tot0 = p'Ap
      S.pAp = tot[0];
      if (S.stop) {
        S.alpha = 0.0;
      } else if (!(S.pAp > 0.0) || !(S.pAp < 1e308)) {
        S.alpha = 0.0;
        S.stop = S.breakdown = 1;
      } else {
        S.alpha = S.rz / S.pAp;
      }
      break;
    }
    case CG_STAGE_UPDATE: {  // tot0 = r'z (new), tot1 = r'r
      if (S.stop) {
        S.beta = 0.0;
        break;
      }
      const double rz_new = tot[0];
      S.rr = tot[1];
      S.iters += 1;
      if (!(S.rr == S.rr) || !(rz_new == rz_new)) {
        S.stop = S.breakdown = 1;
        S.beta = 0.0;
        break;
      }
      S.beta = rz_new / S.rz;
      S.rz = rz_new;
      if (S.rr <= S.tol2 || S.iters >= S.maxit) S.stop = 1;
      break;
    }
    case CG_STAGE_FUPDATE: {  // tot0 = r'r
      if (S.stop) break;
      S.rr = tot[0];
      S.iters += 1;
      if (!(S.rr == S.rr)) {
        S.stop = S.breakdown = 1;
        break;
      }
      if (S.rr <= S.tol2 || S.iters >= S.maxit) S.stop = 1;
      break;
    }
    case CG_STAGE_FINIT:  // tot0 = z'r, tot2 = non-finite z count, tot3 = r'r
      S.rr = tot[3];
      S.iters = 0;
      S.alpha = 0.0;
      S.beta = 0.0;
      S.breakdown = 0;
      S.nfallback = 0;
      S.stop = (S.rr <= S.tol2) ? 1 : 0;
      if (!(S.rr == S.rr)) S.stop = S.breakdown = 1;
      [[fallthrough]];  // then the check of z
    case CG_STAGE_FZ: {  // tot0 = z'r, tot1 = z'Ap, tot2 = non-finite z count
      if (S.stop) {
        S.fallback = 0;
        S.beta = 0.0;
        break;
      }
      const bool bad = tot[2] > 0.0 || !(tot[0] > 0.0) || !(tot[0] < 1e308);
      S.fallback = bad ? 1 : 0;
      if (bad) {
        S.nfallback += 1;
      } else {
        S.beta = stage == CG_STAGE_FINIT ? 0.0 : -S.alpha * tot[1] / S.rz;
        S.rz = tot[0];
      }
      break;
    }
    case CG_STAGE_FZFIX: {  // only after a fallback pass: tot0 = z'r, tot1 = z'Ap of the Jacobi z
      if (S.stop || !S.fallback) break;
      if (!(tot[0] > 0.0) || !(tot[0] < 1e308) || !(tot[1] == tot[1])) {
        S.stop = S.breakdown = 1;
        S.beta = 0.0;
        break;
      }
      S.beta = S.iters == 0 ? 0.0 : -S.alpha * tot[1] / S.rz;
      S.rz = tot[0];
      break;
    }
  }
  *st = S;
}

// ------------------------------------------------------------------ launchers
static unsigned grid_n(int64_t n) {
  int64_t g = (n + RB - 1) / RB;
  return (unsigned)(g < 1 ? 1 : (g > CG_NPART ? CG_NPART : g));
}

int cg_residual(const double *b, const void *Ax, bool ax32, double *r, int64_t n, double *part, CgState *st,
                hipStream_t s) {
  const unsigned g = grid_n(n);
  if (ax32) residual_kernel<float><<<g, RB, 0, s>>>(b, (const float *)Ax, r, n, part);
  else residual_kernel<double><<<g, RB, 0, s>>>(b, (const double *)Ax, r, n, part);
  finalize_kernel<<<1, RB, 0, s>>>(part, (int)g, st, CG_STAGE_RESIDUAL);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

int cg_init(const double *r, const double *dinv, double *p, float *p32, int64_t n, double *part, CgState *st,
            hipStream_t s, void *ap_zero) {
  const unsigned g = grid_n(n);
  init_p_kernel<<<g, RB, 0, s>>>(r, dinv, p, p32, n, part, ap_zero);
  finalize_kernel<<<1, RB, 0, s>>>(part, (int)g, st, CG_STAGE_INIT);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

int cg_step_after_apply(double *x, double *r, double *p, float *p32, void *Ap, bool ap32, const double *dinv,
                        int64_t n, double *part, CgState *st, hipStream_t s) {
  const unsigned g = grid_n(n);
  if (ap32) dot_kernel<float><<<g, RB, 0, s>>>(p, (const float *)Ap, n, part);
  else dot_kernel<double><<<g, RB, 0, s>>>(p, (const double *)Ap, n, part);
  finalize_kernel<<<1, RB, 0, s>>>(part, (int)g, st, CG_STAGE_PAP);
  if (ap32) update_kernel<float><<<g, RB, 0, s>>>(x, r, p, (const float *)Ap, dinv, st, n, part);
  else update_kernel<double><<<g, RB, 0, s>>>(x, r, p, (const double *)Ap, dinv, st, n, part);
  finalize_kernel<<<1, RB, 0, s>>>(part, (int)g, st, CG_STAGE_UPDATE);
  p_update_kernel<<<g, RB, 0, s>>>(p, p32, r, dinv, st, n, Ap);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

int cg_reliable(const double *r, const double *dinv, int64_t n, double *part, CgState *st, hipStream_t s) {
  const unsigned g = grid_n(n);
  rz_kernel<<<g, RB, 0, s>>>(r, dinv, n, part);
  finalize_kernel<<<1, RB, 0, s>>>(part, (int)g, st, CG_STAGE_RELIABLE);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

int cg_axpy(double *x, const double *d, int64_t n, hipStream_t s) {
  axpy_kernel<<<grid_n(n), RB, 0, s>>>(x, d, n);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

int cg_recip(const void *d, bool d32, double *dinv, int64_t n, hipStream_t s) {
  if (d32) recip_kernel<float><<<grid_n(n), RB, 0, s>>>((const float *)d, dinv, n);
  else recip_kernel<double><<<grid_n(n), RB, 0, s>>>((const double *)d, dinv, n);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

int cg_sqrt(const double *a, double *b, int64_t n, hipStream_t s) {
  sqrt_kernel<<<grid_n(n), RB, 0, s>>>(a, b, n);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

int cg_scale(const double *d, const double *a, double *b, int64_t n, hipStream_t s) {
  scale_kernel<<<grid_n(n), RB, 0, s>>>(d, a, b, n);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

int fcg_init(const double *r, double *z, const double *dinv, double *p, float *p32, int64_t n, double *part,
             CgState *st, hipStream_t s, void *ap_zero) {
  const unsigned g = grid_n(n);
  zdot_kernel<double><<<g, RB, 0, s>>>(z, r, nullptr, n, part);
  finalize_kernel<<<1, RB, 0, s>>>(part, (int)g, st, CG_STAGE_FINIT);
  zfix_kernel<double><<<g, RB, 0, s>>>(z, r, dinv, nullptr, st, n, part);
  finalize_kernel<<<1, RB, 0, s>>>(part, (int)g, st, CG_STAGE_FZFIX);
  fp_update_kernel<<<g, RB, 0, s>>>(p, p32, z, st, n, ap_zero, 1);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

int fcg_update(double *x, double *r, const double *p, const void *Ap, bool ap32, int64_t n, double *part,
               CgState *st, hipStream_t s) {
  const unsigned g = grid_n(n);
  if (ap32) dot_kernel<float><<<g, RB, 0, s>>>(p, (const float *)Ap, n, part);
  else dot_kernel<double><<<g, RB, 0, s>>>(p, (const double *)Ap, n, part);
  finalize_kernel<<<1, RB, 0, s>>>(part, (int)g, st, CG_STAGE_PAP);
  if (ap32) fupdate_kernel<float><<<g, RB, 0, s>>>(x, r, p, (const float *)Ap, st, n, part);
  else fupdate_kernel<double><<<g, RB, 0, s>>>(x, r, p, (const double *)Ap, st, n, part);
  finalize_kernel<<<1, RB, 0, s>>>(part, (int)g, st, CG_STAGE_FUPDATE);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

int fcg_direction(const double *r, double *z, const double *dinv, double *p, float *p32, void *Ap, bool ap32,
                  int64_t n, double *part, CgState *st, hipStream_t s) {
  const unsigned g = grid_n(n);
  if (ap32) zdot_kernel<float><<<g, RB, 0, s>>>(z, r, (const float *)Ap, n, part);
  else zdot_kernel<double><<<g, RB, 0, s>>>(z, r, (const double *)Ap, n, part);
  finalize_kernel<<<1, RB, 0, s>>>(part, (int)g, st, CG_STAGE_FZ);
  if (ap32) zfix_kernel<float><<<g, RB, 0, s>>>(z, r, dinv, (const float *)Ap, st, n, part);
  else zfix_kernel<double><<<g, RB, 0, s>>>(z, r, dinv, (const double *)Ap, st, n, part);
  finalize_kernel<<<1, RB, 0, s>>>(part, (int)g, st, CG_STAGE_FZFIX);
  fp_update_kernel<<<g, RB, 0, s>>>(p, p32, z, st, n, Ap, 0);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

int cg_cast(const double *a, float *b, int64_t n, hipStream_t s) {
  cast_kernel<<<grid_n(n), RB, 0, s>>>(a, b, n);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

}  // namespace mf
