// Vector kernels of the batched conjugate-gradient solver.
//
// The vectors of all systems of a batch are concatenated; a chunk table splits
// them into pieces that each belong to one system. Every kernel runs one
// workgroup per chunk and writes per-chunk partial sums; a one-thread-per-system
// finalize kernel adds each system's partials in chunk order (deterministic)
// and advances that system's CG state (same state machine as the single solve).
#include "batch_internal.h"

namespace mf {

constexpr int BR = 256;

__device__ __forceinline__ double bsum(double v, double *sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < BR / 64; i++) s += sh[i];
  __syncthreads();
  return s;
}

template <typename TA>
__global__ void __launch_bounds__(BR) bresid_kernel(const double *__restrict__ b, const TA *__restrict__ Ax,
                                                    double *__restrict__ r, const VChunk *__restrict__ ch,
                                                    double *__restrict__ part) {
  __shared__ double sh[BR / 64];
  const VChunk c = ch[blockIdx.x];
  double s = 0.0;
  for (int64_t i = c.start + threadIdx.x; i < c.start + c.len; i += BR) {
    const double v = b[i] - (double)Ax[i];
    r[i] = v;
    s += v * v;
  }
  s = bsum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(BR) binit_kernel(const double *__restrict__ r, const double *__restrict__ dinv,
                                                   double *__restrict__ p, float *__restrict__ p32,
                                                   const VChunk *__restrict__ ch, int nch, double *__restrict__ part) {
  __shared__ double sh[BR / 64];
  const VChunk c = ch[blockIdx.x];
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i = c.start + threadIdx.x; i < c.start + c.len; i += BR) {
    const double ri = r[i];
    const double z = dinv ? dinv[i] * ri : ri;
    p[i] = z;
    if (p32) p32[i] = (float)z;
    s1 += ri * z;
    s2 += ri * ri;
  }
  s1 = bsum(s1, sh);
  s2 = bsum(s2, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s1;
    part[nch + blockIdx.x] = s2;
  }
}

template <typename TA>
__global__ void __launch_bounds__(BR) bdot_kernel(const double *__restrict__ p, const TA *__restrict__ Ap,
                                                  const VChunk *__restrict__ ch, const CgState *__restrict__ st,
                                                  double *__restrict__ part) {
  __shared__ double sh[BR / 64];
  const VChunk c = ch[blockIdx.x];
  double s = 0.0;
  if (!st[c.sys].stop)
    for (int64_t i = c.start + threadIdx.x; i < c.start + c.len; i += BR) s += p[i] * (double)Ap[i];
  s = bsum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

template <typename TA>
__global__ void __launch_bounds__(BR) bupdate_kernel(double *__restrict__ x, double *__restrict__ r,
                                                     const double *__restrict__ p, const TA *__restrict__ Ap,
                                                     const double *__restrict__ dinv, const CgState *__restrict__ st,
                                                     const VChunk *__restrict__ ch, int nch,
                                                     double *__restrict__ part) {
  __shared__ double sh[BR / 64];
  const VChunk c = ch[blockIdx.x];
  const double alpha = st[c.sys].alpha;
  const bool live = !st[c.sys].stop;
  double s1 = 0.0, s2 = 0.0;
  if (live)
    for (int64_t i = c.start + threadIdx.x; i < c.start + c.len; i += BR) {
      x[i] += alpha * p[i];
      const double ri = r[i] - alpha * (double)Ap[i];
      r[i] = ri;
      const double zi = dinv ? dinv[i] * ri : ri;
      s1 += ri * zi;
      s2 += ri * ri;
    }
  s1 = bsum(s1, sh);
  s2 = bsum(s2, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s1;
    part[nch + blockIdx.x] = s2;
  }
}

__global__ void __launch_bounds__(BR) bpupdate_kernel(double *__restrict__ p, float *__restrict__ p32,
                                                      const double *__restrict__ r, const double *__restrict__ dinv,
                                                      const CgState *__restrict__ st, const VChunk *__restrict__ ch) {
  const VChunk c = ch[blockIdx.x];
  if (st[c.sys].stop) return;
  const double beta = st[c.sys].beta;
  for (int64_t i = c.start + threadIdx.x; i < c.start + c.len; i += BR) {
    const double z = dinv ? dinv[i] * r[i] : r[i];
    const double v = z + beta * p[i];
    p[i] = v;
    if (p32) p32[i] = (float)v;
  }
}

__global__ void baxpy_kernel(double *__restrict__ x, const double *__restrict__ d, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * BR + threadIdx.x; i < n; i += (int64_t)gridDim.x * BR) x[i] += d[i];
}

// One workgroup per system: its chunk partials are summed in a fixed order (a
// strided pass per thread, then a fixed reduction tree), and thread 0 advances the
// system's state.
__global__ void __launch_bounds__(BR) bfinalize_kernel(const double *__restrict__ part, int nch,
                                                       const int32_t *__restrict__ cptr, CgState *st, int nsys,
                                                       int stage) {
  __shared__ double sh[BR / 64];
  const int s = blockIdx.x;
  if (s >= nsys) return;  // uniform over the workgroup
  const bool two = stage == CG_STAGE_UPDATE || stage == CG_STAGE_INIT || stage == CG_STAGE_RELIABLE;
  double a = 0.0, b = 0.0;
  for (int c = cptr[s] + threadIdx.x; c < cptr[s + 1]; c += BR) {
    a += part[c];
    if (two) b += part[nch + c];
  }
  const double t0 = bsum(a, sh);
  const double t1 = two ? bsum(b, sh) : 0.0;
  if (threadIdx.x != 0) return;
  CgState S = st[s];
  switch (stage) {
    case CG_STAGE_RESIDUAL:
      S.rr = t0;
      break;
    case CG_STAGE_INIT:
      S.rz = t0;
      S.rr = t1;
      S.iters = 0;
      S.stop = (S.rr <= S.tol2) ? 1 : 0;
      S.breakdown = 0;
      if (!(S.rr == S.rr) || !(S.rz == S.rz) || S.rz < 0.0) S.stop = S.breakdown = 1;
      break;
    case CG_STAGE_RELIABLE:  // the true residual replaced r: r'z, r'r; p and iters kept
      S.rz = t0;
      S.rr = t1;
      S.breakdown = 0;
      S.stop = (S.rr <= S.tol2 || S.iters >= S.maxit) ? 1 : 0;
      if (!(S.rr == S.rr) || !(S.rz == S.rz) || S.rz < 0.0) S.stop = S.breakdown = 1;
      break;
    case CG_STAGE_PAP:
      S.pAp = t0;
      if (S.stop) {
        S.alpha = 0.0;
      } else if (!(S.pAp > 0.0) || !(S.pAp < 1e308)) {
        S.alpha = 0.0;
        S.stop = S.breakdown = 1;
      } else {
        S.alpha = S.rz / S.pAp;
      }
      break;
    case CG_STAGE_UPDATE: {
      if (S.stop) {
        S.beta = 0.0;
        break;
      }
      S.rr = t1;
      S.iters += 1;
      if (!(S.rr == S.rr) || !(t0 == t0)) {
        S.stop = S.breakdown = 1;
        S.beta = 0.0;
        break;
      }
      S.beta = t0 / S.rz;
      S.rz = t0;
      if (S.rr <= S.tol2 || S.iters >= S.maxit) S.stop = 1;
      break;
    }
  }
  st[s] = S;
}

template <typename T>
__global__ void __launch_bounds__(BR) bfill_kernel(T *__restrict__ y, const VChunk *__restrict__ ch,
                                                   const CgState *__restrict__ st) {
  const VChunk c = ch[blockIdx.x];
  if (st[c.sys].stop) return;
  for (int64_t i = c.start + threadIdx.x; i < c.start + c.len; i += BR) y[i] = T(0);
}

// ------------------------------------------------------------------ launchers
template <typename T> int batch_fill(const BatchVec &v, T *y, const CgState *st, hipStream_t s) {
  bfill_kernel<T><<<v.nch, BR, 0, s>>>(y, v.chunks, st);
  MF_HIP(hipGetLastError());
  return MF_OK;
}
template int batch_fill<double>(const BatchVec &, double *, const CgState *, hipStream_t);
template int batch_fill<float>(const BatchVec &, float *, const CgState *, hipStream_t);

static int fin(const BatchVec &v, CgState *st, int stage, hipStream_t s) {
  bfinalize_kernel<<<v.nsys, BR, 0, s>>>(v.part, v.nch, v.cptr, st, v.nsys, stage);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

int batch_residual(const BatchVec &v, const double *b, const void *Ax, bool ax32, double *r, CgState *st,
                   hipStream_t s) {
  if (ax32) bresid_kernel<float><<<v.nch, BR, 0, s>>>(b, (const float *)Ax, r, v.chunks, v.part);
  else bresid_kernel<double><<<v.nch, BR, 0, s>>>(b, (const double *)Ax, r, v.chunks, v.part);
  MF_HIP(hipGetLastError());
  return fin(v, st, CG_STAGE_RESIDUAL, s);
}

int batch_init(const BatchVec &v, const double *r, const double *dinv, double *p, float *p32, CgState *st,
               hipStream_t s) {
  binit_kernel<<<v.nch, BR, 0, s>>>(r, dinv, p, p32, v.chunks, v.nch, v.part);
  MF_HIP(hipGetLastError());
  return fin(v, st, CG_STAGE_INIT, s);
}

// partials of r'z (z = M^{-1} r) and r'r per chunk
__global__ void __launch_bounds__(BR) brz_kernel(const double *__restrict__ r, const double *__restrict__ dinv,
                                                 const VChunk *__restrict__ ch, int nch, double *__restrict__ part) {
  __shared__ double sh[BR / 64];
  const VChunk c = ch[blockIdx.x];
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i = c.start + threadIdx.x; i < c.start + c.len; i += BR) {
    const double ri = r[i];
    s1 += ri * (dinv ? dinv[i] * ri : ri);
    s2 += ri * ri;
  }
  s1 = bsum(s1, sh);
  s2 = bsum(s2, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s1;
    part[nch + blockIdx.x] = s2;
  }
}

int batch_reliable(const BatchVec &v, const double *r, const double *dinv, CgState *st, hipStream_t s) {
  brz_kernel<<<v.nch, BR, 0, s>>>(r, dinv, v.chunks, v.nch, v.part);
  MF_HIP(hipGetLastError());
  return fin(v, st, CG_STAGE_RELIABLE, s);
}

int batch_step_after_apply(const BatchVec &v, double *x, double *r, double *p, float *p32, const void *Ap, bool ap32,
                           const double *dinv, CgState *st, hipStream_t s) {
  if (ap32) bdot_kernel<float><<<v.nch, BR, 0, s>>>(p, (const float *)Ap, v.chunks, st, v.part);
  else bdot_kernel<double><<<v.nch, BR, 0, s>>>(p, (const double *)Ap, v.chunks, st, v.part);
  MF_HIP(hipGetLastError());
  int rc = fin(v, st, CG_STAGE_PAP, s);
  if (rc) return rc;
  if (ap32) bupdate_kernel<float><<<v.nch, BR, 0, s>>>(x, r, p, (const float *)Ap, dinv, st, v.chunks, v.nch, v.part);
  else bupdate_kernel<double><<<v.nch, BR, 0, s>>>(x, r, p, (const double *)Ap, dinv, st, v.chunks, v.nch, v.part);
  MF_HIP(hipGetLastError());
  rc = fin(v, st, CG_STAGE_UPDATE, s);
  if (rc) return rc;
  bpupdate_kernel<<<v.nch, BR, 0, s>>>(p, p32, r, dinv, st, v.chunks);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

int batch_axpy(double *x, const double *d, int64_t n, hipStream_t s) {
  int64_t g = (n + BR - 1) / BR;
  if (g > 8192) g = 8192;
  baxpy_kernel<<<(unsigned)(g < 1 ? 1 : g), BR, 0, s>>>(x, d, n);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

}  // namespace mf
