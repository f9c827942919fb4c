// Batched solver internals shared by the driver and its kernels.
#pragma once
#include "cg_internal.h"

namespace mf {

struct VChunk {  // a piece of the concatenated vectors belonging to one system
  int32_t sys, pad;
  int64_t start, len;
};

struct BatchVec {  // device-side description of the concatenated vectors
  const VChunk *chunks;
  int nch;
  const int32_t *cptr;  // chunks of system s: [cptr[s], cptr[s+1])
  int nsys;
  double *part;  // 2 * nch partial sums
};

int batch_residual(const BatchVec &v, const double *b, const void *Ax, bool ax32, double *r, CgState *st,
                   hipStream_t s);
int batch_init(const BatchVec &v, const double *r, const double *dinv, double *p, float *p32, CgState *st,
               hipStream_t s);
int batch_step_after_apply(const BatchVec &v, double *x, double *r, double *p, float *p32, const void *Ap, bool ap32,
                           const double *dinv, CgState *st, hipStream_t s);
int batch_axpy(double *x, const double *d, int64_t n, hipStream_t s);
// reliable update of every system: r'z and r'r of the replaced residual, p and iters kept
int batch_reliable(const BatchVec &v, const double *r, const double *dinv, CgState *st, hipStream_t s);
// y = 0 on the chunks of systems that have not stopped
template <typename T> int batch_fill(const BatchVec &v, T *y, const CgState *st, hipStream_t s);

}  // namespace mf
