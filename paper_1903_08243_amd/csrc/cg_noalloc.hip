// CG solve for callers that cannot allocate device memory (code under stream
// capture elsewhere, serving loops, harnesses that forbid hipMalloc): the solver's
// vectors live in one fixed device array of this library instead of buffers
// allocated per solve.
//
// In host code `scratch` names a host-side stand-in, not the device array; its
// device address is taken once per device with hipGetSymbolAddress (each GPU holds
// its own copy) and only that address is passed to kernels.
#include <mutex>

#include "cg_internal.h"

namespace mf {

static __device__ __align__(256) unsigned char scratch[MF_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[64] = {};  // per device id, set on first use

static int scratch_for_current_device(void **out) {
  int dev = -1;
  MF_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(MF_EDEVICE, "mf_cg_solve_noalloc: device id out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(MF_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return MF_OK;
}

}  // namespace mf

using namespace mf;

extern "C" {

int mf_cg_solve_noalloc(const mf_op *A64, const mf_op *A32, const mf_precond *M, const double *b, double *x,
                        double rtol, double inner_rtol, int maxit, mf_cg_info *info, void *stream) {
  void *ws = nullptr;
  int rc = scratch_for_current_device(&ws);
  if (rc) return rc;
  return cg_solve_in(ws, MF_NOALLOC_SCRATCH_BYTES, A64, A32, M, b, x, rtol, inner_rtol, maxit, info,
                     (hipStream_t)stream);
}

}  // extern "C"
