// Small vector kernels used around the operator action: clearing the output
// (a fill kernel rather than a memset, so the sequence stays graph-capturable),
// and the rows of constrained (Dirichlet) degrees of freedom.
#include "mf_internal.h"

namespace mf {

template <typename T> __global__ void fill_kernel(T *__restrict__ y, T v, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) y[i] = v;
}

template <typename T>
__global__ void copy_constrained_kernel(const int32_t *__restrict__ dofs, int64_t n, const T *__restrict__ x,
                                        T *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[dofs[i]] = x[dofs[i]];
}

template <typename T>
__global__ void set_constrained_kernel(const int32_t *__restrict__ dofs, int64_t n, T v, T *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[dofs[i]] = v;
}

template <typename T>
__global__ void to_internal_kernel(const int32_t *__restrict__ uoi, int64_t nnodes, int nc, const T *__restrict__ xu,
                                   T *__restrict__ xi) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nnodes) return;
  const int64_t u = uoi[i];
  for (int c = 0; c < nc; c++) xi[i * nc + c] = xu[u * nc + c];
}

template <typename T>
__global__ void from_internal_kernel(const int32_t *__restrict__ uoi, int64_t nnodes, int nc, const T *__restrict__ yi,
                                     T *__restrict__ yu, bool acc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nnodes) return;
  const int64_t u = uoi[i];
  for (int c = 0; c < nc; c++) {
    const T v = yi[i * nc + c];
    yu[u * nc + c] = acc ? yu[u * nc + c] + v : v;
  }
}

// The same permutation as a gather over user nodes: random reads, sequential writes
// (random partial-line writes cost more than random reads).
template <typename T>
__global__ void from_internal_gather_kernel(const int32_t *__restrict__ iou, int64_t nnodes, int nc,
                                            const T *__restrict__ yi, T *__restrict__ yu, bool acc) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= nnodes) return;
  const int64_t i = iou[u];
  for (int c = 0; c < nc; c++) {
    const T v = yi[i * nc + c];
    yu[u * nc + c] = acc ? yu[u * nc + c] + v : v;
  }
}

static unsigned grid_for(int64_t n, int block, int64_t cap) {
  int64_t g = (n + block - 1) / block;
  if (g > cap) g = cap;
  return (unsigned)(g < 1 ? 1 : g);
}

template <typename T> int launch_fill(T *y, T v, int64_t n, hipStream_t s) {
  if (n <= 0) return MF_OK;
  fill_kernel<T><<<grid_for(n, 256, 8192), 256, 0, s>>>(y, v, n);
  MF_HIP(hipGetLastError());
  return MF_OK;
}
template <typename T> int launch_copy_constrained(const int32_t *dofs, int64_t n, const T *x, T *y, hipStream_t s) {
  if (n <= 0) return MF_OK;
  copy_constrained_kernel<T><<<grid_for(n, 256, 1ll << 30), 256, 0, s>>>(dofs, n, x, y);
  MF_HIP(hipGetLastError());
  return MF_OK;
}
template <typename T> int launch_set_constrained(const int32_t *dofs, int64_t n, T v, T *y, hipStream_t s) {
  if (n <= 0) return MF_OK;
  set_constrained_kernel<T><<<grid_for(n, 256, 1ll << 30), 256, 0, s>>>(dofs, n, v, y);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

template <typename T>
int launch_to_internal(const int32_t *uoi, int64_t nnodes, int nc, const T *xu, T *xi, hipStream_t s) {
  if (nnodes <= 0) return MF_OK;
  to_internal_kernel<T><<<grid_for(nnodes, 256, 1ll << 30), 256, 0, s>>>(uoi, nnodes, nc, xu, xi);
  MF_HIP(hipGetLastError());
  return MF_OK;
}
template <typename T>
int launch_from_internal(const int32_t *uoi, int64_t nnodes, int nc, const T *yi, T *yu, bool acc, hipStream_t s) {
  if (nnodes <= 0) return MF_OK;
  from_internal_kernel<T><<<grid_for(nnodes, 256, 1ll << 30), 256, 0, s>>>(uoi, nnodes, nc, yi, yu, acc);
  MF_HIP(hipGetLastError());
  return MF_OK;
}
template <typename T>
int launch_from_internal_gather(const int32_t *iou, int64_t nnodes, int nc, const T *yi, T *yu, bool acc,
                                hipStream_t s) {
  if (nnodes <= 0) return MF_OK;
  from_internal_gather_kernel<T><<<grid_for(nnodes, 256, 1ll << 30), 256, 0, s>>>(iou, nnodes, nc, yi, yu, acc);
  MF_HIP(hipGetLastError());
  return MF_OK;
}
template int launch_from_internal_gather<double>(const int32_t *, int64_t, int, const double *, double *, bool,
                                                 hipStream_t);
template int launch_from_internal_gather<float>(const int32_t *, int64_t, int, const float *, float *, bool,
                                                hipStream_t);
template int launch_to_internal<double>(const int32_t *, int64_t, int, const double *, double *, hipStream_t);
template int launch_to_internal<float>(const int32_t *, int64_t, int, const float *, float *, hipStream_t);
template int launch_from_internal<double>(const int32_t *, int64_t, int, const double *, double *, bool, hipStream_t);
template int launch_from_internal<float>(const int32_t *, int64_t, int, const float *, float *, bool, hipStream_t);

template int launch_fill<double>(double *, double, int64_t, hipStream_t);
template int launch_fill<float>(float *, float, int64_t, hipStream_t);
template int launch_copy_constrained<double>(const int32_t *, int64_t, const double *, double *, hipStream_t);
template int launch_copy_constrained<float>(const int32_t *, int64_t, const float *, float *, hipStream_t);
template int launch_set_constrained<double>(const int32_t *, int64_t, double, double *, hipStream_t);
template int launch_set_constrained<float>(const int32_t *, int64_t, float, float *, hipStream_t);

}  // namespace mf
