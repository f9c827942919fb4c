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

// Two-stage permutation out[i] = in[src[i]] for a random src (the user <-> internal
// node numbering). A single pass reads or writes at random, one L2 request per
// element. Stage 1 reads `in` in order and streams each element into the bucket of
// its destination (buckets of kPermBucket consecutive destinations, filled in source
// order, so every bucket is written front to back); stage 2 gives each bucket to one
// workgroup, which loads it into LDS with coalesced reads, permutes it there and
// writes its range of `out` in order. Work is one lane per value (node, component),
// so the components of a node are moved by neighbouring lanes as one contiguous run.
// Blocks are mapped so that each XCD takes a contiguous range (workgroup w runs on
// XCD w % 8).
__device__ __forceinline__ int64_t vec_xcd_block(int64_t w, int64_t nb) {
  const int64_t per = (nb + 7) / 8;
  return (w % 8) * per + w / 8;
}

template <typename T, int NC>
__global__ void __launch_bounds__(256) perm_stage1_kernel(const int32_t *__restrict__ pos1, int64_t n,
                                                          const T *__restrict__ in, T *__restrict__ tmp, int64_t nblk) {
  const int64_t b = vec_xcd_block(blockIdx.x, nblk);
  const int64_t v = b * 256 + threadIdx.x;
  if (b >= nblk || v >= n * NC) return;
  const int64_t j = v / NC;
  const int c = (int)(v - j * NC);
  tmp[(int64_t)pos1[j] * NC + c] = in[v];
}

constexpr int kPermThreads = 1024;
template <typename T, int NC>
__global__ void __launch_bounds__(kPermThreads) perm_stage2_kernel(const int32_t *__restrict__ pos2, int64_t n,
                                                                   const T *__restrict__ tmp, T *__restrict__ out,
                                                                   bool acc, int64_t nbk) {
  __shared__ T buf[kPermBucket * NC];
  const int64_t b = vec_xcd_block(blockIdx.x, nbk);
  if (b >= nbk) return;
  const int64_t lo = b * kPermBucket;
  const int cnt = (int)((n - lo < kPermBucket ? n - lo : kPermBucket) * NC);
  for (int v = threadIdx.x; v < cnt; v += kPermThreads) buf[v] = tmp[lo * NC + v];
  __syncthreads();
  for (int v = threadIdx.x; v < cnt; v += kPermThreads) {
    const int j = v / NC, c = v - j * NC;
    // the slot of a destination in this bucket lies in this bucket (see permute2_positions)
    const T x = buf[(pos2[lo + j] - lo) * NC + c];
    out[lo * NC + v] = acc ? out[lo * NC + v] + x : x;
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
template <typename T, int NC>
static void permute2_nc(const int32_t *pos1, const int32_t *pos2, int64_t n, const T *in, T *tmp, T *out, bool acc,
                        hipStream_t s) {
  const int64_t nblk = (n * NC + 255) / 256, nbk = (n + kPermBucket - 1) / kPermBucket;
  perm_stage1_kernel<T, NC><<<(unsigned)(((nblk + 7) / 8) * 8), 256, 0, s>>>(pos1, n, in, tmp, nblk);
  perm_stage2_kernel<T, NC><<<(unsigned)(((nbk + 7) / 8) * 8), kPermThreads, 0, s>>>(pos2, n, tmp, out, acc, nbk);
}
template <typename T>
int launch_permute2(const int32_t *pos1, const int32_t *pos2, int64_t n, int nc, const T *in, T *tmp, T *out,
                    bool acc, hipStream_t s) {
  if (n <= 0) return MF_OK;
  switch (nc) {
    case 1: permute2_nc<T, 1>(pos1, pos2, n, in, tmp, out, acc, s); break;
    case 2: permute2_nc<T, 2>(pos1, pos2, n, in, tmp, out, acc, s); break;
    case 3: permute2_nc<T, 3>(pos1, pos2, n, in, tmp, out, acc, s); break;
    default: return fail(MF_EINVAL, "launch_permute2: ncomp must be 1..3");
  }
  MF_HIP(hipGetLastError());
  return MF_OK;
}
template <typename T>
int launch_permute_stage1(const int32_t *pos1, int64_t n, int nc, const T *in, T *tmp, hipStream_t s) {
  if (n <= 0) return MF_OK;
  const int64_t nblk = (n * nc + 255) / 256;
  const unsigned g = (unsigned)(((nblk + 7) / 8) * 8);
  switch (nc) {
    case 1: perm_stage1_kernel<T, 1><<<g, 256, 0, s>>>(pos1, n, in, tmp, nblk); break;
    case 2: perm_stage1_kernel<T, 2><<<g, 256, 0, s>>>(pos1, n, in, tmp, nblk); break;
    case 3: perm_stage1_kernel<T, 3><<<g, 256, 0, s>>>(pos1, n, in, tmp, nblk); break;
    default: return fail(MF_EINVAL, "launch_permute_stage1: ncomp must be 1..3");
  }
  MF_HIP(hipGetLastError());
  return MF_OK;
}
template int launch_permute_stage1<double>(const int32_t *, int64_t, int, const double *, double *, hipStream_t);
template int launch_permute_stage1<float>(const int32_t *, int64_t, int, const float *, float *, hipStream_t);
template int launch_permute2<double>(const int32_t *, const int32_t *, int64_t, int, const double *, double *,
                                     double *, bool, hipStream_t);
template int launch_permute2<float>(const int32_t *, const int32_t *, int64_t, int, const float *, float *, float *,
                                    bool, hipStream_t);

void permute2_positions(const int32_t *src, int64_t n, std::vector<int32_t> &pos1, std::vector<int32_t> &pos2) {
  // destination buckets of S consecutive elements; inside a bucket, source order
  const int64_t S = kPermBucket, nbk = (n + S - 1) / S;
  std::vector<int32_t> dst((size_t)n);
  for (int64_t i = 0; i < n; i++) dst[src[i]] = (int32_t)i;
  std::vector<int64_t> fill((size_t)nbk, 0);
  pos1.assign((size_t)n, 0);
  pos2.assign((size_t)n, 0);
  for (int64_t j = 0; j < n; j++) {
    const int64_t b = dst[j] / S;
    pos1[j] = (int32_t)(b * S + fill[b]++);
  }
  for (int64_t i = 0; i < n; i++) pos2[i] = pos1[src[i]];
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
