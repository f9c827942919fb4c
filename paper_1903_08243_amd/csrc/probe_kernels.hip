// Attainable peaks of the device, measured the way the paper measured its CPUs'
// (Section 4.1: STREAM for memory bandwidth, LINPACK for arithmetic): a streaming
// copy kernel for HBM bandwidth and long chains of independent multiply-adds for the
// vector (FP64, FP32 without packed math) and matrix (FP32 4x4x1, FP64 4x4x4) units.
// These figures sit beside the vendor peaks in the roofline reports.
#include "mf_internal.h"

namespace mf {

// 16-byte vector copy, grid-stride.
__global__ void __launch_bounds__(256) probe_copy_kernel(const float4 *__restrict__ a, float4 *__restrict__ b,
                                                         int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

// CH independent FMA chains per thread, ITER rounds; the result is stored only when
// it equals an impossible value, so nothing is written but the chains stay live.
template <typename T, int CH, int ITER>
__global__ void __launch_bounds__(256) probe_fma_kernel(T *sink, T a, T b) {
  T acc[CH];
#pragma unroll
  for (int c = 0; c < CH; c++) acc[c] = T(threadIdx.x + c);
  for (int it = 0; it < ITER; it++) {
#pragma unroll
    for (int c = 0; c < CH; c++) acc[c] = __builtin_fma(acc[c], a, b);
  }
  T s = T(0);
#pragma unroll
  for (int c = 0; c < CH; c++) s += acc[c];
  if (s == T(-12345.678)) sink[threadIdx.x] = s;
}

template <int CH, int ITER>
__global__ void __launch_bounds__(256) probe_fma32_kernel(float *sink, float a, float b) {
  float acc[CH];
#pragma unroll
  for (int c = 0; c < CH; c++) acc[c] = float(threadIdx.x + c);
  for (int it = 0; it < ITER; it++) {
#pragma unroll
    for (int c = 0; c < CH; c++) acc[c] = __builtin_fmaf(acc[c], a, b);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < CH; c++) s += acc[c];
  if (s == -12345.678f) sink[threadIdx.x] = s;
}

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));

// CH independent accumulators of v_mfma_f32_4x4x1_16b_f32 (512 flops each).
template <int CH, int ITER>
__global__ void __launch_bounds__(256) probe_mfma32_kernel(float *sink, float a) {
  f4 acc[CH];
#pragma unroll
  for (int c = 0; c < CH; c++) acc[c] = f4{0.f, 0.f, 0.f, float(c)};
  const float x = a * float(threadIdx.x & 3);
  for (int it = 0; it < ITER; it++) {
#pragma unroll
    for (int c = 0; c < CH; c++) acc[c] = __builtin_amdgcn_mfma_f32_4x4x1f32(x, a, acc[c], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < CH; c++) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  if (s == -12345.678f) sink[threadIdx.x] = s;
}

// CH independent accumulators of v_mfma_f64_4x4x4_4b_f64 (512 flops each).
template <int CH, int ITER>
__global__ void __launch_bounds__(256) probe_mfma64_kernel(double *sink, double a) {
  double acc[CH];
#pragma unroll
  for (int c = 0; c < CH; c++) acc[c] = double(c);
  const double x = a * double(threadIdx.x & 3);
  for (int it = 0; it < ITER; it++) {
#pragma unroll
    for (int c = 0; c < CH; c++) acc[c] = __builtin_amdgcn_mfma_f64_4x4x4f64(x, a, acc[c], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < CH; c++) s += acc[c];
  if (s == -12345.678) sink[threadIdx.x] = s;
}

}  // namespace mf

using namespace mf;

namespace {
// Mean seconds per launch of fn over reps launches after one warm-up launch.
template <class F>
int time_launches(F fn, int reps, hipStream_t s, double *sec) {
  hipEvent_t e0, e1;
  MF_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(MF_EDEVICE, "hipEventCreate");
  }
  int rc = MF_OK;
  fn();
  if (hipEventRecord(e0, s) != hipSuccess) rc = fail(MF_EDEVICE, "hipEventRecord");
  for (int r = 0; rc == MF_OK && r < reps; r++) fn();
  if (rc == MF_OK && hipEventRecord(e1, s) != hipSuccess) rc = fail(MF_EDEVICE, "hipEventRecord");
  if (rc == MF_OK && hipGetLastError() != hipSuccess) rc = fail(MF_EDEVICE, "probe kernel launch");
  if (rc == MF_OK && hipEventSynchronize(e1) != hipSuccess) rc = fail(MF_EDEVICE, "hipEventSynchronize");
  float ms = 0.f;
  if (rc == MF_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = fail(MF_EDEVICE, "hipEventElapsedTime");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc == MF_OK) *sec = ms * 1e-3 / reps;
  return rc;
}
}  // namespace

extern "C" {

int mf_probe_peaks(double *out, void *stream) {
  if (!out) return fail(MF_EINVAL, "mf_probe_peaks: out is NULL");
  hipStream_t s = (hipStream_t)stream;
  int dev = 0, ncu = 0;
  MF_HIP(hipGetDevice(&dev));
  MF_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const int64_t n4 = (int64_t)1 << 26;  // 64 Mi float4 = 1 GiB per buffer
  DeviceBuffer a, b, sink;
  if (a.alloc(n4 * 16) || b.alloc(n4 * 16) || sink.alloc(4096)) return fail(MF_ENOMEM, "mf_probe_peaks: buffers");
  MF_HIP(hipMemsetAsync(a.ptr, 0, n4 * 16, s));
  double res[5] = {0, 0, 0, 0, 0}, t = 0;
  int rc = time_launches([&] {
    probe_copy_kernel<<<ncu * 16, 256, 0, s>>>(a.as<float4>(), b.as<float4>(), n4);
  }, 10, s, &t);
  if (rc) return rc;
  res[0] = 2.0 * n4 * 16 / t / 1e9;
  constexpr int CH = 8, IT = 4096;
  const unsigned blocks = (unsigned)ncu * 32;
  rc = time_launches([&] { probe_fma_kernel<double, CH, IT><<<blocks, 256, 0, s>>>(sink.as<double>(), 0.999, 1e-3); },
                     3, s, &t);
  if (rc) return rc;
  res[1] = 2.0 * CH * IT * blocks * 256.0 / t / 1e12;
  rc = time_launches([&] { probe_fma32_kernel<CH, IT><<<blocks, 256, 0, s>>>(sink.as<float>(), 0.999f, 1e-3f); },
                     3, s, &t);
  if (rc) return rc;
  res[2] = 2.0 * CH * IT * blocks * 256.0 / t / 1e12;
  constexpr int MIT = 1024;
  rc = time_launches([&] { probe_mfma32_kernel<CH, MIT><<<blocks, 256, 0, s>>>(sink.as<float>(), 0.5f); }, 3, s, &t);
  if (rc) return rc;
  res[3] = 512.0 * CH * MIT * blocks * 4.0 / t / 1e12;  // 4 wavefronts per block
  rc = time_launches([&] { probe_mfma64_kernel<CH, MIT><<<blocks, 256, 0, s>>>(sink.as<double>(), 0.5); }, 3, s, &t);
  if (rc) return rc;
  res[4] = 512.0 * CH * MIT * blocks * 4.0 / t / 1e12;
  for (int i = 0; i < 5; i++) out[i] = res[i];
  return MF_OK;
}

}  // extern "C"
