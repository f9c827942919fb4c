// Kernels of the learned convolutional preconditioner (FP32 network, FP64 vectors).
//
// Lattices are channel-last, [batch][z][y][x][channel], so the channels of one
// point are contiguous (one or two 16-byte loads for 4..8 channels). One thread
// computes all output channels of one point; the weights of a tap are the same for
// every lane, so they are read through the scalar cache and used as scalar FMA
// operands.
#include "cnn_internal.h"

namespace mf {

constexpr int CB = 256;  // threads per block of the pointwise kernels

__device__ __forceinline__ void decode(int64_t p, int X, int Y, int Z, int &b, int &z, int &y, int &x) {
  x = (int)(p % X);
  int64_t q = p / X;
  y = (int)(q % Y);
  q /= Y;
  z = (int)(q % Z);
  b = (int)(q / Z);
}

// ------------------------------------------------------------------ convolution
template <int CI, int CO, bool FLIP, bool RELU>
__global__ void __launch_bounds__(CB) conv_kernel(const float *__restrict__ in, const float *__restrict__ W,
                                                  float *__restrict__ out, const float *__restrict__ mask,
                                                  const float *__restrict__ add, int B, int Z, int Y, int X) {
  const int64_t np = (int64_t)B * Z * Y * X;
  const int64_t p = (int64_t)blockIdx.x * CB + threadIdx.x;
  if (p >= np) return;
  int b, z, y, x;
  decode(p, X, Y, Z, b, z, y, x);
  float acc[CO];
#pragma unroll
  for (int o = 0; o < CO; o++) acc[o] = 0.0f;
  for (int dz = -1; dz <= 1; dz++) {
    const int zz = FLIP ? z - dz : z + dz;
    if (zz < 0 || zz >= Z) continue;
    for (int dy = -1; dy <= 1; dy++) {
      const int yy = FLIP ? y - dy : y + dy;
      if (yy < 0 || yy >= Y) continue;
#pragma unroll
      for (int dx = -1; dx <= 1; dx++) {
        const int xx = FLIP ? x - dx : x + dx;
        if (xx < 0 || xx >= X) continue;
        const int t = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
        const float *src = in + ((((int64_t)b * Z + zz) * Y + yy) * X + xx) * CI;
        float v[CI];
#pragma unroll
        for (int i = 0; i < CI; i++) v[i] = src[i];
        const float *w = W + t * CI * CO;
#pragma unroll
        for (int i = 0; i < CI; i++)
#pragma unroll
          for (int o = 0; o < CO; o++) acc[o] = fmaf(v[i], FLIP ? w[o * CI + i] : w[i * CO + o], acc[o]);
      }
    }
  }
  float *dst = out + p * CO;
#pragma unroll
  for (int o = 0; o < CO; o++) {
    float r = RELU ? fmaxf(acc[o], 0.0f) : acc[o];
    if (mask) r = mask[p * CO + o] > 0.0f ? r : 0.0f;
    if (add) r += add[p * CO + o];
    dst[o] = r;
  }
}

template <int CI, int CO>
static int conv_launch(const float *in, const float *W, float *out, const float *mask, const float *add,
                       const Grid3 &g, bool relu, bool flip, hipStream_t s) {
  const int64_t np = g.points();
  const unsigned nb = (unsigned)((np + CB - 1) / CB);
  if (flip) {
    if (relu) conv_kernel<CI, CO, true, true><<<nb, CB, 0, s>>>(in, W, out, mask, add, g.B, g.Z, g.Y, g.X);
    else conv_kernel<CI, CO, true, false><<<nb, CB, 0, s>>>(in, W, out, mask, add, g.B, g.Z, g.Y, g.X);
  } else {
    if (relu) conv_kernel<CI, CO, false, true><<<nb, CB, 0, s>>>(in, W, out, mask, add, g.B, g.Z, g.Y, g.X);
    else conv_kernel<CI, CO, false, false><<<nb, CB, 0, s>>>(in, W, out, mask, add, g.B, g.Z, g.Y, g.X);
  }
  MF_HIP(hipGetLastError());
  return MF_OK;
}

template <int C>
static int conv_dispatch(const float *in, const float *W, float *out, const float *mask, const float *add,
                         const Grid3 &g, int ci, int co, bool relu, bool flip, hipStream_t s) {
  if (ci == 1 && co == C) return conv_launch<1, C>(in, W, out, mask, add, g, relu, flip, s);
  if (ci == C && co == C) return conv_launch<C, C>(in, W, out, mask, add, g, relu, flip, s);
  if (ci == C && co == 1) return conv_launch<C, 1>(in, W, out, mask, add, g, relu, flip, s);
  return fail(MF_EUNSUPPORTED, "cnn_conv: channel pair");
}

int cnn_conv(const float *in, const float *W, float *out, const float *mask, const Grid3 &g, int ci, int co,
             bool relu, bool flip, hipStream_t s, const float *add) {
  if (g.points() == 0) return MF_OK;
  const int C = ci > co ? ci : co;
  switch (C) {
    case 4: return conv_dispatch<4>(in, W, out, mask, add, g, ci, co, relu, flip, s);
    case 8: return conv_dispatch<8>(in, W, out, mask, add, g, ci, co, relu, flip, s);
    case 16: return conv_dispatch<16>(in, W, out, mask, add, g, ci, co, relu, flip, s);
  }
  return fail(MF_EUNSUPPORTED, "cnn_conv: channels must be 4, 8 or 16");
}

// ------------------------------------------------------------------ weight gradient
constexpr int WG_GROUP = 8;  // output channels per block (bounds the accumulators per thread)

static int64_t wgrad_chunk(int64_t np) {
  int64_t c = (np + 63) / 64;
  return c < 2048 ? 2048 : c;
}
static int64_t wgrad_nchunks(int64_t np) { return (np + wgrad_chunk(np) - 1) / wgrad_chunk(np); }

int64_t cnn_wgrad_part_floats(const Grid3 &g, int ci, int co) { return wgrad_nchunks(g.points()) * 27 * ci * co; }

// block (chunk, tap, output group): part[(chunk*27 + t)][ci][co] for its co group
template <int CI, int CG>
__global__ void __launch_bounds__(CB) wgrad_kernel(const float *__restrict__ a, const float *__restrict__ gr,
                                                   float *__restrict__ part, int co, int B, int Z, int Y, int X,
                                                   int64_t chunk) {
  __shared__ float sh[CB / 64][CI * CG];
  const int t = blockIdx.y, og = blockIdx.z * CG;
  const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
  const int64_t np = (int64_t)B * Z * Y * X;
  const int64_t p0 = (int64_t)blockIdx.x * chunk;
  const int64_t p1 = p0 + chunk < np ? p0 + chunk : np;
  float acc[CI * CG];
#pragma unroll
  for (int j = 0; j < CI * CG; j++) acc[j] = 0.0f;
  for (int64_t p = p0 + threadIdx.x; p < p1; p += CB) {
    int b, z, y, x;
    decode(p, X, Y, Z, b, z, y, x);
    const int zz = z + dz, yy = y + dy, xx = x + dx;
    if (zz < 0 || zz >= Z || yy < 0 || yy >= Y || xx < 0 || xx >= X) continue;
    const float *src = a + ((((int64_t)b * Z + zz) * Y + yy) * X + xx) * CI;
    float av[CI], gv[CG];
#pragma unroll
    for (int i = 0; i < CI; i++) av[i] = src[i];
#pragma unroll
    for (int o = 0; o < CG; o++) gv[o] = gr[p * co + og + o];
#pragma unroll
    for (int i = 0; i < CI; i++)
#pragma unroll
      for (int o = 0; o < CG; o++) acc[i * CG + o] = fmaf(av[i], gv[o], acc[i * CG + o]);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < CI * CG; j++) {
    float v = acc[j];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if (lane == 0) sh[w][j] = v;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < CI * CG; j += CB) {
    float v = 0.0f;
    for (int q = 0; q < CB / 64; q++) v += sh[q][j];
    const int i = j / CG, o = j % CG;
    part[((int64_t)blockIdx.x * 27 + t) * CI * co + i * co + og + o] = v;
  }
}

// dW[j] = sum over chunks (in order, FP64)
__global__ void wgrad_sum_kernel(const float *__restrict__ part, float *__restrict__ dW, int per, int64_t nch) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= per) return;
  double s = 0.0;
  for (int64_t c = 0; c < nch; c++) s += part[c * per + j];
  dW[j] = (float)s;
}

template <int CI>
static int wgrad_ci(const float *a, const float *gr, float *part, const Grid3 &g, int co, int64_t chunk,
                    int64_t nch, hipStream_t s) {
  const int cg = co < WG_GROUP ? co : WG_GROUP;
  dim3 grid((unsigned)nch, 27, (unsigned)(co / cg));
  if (cg == 1) wgrad_kernel<CI, 1><<<grid, CB, 0, s>>>(a, gr, part, co, g.B, g.Z, g.Y, g.X, chunk);
  else if (cg == 4) wgrad_kernel<CI, 4><<<grid, CB, 0, s>>>(a, gr, part, co, g.B, g.Z, g.Y, g.X, chunk);
  else if (cg == 8) wgrad_kernel<CI, 8><<<grid, CB, 0, s>>>(a, gr, part, co, g.B, g.Z, g.Y, g.X, chunk);
  else return fail(MF_EUNSUPPORTED, "cnn_wgrad: output channels");
  MF_HIP(hipGetLastError());
  return MF_OK;
}

int cnn_wgrad(const float *a, const float *gr, float *dW, float *part, const Grid3 &g, int ci, int co,
              hipStream_t s) {
  const int64_t np = g.points();
  if (np == 0) return launch_fill<float>(dW, 0.0f, 27LL * ci * co, s);
  const int64_t chunk = wgrad_chunk(np), nch = wgrad_nchunks(np);
  int rc;
  switch (ci) {
    case 1: rc = wgrad_ci<1>(a, gr, part, g, co, chunk, nch, s); break;
    case 4: rc = wgrad_ci<4>(a, gr, part, g, co, chunk, nch, s); break;
    case 8: rc = wgrad_ci<8>(a, gr, part, g, co, chunk, nch, s); break;
    case 16: rc = wgrad_ci<16>(a, gr, part, g, co, chunk, nch, s); break;
    default: return fail(MF_EUNSUPPORTED, "cnn_wgrad: input channels");
  }
  if (rc) return rc;
  const int per = 27 * ci * co;
  wgrad_sum_kernel<<<(per + 255) / 256, 256, 0, s>>>(part, dW, per, nch);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

// ------------------------------------------------------------------ transfers between levels
template <int CH>
__global__ void __launch_bounds__(CB) restrict_kernel(const float *__restrict__ f, float *__restrict__ c,
                                                      const float *__restrict__ mask, float scale, int B, int Z,
                                                      int Y, int X) {
  const int Zc = (Z + 1) / 2, Yc = (Y + 1) / 2, Xc = (X + 1) / 2;
  const int64_t np = (int64_t)B * Zc * Yc * Xc;
  const int64_t p = (int64_t)blockIdx.x * CB + threadIdx.x;
  if (p >= np) return;
  int b, I, J, K;
  decode(p, Xc, Yc, Zc, b, K, J, I);  // K: z, J: y, I: x
  float acc[CH];
#pragma unroll
  for (int ch = 0; ch < CH; ch++) acc[ch] = 0.0f;
  for (int dz = -1; dz <= 1; dz++) {
    const int zz = 2 * K + dz;
    if (zz < 0 || zz >= Z) continue;
    const float wz = dz == 0 ? 0.5f : 0.25f;
    for (int dy = -1; dy <= 1; dy++) {
      const int yy = 2 * J + dy;
      if (yy < 0 || yy >= Y) continue;
      const float wy = wz * (dy == 0 ? 0.5f : 0.25f);
      for (int dx = -1; dx <= 1; dx++) {
        const int xx = 2 * I + dx;
        if (xx < 0 || xx >= X) continue;
        const float w = wy * (dx == 0 ? 0.5f : 0.25f);
        const float *src = f + ((((int64_t)b * Z + zz) * Y + yy) * X + xx) * CH;
#pragma unroll
        for (int ch = 0; ch < CH; ch++) acc[ch] = fmaf(w, src[ch], acc[ch]);
      }
    }
  }
#pragma unroll
  for (int ch = 0; ch < CH; ch++) {
    float r = scale * acc[ch];
    if (mask) r = mask[p * CH + ch] > 0.0f ? r : 0.0f;
    c[p * CH + ch] = r;
  }
}

template <int CH>
__global__ void __launch_bounds__(CB) prolong_add_kernel(const float *__restrict__ c, const float *h, float *out,
                                                         const float *__restrict__ mask, float scale, int B, int Z,
                                                         int Y, int X) {
  const int Zc = (Z + 1) / 2, Yc = (Y + 1) / 2, Xc = (X + 1) / 2;
  const int64_t np = (int64_t)B * Z * Y * X;
  const int64_t p = (int64_t)blockIdx.x * CB + threadIdx.x;
  if (p >= np) return;
  int b, z, y, x;
  decode(p, X, Y, Z, b, z, y, x);
  // parents along each axis: even i -> i/2 (weight 1); odd i -> i/2, i/2 + 1 (1/2 each)
  const int nz = (z & 1) + 1, ny = (y & 1) + 1, nx = (x & 1) + 1;
  const float wz = nz == 1 ? 1.0f : 0.5f, wy = ny == 1 ? 1.0f : 0.5f, wx = nx == 1 ? 1.0f : 0.5f;
  float acc[CH];
#pragma unroll
  for (int ch = 0; ch < CH; ch++) acc[ch] = 0.0f;
  for (int a = 0; a < nz; a++)
    for (int e = 0; e < ny; e++)
      for (int q = 0; q < nx; q++) {
        const int K = z / 2 + a, J = y / 2 + e, I = x / 2 + q;
        const float w = wz * wy * wx;
        const float *src = c + ((((int64_t)b * Zc + K) * Yc + J) * Xc + I) * CH;
#pragma unroll
        for (int ch = 0; ch < CH; ch++) acc[ch] = fmaf(w, src[ch], acc[ch]);
      }
#pragma unroll
  for (int ch = 0; ch < CH; ch++) {
    float r = h[p * CH + ch] + scale * acc[ch];
    if (mask) r = mask[p * CH + ch] > 0.0f ? r : 0.0f;
    out[p * CH + ch] = r;
  }
}

int cnn_restrict(const float *f, float *c, const float *mask, float scale, const Grid3 &g, int ch, hipStream_t s) {
  const Grid3 gc = coarser(g);
  const int64_t np = gc.points();
  if (np == 0) return MF_OK;
  const unsigned nb = (unsigned)((np + CB - 1) / CB);
  switch (ch) {
    case 4: restrict_kernel<4><<<nb, CB, 0, s>>>(f, c, mask, scale, g.B, g.Z, g.Y, g.X); break;
    case 8: restrict_kernel<8><<<nb, CB, 0, s>>>(f, c, mask, scale, g.B, g.Z, g.Y, g.X); break;
    case 16: restrict_kernel<16><<<nb, CB, 0, s>>>(f, c, mask, scale, g.B, g.Z, g.Y, g.X); break;
    default: return fail(MF_EUNSUPPORTED, "cnn_restrict: channels");
  }
  MF_HIP(hipGetLastError());
  return MF_OK;
}

int cnn_prolong_add(const float *c, const float *h, float *out, const float *mask, float scale, const Grid3 &g,
                    int ch, hipStream_t s) {
  const int64_t np = g.points();
  if (np == 0) return MF_OK;
  const unsigned nb = (unsigned)((np + CB - 1) / CB);
  switch (ch) {
    case 4: prolong_add_kernel<4><<<nb, CB, 0, s>>>(c, h, out, mask, scale, g.B, g.Z, g.Y, g.X); break;
    case 8: prolong_add_kernel<8><<<nb, CB, 0, s>>>(c, h, out, mask, scale, g.B, g.Z, g.Y, g.X); break;
    case 16: prolong_add_kernel<16><<<nb, CB, 0, s>>>(c, h, out, mask, scale, g.B, g.Z, g.Y, g.X); break;
    default: return fail(MF_EUNSUPPORTED, "cnn_prolong_add: channels");
  }
  MF_HIP(hipGetLastError());
  return MF_OK;
}

// ------------------------------------------------------------------ loss
constexpr int LOSS_BLK = 64;  // blocks per sample

__global__ void __launch_bounds__(CB) loss_part_kernel(const float *__restrict__ y, const float *__restrict__ t,
                                                       double *__restrict__ part, int64_t npts) {
  __shared__ double sh[2][CB / 64];
  const int b = blockIdx.y;
  const int64_t per = (npts + LOSS_BLK - 1) / LOSS_BLK;
  const int64_t i0 = blockIdx.x * per, i1 = i0 + per < npts ? i0 + per : npts;
  double dd = 0.0, tt = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += CB) {
    const double tv = t[(int64_t)b * npts + i], d = (double)y[(int64_t)b * npts + i] - tv;
    dd += d * d;
    tt += tv * tv;
  }
  for (int o = 32; o > 0; o >>= 1) {
    dd += __shfl_down(dd, o, 64);
    tt += __shfl_down(tt, o, 64);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    sh[0][w] = dd;
    sh[1][w] = tt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, c = 0.0;
    for (int q = 0; q < CB / 64; q++) {
      a += sh[0][q];
      c += sh[1][q];
    }
    part[((int64_t)b * LOSS_BLK + blockIdx.x) * 2] = a;
    part[((int64_t)b * LOSS_BLK + blockIdx.x) * 2 + 1] = c;
  }
}

// one thread: per-sample sums in block order, loss, and the per-sample factors 2 / (B tt_b)
__global__ void loss_final_kernel(double *__restrict__ part, double *__restrict__ loss, int B) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double *fac = part + (int64_t)B * LOSS_BLK * 2;
  double L = 0.0;
  for (int b = 0; b < B; b++) {
    double dd = 0.0, tt = 0.0;
    for (int q = 0; q < LOSS_BLK; q++) {
      dd += part[((int64_t)b * LOSS_BLK + q) * 2];
      tt += part[((int64_t)b * LOSS_BLK + q) * 2 + 1];
    }
    // a sample with a zero target contributes nothing (its relative error is undefined)
    L += tt > 0.0 ? dd / tt : 0.0;
    fac[b] = tt > 0.0 ? 2.0 / ((double)B * tt) : 0.0;
  }
  *loss = L / B;
}

__global__ void __launch_bounds__(CB) loss_grad_kernel(const float *__restrict__ y, const float *__restrict__ t,
                                                       float *__restrict__ gy, const double *__restrict__ fac,
                                                       int64_t npts, int B) {
  const int64_t i = (int64_t)blockIdx.x * CB + threadIdx.x;
  if (i >= npts * B) return;
  const int b = (int)(i / npts);
  gy[i] = (float)(fac[b] * ((double)y[i] - (double)t[i]));
}

int64_t cnn_loss_part_doubles(int B) { return (int64_t)B * LOSS_BLK * 2 + B; }

int cnn_loss(const float *y, const float *t, float *gy, double *loss, double *part, int B, int64_t npts,
             hipStream_t s) {
  loss_part_kernel<<<dim3(LOSS_BLK, B), CB, 0, s>>>(y, t, part, npts);
  MF_HIP(hipGetLastError());
  loss_final_kernel<<<1, 64, 0, s>>>(part, loss, B);
  MF_HIP(hipGetLastError());
  const int64_t n = npts * B;
  loss_grad_kernel<<<(unsigned)((n + CB - 1) / CB), CB, 0, s>>>(y, t, gy, part + (int64_t)B * LOSS_BLK * 2, npts,
                                                                  B);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

// ------------------------------------------------------------------ Adam
__global__ void adam_kernel(float *__restrict__ th, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float bc1,
                            float bc2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

int cnn_adam(float *theta, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2, float eps,
             float bc1, float bc2, hipStream_t s) {
  adam_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(theta, g, m, v, n, lr, b1, b2, eps, bc1, bc2);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

// ------------------------------------------------------------------ lattice transfers
__global__ void to_grid_kernel(const double *__restrict__ v, const double *__restrict__ sd, int pw,
                               const int32_t *__restrict__ gidx, float *__restrict__ grid, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * CB + threadIdx.x;
  if (i >= n) return;
  const double sc = pw > 0 ? sd[i] : 1.0 / sd[i];
  grid[gidx[i]] = (float)(v[i] * sc);
}

__global__ void from_grid_kernel(const float *__restrict__ grid, const double *__restrict__ sd,
                                 const int32_t *__restrict__ gidx, const uint8_t *__restrict__ bc,
                                 const double *__restrict__ r, double *__restrict__ z, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * CB + threadIdx.x;
  if (i >= n) return;
  z[i] = (bc && bc[i]) ? r[i] : sd[i] * (double)grid[gidx[i]];
}

int cnn_to_grid(const double *v, const double *sd, int pw, const int32_t *gidx, float *grid, int64_t n,
                hipStream_t s) {
  if (n == 0) return MF_OK;
  to_grid_kernel<<<(unsigned)((n + CB - 1) / CB), CB, 0, s>>>(v, sd, pw, gidx, grid, n);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

int cnn_from_grid(const float *grid, const double *sd, const int32_t *gidx, const uint8_t *bc, const double *r,
                  double *z, int64_t n, hipStream_t s) {
  if (n == 0) return MF_OK;
  from_grid_kernel<<<(unsigned)((n + CB - 1) / CB), CB, 0, s>>>(grid, sd, gidx, bc, r, z, n);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

__global__ void __launch_bounds__(CB) crops_kernel(const float *__restrict__ gr, const float *__restrict__ ge, int Z,
                                                   int Y, int X, const int32_t *__restrict__ corners, int n,
                                                   float *__restrict__ r_out, float *__restrict__ e_out) {
  __shared__ double sh[CB / 64];
  const int c = blockIdx.x;
  const int z0 = corners[3 * c], y0 = corners[3 * c + 1], x0 = corners[3 * c + 2];
  const int64_t n3 = (int64_t)n * n * n;
  double ss = 0.0;
  for (int64_t i = threadIdx.x; i < n3; i += CB) {
    const int x = (int)(i % n), y = (int)((i / n) % n), z = (int)(i / ((int64_t)n * n));
    const double v = gr[((int64_t)(z0 + z) * Y + (y0 + y)) * X + (x0 + x)];
    ss += v * v;
  }
  for (int o = 32; o > 0; o >>= 1) ss += __shfl_down(ss, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = ss;
  __syncthreads();
  double tot = 0.0;
  for (int q = 0; q < CB / 64; q++) tot += sh[q];
  const float sc = tot > 0.0 ? (float)(1.0 / sqrt(tot / (double)n3)) : 1.0f;
  for (int64_t i = threadIdx.x; i < n3; i += CB) {
    const int x = (int)(i % n), y = (int)((i / n) % n), z = (int)(i / ((int64_t)n * n));
    const int64_t src = ((int64_t)(z0 + z) * Y + (y0 + y)) * X + (x0 + x);
    r_out[(int64_t)c * n3 + i] = sc * gr[src];
    e_out[(int64_t)c * n3 + i] = sc * ge[src];
  }
}

int cnn_crops(const float *gr, const float *ge, int Z, int Y, int X, const int32_t *corners, int ncrops, int n,
              float *r_out, float *e_out, hipStream_t s) {
  if (ncrops == 0) return MF_OK;
  crops_kernel<<<ncrops, CB, 0, s>>>(gr, ge, Z, Y, X, corners, n, r_out, e_out);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

// ------------------------------------------------------------------ energy (Ritz) loss
constexpr int EN_BLK = 1024;

// partials of z'Az, z'r and r'D^{-1}r (FP64)
__global__ void __launch_bounds__(CB) energy_part_kernel(const double *__restrict__ z, const double *__restrict__ Az,
                                                         const double *__restrict__ r, const double *__restrict__ dinv,
                                                         int64_t n, double *__restrict__ part) {
  __shared__ double sh[3][CB / 64];
  double a = 0.0, b = 0.0, c = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * CB + threadIdx.x; i < n; i += (int64_t)gridDim.x * CB) {
    const double zi = z[i], ri = r[i];
    a += zi * Az[i];
    b += zi * ri;
    c += ri * ri * dinv[i];
  }
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_down(a, o, 64);
    b += __shfl_down(b, o, 64);
    c += __shfl_down(c, o, 64);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    sh[0][w] = a;
    sh[1][w] = b;
    sh[2][w] = c;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double t = 0.0;
    for (int q = 0; q < CB / 64; q++) t += sh[threadIdx.x][q];
    part[threadIdx.x * EN_BLK + blockIdx.x] = t;
  }
}

// one thread: loss = (z'Az - 2 z'r) / (r'D^{-1}r) into *loss, gradient scale 2 / (r'D^{-1}r) into *scale
__global__ void energy_final_kernel(const double *__restrict__ part, int nblk, double *__restrict__ loss,
                                    double *__restrict__ scale) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double a = 0.0, b = 0.0, c = 0.0;
  for (int q = 0; q < nblk; q++) {
    a += part[q];
    b += part[EN_BLK + q];
    c += part[2 * EN_BLK + q];
  }
  const bool ok = c > 0.0;
  *loss = ok ? (a - 2.0 * b) / c : 0.0;
  *scale = ok ? 2.0 / c : 0.0;
}

// dLoss/dy on the lattice: y enters z = D^{-1/2} y on free dofs, so g_y = D^{-1/2} g_z
__global__ void energy_grad_kernel(const double *__restrict__ Az, const double *__restrict__ r,
                                   const double *__restrict__ sd, const int32_t *__restrict__ gidx,
                                   const uint8_t *__restrict__ bc, const double *__restrict__ scale, int64_t n,
                                   float *__restrict__ gy) {
  const int64_t i = (int64_t)blockIdx.x * CB + threadIdx.x;
  if (i >= n) return;
  gy[gidx[i]] = (bc && bc[i]) ? 0.0f : (float)(sd[i] * (*scale) * (Az[i] - r[i]));
}

int64_t cnn_energy_part_doubles() { return 3 * EN_BLK; }

int cnn_energy(const double *z, const double *Az, const double *r, const double *dinv, const double *sd,
               const int32_t *gidx, const uint8_t *bc, int64_t n, double *part, double *loss, double *scale, float *gy,
               hipStream_t s) {
  if (n <= 0) return fail(MF_EINVAL, "cnn_energy: empty vector");
  int64_t g = (n + CB - 1) / CB;
  const int nblk = (int)(g < EN_BLK ? g : EN_BLK);
  energy_part_kernel<<<nblk, CB, 0, s>>>(z, Az, r, dinv, n, part);
  MF_HIP(hipGetLastError());
  energy_final_kernel<<<1, 64, 0, s>>>(part, nblk, loss, scale);
  MF_HIP(hipGetLastError());
  energy_grad_kernel<<<(unsigned)((n + CB - 1) / CB), CB, 0, s>>>(Az, r, sd, gidx, bc, scale, n, gy);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

__global__ void mark_kernel(const int32_t *__restrict__ idx, int64_t n, uint8_t *__restrict__ mask) {
  const int64_t i = (int64_t)blockIdx.x * CB + threadIdx.x;
  if (i < n) mask[idx[i]] = 1;
}

int cnn_mark(const int32_t *idx, int64_t n, uint8_t *mask, hipStream_t s) {
  if (n == 0) return MF_OK;
  mark_kernel<<<(unsigned)((n + CB - 1) / CB), CB, 0, s>>>(idx, n, mask);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

}  // namespace mf
