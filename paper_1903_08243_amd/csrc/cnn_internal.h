// Learned convolutional preconditioner: network object, kernels and launchers.
//
// The network is an L-level U-Net on channel-last FP32 lattices
// ([batch][z][y][x][channel]) with (n - 1) divisible by 2^(L-1) per direction:
//   h_0 = relu(A x);  c_l = R h_(l-1), h_l = relu(B_l c_l)     (l = 1 .. L-1)
//   g_(L-1) = relu(D h_(L-1));  u_l = P g_(l+1) + h_l         (l = L-2 .. 0)
//   g_l = relu(E_l u_l) (l = L-2 .. 1);  y = x + F u_0.
// Convolutions have 3x3x3 taps, zero padding and no bias; weights W[tap][cin][cout]
// with tap = (dx+1) + 3 (dy+1) + 9 (dz+1) and out[v] = sum_d in[v + d] W[tap(d)].
// R is full weighting (1/4, 1/2, 1/4 per direction), P trilinear interpolation
// (P^T = 8 R). Without biases the network is positively homogeneous of degree one,
// and with zero weights it is the identity.
#pragma once
#include "mf_internal.h"

namespace mf {

constexpr int CNN_MAX_LEVELS = 8;

// Offsets of the 2L weight tensors in the flat parameter vector, stored in the
// order A, B_1 .. B_(L-1), D, E_(L-2) .. E_1, F.
struct CnnLayout {
  int C = 0, L = 0;
  int64_t off[2 * CNN_MAX_LEVELS + 1] = {};
  CnnLayout(int c = 0, int levels = 0) : C(c), L(levels) {
    off[0] = 0;
    for (int t = 0; t < 2 * L; t++) off[t + 1] = off[t] + ((t == 0 || t == 2 * L - 1) ? 27LL * c : 27LL * c * c);
  }
  int64_t nparams() const { return off[2 * L]; }
  int64_t A() const { return off[0]; }
  int64_t B(int l) const { return off[l]; }                  // l = 1 .. L-1
  int64_t Dl() const { return off[L]; }
  int64_t E(int l) const { return off[L + (L - 1 - l)]; }    // l = L-2 .. 1
  int64_t F() const { return off[2 * L - 1]; }
};

struct Grid3 {
  int B, Z, Y, X;
  int64_t points() const { return (int64_t)B * Z * Y * X; }
};
inline Grid3 coarser(const Grid3 &g) { return {g.B, (g.Z + 1) / 2, (g.Y + 1) / 2, (g.X + 1) / 2}; }

// out = conv(in) (channels ci -> co) [+ add], optional ReLU; FLIP: the transposed
// convolution of the backward pass (taps mirrored, weight W[t][co][ci] of the
// forward layer with ci/co swapped), its result multiplied by (mask > 0) if mask
// is set.
int cnn_conv(const float *in, const float *W, float *out, const float *mask, const Grid3 &g, int ci, int co,
             bool relu, bool flip, hipStream_t s, const float *add = nullptr);
// dW[t][ci][co] = sum over points of a[v + d_t][ci] g[v][co]; partials per chunk,
// then an ordered FP64 sum over chunks (deterministic). part: workspace of
// cnn_wgrad_part_floats(g, ci, co) floats.
int64_t cnn_wgrad_part_floats(const Grid3 &g, int ci, int co);
int cnn_wgrad(const float *a, const float *gr, float *dW, float *part, const Grid3 &g, int ci, int co,
              hipStream_t s);
// c = scale * R f (fine grid g -> coarser(g)), optionally times (mask > 0) (mask on the coarse grid)
int cnn_restrict(const float *f, float *c, const float *mask, float scale, const Grid3 &g, int ch, hipStream_t s);
// out = (h + scale * P c) [* (mask > 0)], fine grid g; out may alias h
int cnn_prolong_add(const float *c, const float *h, float *out, const float *mask, float scale, const Grid3 &g,
                    int ch, hipStream_t s);
// per-sample sums: dd[b] = |y_b - t_b|^2, tt[b] = |t_b|^2 (FP64), loss = mean(dd/tt)
// written to *loss; gy = (2/B) (y - t) / tt[b]. part: workspace of cnn_loss_part_doubles(B) doubles.
int64_t cnn_loss_part_doubles(int B);
int cnn_loss(const float *y, const float *t, float *gy, double *loss, double *part, int B, int64_t npts,
             hipStream_t s);
// Adam (Kingma and Ba): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
// theta -= lr (m / bc1) / (sqrt(v / bc2) + eps)
int cnn_adam(float *theta, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2, float eps,
             float bc1, float bc2, hipStream_t s);

// Lattice transfers for the preconditioner (vectors in the operator's internal numbering).
// grid[gidx[i]] = (float)(v[i] * sd[i]^pw), pw = +1 or -1
int cnn_to_grid(const double *v, const double *sd, int pw, const int32_t *gidx, float *grid, int64_t n,
                hipStream_t s);
// z[i] = bc[i] ? r[i] : sd[i] * grid[gidx[i]]
int cnn_from_grid(const float *grid, const double *sd, const int32_t *gidx, const uint8_t *bc, const double *r,
                  double *z, int64_t n, hipStream_t s);
// crops of the lattice pair (gr, ge) (Z, Y, X): sample c starts at corner (z, y, x) =
// corners[3c..3c+2], size n^3; both scaled by 1 / rms of the r crop (1 if zero)
int cnn_crops(const float *gr, const float *ge, int Z, int Y, int X, const int32_t *corners, int ncrops, int n,
              float *r_out, float *e_out, hipStream_t s);
int cnn_mark(const int32_t *idx, int64_t n, uint8_t *mask, hipStream_t s);
// Energy (Ritz) loss of z = M r: loss = (z'Az - 2 z'r) / (r'D^{-1}r) into *loss (device),
// and its gradient with respect to the network output on the lattice into gy
// (constrained dofs: 0). part: cnn_energy_part_doubles() doubles; scale: 1 double.
int64_t cnn_energy_part_doubles();
int cnn_energy(const double *z, const double *Az, const double *r, const double *dinv, const double *sd,
               const int32_t *gidx, const uint8_t *bc, int64_t n, double *part, double *loss, double *scale, float *gy,
               hipStream_t s);

// Activations of one forward pass (kept for the backward pass when training):
// per level l the lattice grid[l], h[l], c[l] (l >= 1), g[l] (l >= 1), u[l] (l <= L-2).
struct CnnActs {
  Grid3 grid[CNN_MAX_LEVELS] = {};
  int C = 0, L = 0;
  DeviceBuffer h[CNN_MAX_LEVELS], c[CNN_MAX_LEVELS], g[CNN_MAX_LEVELS], u[CNN_MAX_LEVELS], y;
  int ensure(const Grid3 &g0, int C, int L);
};

// Forward pass over a.grid[0] (x: [B][Z][Y][X], one channel); result in a.y.
int cnn_forward(const float *theta, const CnnLayout &L, const float *x, CnnActs &a, hipStream_t s);

}  // namespace mf

struct mf_cnn {
  int C = 0, levels = 0;
  mf::CnnLayout L;
  mf::DeviceBuffer theta, grad, m, v;
  int64_t step = 0;  // Adam steps taken
  // training workspaces (grown on demand)
  mf::CnnActs acts;
  mf::DeviceBuffer xb, tb, gy, gh[mf::CNN_MAX_LEVELS], s1, s2, part, lpart, loss;
};
