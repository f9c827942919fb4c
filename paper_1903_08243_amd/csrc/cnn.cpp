// Learned convolutional preconditioner: network object, forward and backward
// passes, training loop (Adam), and the lattice preconditioner built on an
// operator (diagonal scaling, Dirichlet pass-through, training-pair crops).
//
// Not part of the paper: the paper's operator action is the consumer (the
// preconditioned solver calls it every iteration). The exact network definition
// is stated in cnn_internal.h.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <vector>

#include "cg_internal.h"
#include "cnn_internal.h"

namespace mf {

// every direction: (n - 1) divisible by 2^(L-1) with a coarsest lattice of at least 2 points
static bool lattice_ok(int n, int L) {
  const int q = 1 << (L - 1);
  return n >= q + 1 && (n - 1) % q == 0;
}

// Grows a buffer to at least `bytes`.
static int grow(DeviceBuffer &b, size_t bytes) {
  if (b.ptr && b.bytes >= bytes) return MF_OK;
  if (b.ptr) {
    (void)hipFree(b.ptr);
    b.ptr = nullptr;
    b.bytes = 0;
  }
  return b.alloc(bytes);
}

int CnnActs::ensure(const Grid3 &g0, int c, int levels) {
  const Grid3 &o = grid[0];
  if (g0.B == o.B && g0.Z == o.Z && g0.Y == o.Y && g0.X == o.X && c == C && levels == L && h[0].ptr) return MF_OK;
  C = 0;  // set once every buffer is allocated
  L = levels;
  grid[0] = g0;
  for (int l = 1; l < L; l++) grid[l] = coarser(grid[l - 1]);
  int rc = MF_OK;
  for (int l = 0; l < L && !rc; l++) {
    const size_t f = (size_t)grid[l].points() * c * 4;
    rc = grow(h[l], f);
    if (!rc && l >= 1) rc = grow(this->c[l], f);
    if (!rc && l >= 1) rc = grow(g[l], f);
    if (!rc && l <= L - 2) rc = grow(u[l], f);
  }
  if (!rc) rc = grow(y, (size_t)g0.points() * 4);
  if (!rc) C = c;
  return rc;
}

int cnn_forward(const float *theta, const CnnLayout &Ly, const float *x, CnnActs &a, hipStream_t s) {
  const int C = Ly.C, L = Ly.L;
  auto F = [&](DeviceBuffer &b) { return b.as<float>(); };
  int rc = cnn_conv(x, theta + Ly.A(), F(a.h[0]), nullptr, a.grid[0], 1, C, true, false, s);
  for (int l = 1; l < L && !rc; l++) {
    rc = cnn_restrict(F(a.h[l - 1]), F(a.c[l]), nullptr, 1.0f, a.grid[l - 1], C, s);
    if (!rc) rc = cnn_conv(F(a.c[l]), theta + Ly.B(l), F(a.h[l]), nullptr, a.grid[l], C, C, true, false, s);
  }
  if (!rc) rc = cnn_conv(F(a.h[L - 1]), theta + Ly.Dl(), F(a.g[L - 1]), nullptr, a.grid[L - 1], C, C, true, false, s);
  for (int l = L - 2; l >= 0 && !rc; l--) {
    rc = cnn_prolong_add(F(a.g[l + 1]), F(a.h[l]), F(a.u[l]), nullptr, 1.0f, a.grid[l], C, s);
    if (!rc && l >= 1) rc = cnn_conv(F(a.u[l]), theta + Ly.E(l), F(a.g[l]), nullptr, a.grid[l], C, C, true, false, s);
  }
  // y = x + F u_0
  if (!rc) rc = cnn_conv(F(a.u[0]), theta + Ly.F(), F(a.y), nullptr, a.grid[0], C, 1, false, false, s, x);
  return rc;
}

// Gradient of every weight into net->grad from gy = dLoss/dy, for the forward pass
// kept in `a` (its input x).
static int cnn_backward(mf_cnn *net, CnnActs &a, const float *x, const float *gyp, hipStream_t s) {
  const int C = net->C, L = net->levels;
  const CnnLayout &Ly = net->L;
  int64_t pf = 0;
  int rc = MF_OK;
  for (int l = 0; l < L && !rc; l++) {
    const int64_t v = cnn_wgrad_part_floats(a.grid[l], C, C);
    pf = v > pf ? v : pf;
    rc = grow(net->gh[l], (size_t)a.grid[l].points() * C * 4);
  }
  const size_t f1 = (size_t)a.grid[1].points() * C * 4;
  if (!rc) rc = grow(net->s1, f1);
  if (!rc) rc = grow(net->s2, f1);
  if (!rc) rc = grow(net->part, (size_t)pf * 4);
  if (rc) return rc;
  auto F = [&](DeviceBuffer &b) { return b.as<float>(); };
  const float *th = net->theta.as<float>();
  float *gr = net->grad.as<float>();
  float *part = net->part.as<float>();
  float *S1 = F(net->s1), *S2 = F(net->s2);
  // decoder, fine to coarse. y = x + F u_0: gh[0] starts as g(u_0) (the skip u_0 = P g_1 + h_0)
  rc = cnn_wgrad(F(a.u[0]), gyp, gr + Ly.F(), part, a.grid[0], C, 1, s);
  if (!rc) rc = cnn_conv(gyp, th + Ly.F(), F(net->gh[0]), nullptr, a.grid[0], 1, C, false, true, s);
  for (int l = 0; l < L - 1 && !rc; l++) {
    // g(g_(l+1)) = 8 R g(u_l) masked by g_(l+1) > 0
    rc = cnn_restrict(F(net->gh[l]), S1, F(a.g[l + 1]), 8.0f, a.grid[l], C, s);
    if (rc) break;
    if (l + 1 <= L - 2) {  // g_(l+1) = relu(E_(l+1) u_(l+1)): g(u_(l+1)) starts gh[l+1]
      rc = cnn_wgrad(F(a.u[l + 1]), S1, gr + Ly.E(l + 1), part, a.grid[l + 1], C, C, s);
      if (!rc) rc = cnn_conv(S1, th + Ly.E(l + 1), F(net->gh[l + 1]), nullptr, a.grid[l + 1], C, C, false, true, s);
    } else {  // g_(L-1) = relu(D h_(L-1)): g(h_(L-1)), masked by h_(L-1) > 0
      rc = cnn_wgrad(F(a.h[L - 1]), S1, gr + Ly.Dl(), part, a.grid[L - 1], C, C, s);
      if (!rc)
        rc = cnn_conv(S1, th + Ly.Dl(), F(net->gh[L - 1]), F(a.h[L - 1]), a.grid[L - 1], C, C, false, true, s);
    }
  }
  // encoder, coarse to fine: gh[l] holds the pre-activation gradient of h_l
  for (int l = L - 1; l >= 1 && !rc; l--) {
    rc = cnn_wgrad(F(a.c[l]), F(net->gh[l]), gr + Ly.B(l), part, a.grid[l], C, C, s);
    if (!rc) rc = cnn_conv(F(net->gh[l]), th + Ly.B(l), S2, nullptr, a.grid[l], C, C, false, true, s);
    // c_l = R h_(l-1): g(h_(l-1)) += P g(c_l) / 8, then masked by h_(l-1) > 0
    if (!rc) rc = cnn_prolong_add(S2, F(net->gh[l - 1]), F(net->gh[l - 1]), F(a.h[l - 1]), 0.125f, a.grid[l - 1], C, s);
  }
  if (!rc) rc = cnn_wgrad(x, F(net->gh[0]), gr + Ly.A(), part, a.grid[0], 1, C, s);
  return rc;
}

// Loss of the batch (x, t) and the gradient of every weight into net->grad.
// x, t: [B][Z][Y][X]; the loss (FP64) is left in net->loss on the device.
static int loss_grad(mf_cnn *net, const Grid3 &g0, const float *x, const float *t, hipStream_t s) {
  CnnActs &a = net->acts;
  int rc = a.ensure(g0, net->C, net->levels);
  if (!rc) rc = grow(net->gy, (size_t)g0.points() * 4);
  if (!rc) rc = grow(net->lpart, (size_t)cnn_loss_part_doubles(g0.B) * 8);
  if (!rc) rc = grow(net->loss, 8);
  if (!rc) rc = cnn_forward(net->theta.as<float>(), net->L, x, a, s);
  if (!rc) rc = cnn_loss(a.y.as<float>(), t, net->gy.as<float>(), net->loss.as<double>(), net->lpart.as<double>(),
                         g0.B, (int64_t)g0.Z * g0.Y * g0.X, s);
  if (!rc) rc = cnn_backward(net, a, x, net->gy.as<float>(), s);
  return rc;
}

static int adam(mf_cnn *net, float lr, hipStream_t s) {
  net->step += 1;
  const double b1 = 0.9, b2 = 0.999;
  const double bc1 = 1.0 - std::pow(b1, (double)net->step), bc2 = 1.0 - std::pow(b2, (double)net->step);
  return cnn_adam(net->theta.as<float>(), net->grad.as<float>(), net->m.as<float>(), net->v.as<float>(),
                  net->L.nparams(), lr, (float)b1, (float)b2, 1e-8f, (float)bc1, (float)bc2, s);
}

static int check_grid(int B, int nz, int ny, int nx, int L, const char *who) {
  if (B < 1 || !lattice_ok(nz, L) || !lattice_ok(ny, L) || !lattice_ok(nx, L))
    return fail(MF_EINVAL, std::string(who) + ": every lattice size must be j 2^(L-1) + 1 (j >= 1), batch >= 1");
  return MF_OK;
}

static bool channels_ok(int c) { return c == 4 || c == 8 || c == 16; }
static bool levels_ok(int l) { return l >= 2 && l <= CNN_MAX_LEVELS; }

}  // namespace mf

using namespace mf;

struct CnnFileHeader {
  char magic[8];
  int32_t channels, levels;
  int64_t nparams;
};

extern "C" {

int64_t mf_cnn_nparams(int channels, int levels) {
  if (!channels_ok(channels) || !levels_ok(levels)) return -1;
  return CnnLayout(channels, levels).nparams();
}

int mf_cnn_create(int channels, int levels, const float *theta, mf_cnn **out) {
  if (!out || !theta) return fail(MF_EINVAL, "mf_cnn_create: null argument");
  if (!channels_ok(channels) || !levels_ok(levels))
    return fail(MF_EUNSUPPORTED, "mf_cnn_create: channels must be 4, 8 or 16 and levels 2..8");
  std::unique_ptr<mf_cnn> net(new (std::nothrow) mf_cnn);
  if (!net) return fail(MF_ENOMEM, "mf_cnn_create: host allocation");
  net->C = channels;
  net->levels = levels;
  net->L = CnnLayout(channels, levels);
  const size_t nb = (size_t)net->L.nparams() * 4;
  int rc = net->theta.alloc(nb);
  if (!rc) rc = net->grad.alloc(nb);
  if (!rc) rc = net->m.alloc(nb);
  if (!rc) rc = net->v.alloc(nb);
  if (rc) return rc;
  MF_HIP(hipMemcpy(net->theta.ptr, theta, nb, hipMemcpyHostToDevice));
  MF_HIP(hipMemset(net->m.ptr, 0, nb));
  MF_HIP(hipMemset(net->v.ptr, 0, nb));
  MF_HIP(hipMemset(net->grad.ptr, 0, nb));
  *out = net.release();
  return MF_OK;
}

int mf_cnn_get_params(const mf_cnn *net, float *theta) {
  if (!net || !theta) return fail(MF_EINVAL, "mf_cnn_get_params: null argument");
  MF_HIP(hipDeviceSynchronize());
  MF_HIP(hipMemcpy(theta, net->theta.ptr, (size_t)net->L.nparams() * 4, hipMemcpyDeviceToHost));
  return MF_OK;
}

int mf_cnn_set_params(mf_cnn *net, const float *theta) {
  if (!net || !theta) return fail(MF_EINVAL, "mf_cnn_set_params: null argument");
  const size_t nb = (size_t)net->L.nparams() * 4;
  MF_HIP(hipDeviceSynchronize());
  MF_HIP(hipMemcpy(net->theta.ptr, theta, nb, hipMemcpyHostToDevice));
  MF_HIP(hipMemset(net->m.ptr, 0, nb));
  MF_HIP(hipMemset(net->v.ptr, 0, nb));
  net->step = 0;
  return MF_OK;
}

int mf_cnn_save(const mf_cnn *net, const char *path) {
  if (!net || !path) return fail(MF_EINVAL, "mf_cnn_save: null argument");
  std::vector<float> th((size_t)net->L.nparams());
  int rc = mf_cnn_get_params(net, th.data());
  if (rc) return rc;
  FILE *f = std::fopen(path, "wb");
  if (!f) return fail(MF_EINVAL, std::string("mf_cnn_save: cannot open ") + path);
  CnnFileHeader h{};
  std::memcpy(h.magic, "MFCNN02", 8);
  h.channels = net->C;
  h.levels = net->levels;
  h.nparams = net->L.nparams();
  const bool ok = std::fwrite(&h, sizeof h, 1, f) == 1 && std::fwrite(th.data(), 4, th.size(), f) == th.size();
  if (std::fclose(f) != 0 || !ok) return fail(MF_EINVAL, std::string("mf_cnn_save: write failed: ") + path);
  return MF_OK;
}

int mf_cnn_load(const char *path, mf_cnn **out) {
  if (!path || !out) return fail(MF_EINVAL, "mf_cnn_load: null argument");
  FILE *f = std::fopen(path, "rb");
  if (!f) return fail(MF_EINVAL, std::string("mf_cnn_load: cannot open ") + path);
  CnnFileHeader h{};
  bool ok = std::fread(&h, sizeof h, 1, f) == 1 && std::memcmp(h.magic, "MFCNN02", 8) == 0 &&
            channels_ok(h.channels) && levels_ok(h.levels) &&
            h.nparams == CnnLayout(h.channels, h.levels).nparams();
  std::vector<float> th;
  if (ok) {
    th.resize((size_t)h.nparams);
    ok = std::fread(th.data(), 4, th.size(), f) == th.size();
  }
  std::fclose(f);
  if (!ok) return fail(MF_EINVAL, std::string("mf_cnn_load: not a network file: ") + path);
  return mf_cnn_create(h.channels, h.levels, th.data(), out);
}

void mf_cnn_destroy(mf_cnn *net) {
  if (!net) return;
  (void)hipDeviceSynchronize();
  delete net;
}

int mf_cnn_forward(mf_cnn *net, int batch, int nz, int ny, int nx, const float *x, float *y, void *stream) {
  if (!net || !x || !y) return fail(MF_EINVAL, "mf_cnn_forward: null argument");
  int rc = check_grid(batch, nz, ny, nx, net->levels, "mf_cnn_forward");
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const Grid3 g{batch, nz, ny, nx};
  rc = net->acts.ensure(g, net->C, net->levels);
  if (!rc) rc = cnn_forward(net->theta.as<float>(), net->L, x, net->acts, s);
  if (rc) return rc;
  MF_HIP(hipMemcpyAsync(y, net->acts.y.ptr, (size_t)g.points() * 4, hipMemcpyDeviceToDevice, s));
  return MF_OK;
}

int mf_cnn_loss_grad(mf_cnn *net, int batch, int nz, int ny, int nx, const float *x, const float *t, double *loss,
                     float *grad, void *stream) {
  if (!net || !x || !t) return fail(MF_EINVAL, "mf_cnn_loss_grad: null argument");
  int rc = check_grid(batch, nz, ny, nx, net->levels, "mf_cnn_loss_grad");
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  rc = loss_grad(net, Grid3{batch, nz, ny, nx}, x, t, s);
  if (rc) return rc;
  if (grad)
    MF_HIP(hipMemcpyAsync(grad, net->grad.ptr, (size_t)net->L.nparams() * 4, hipMemcpyDeviceToDevice, s));
  if (loss) {
    MF_HIP(hipMemcpyAsync(loss, net->loss.ptr, 8, hipMemcpyDeviceToHost, s));
    MF_HIP(hipStreamSynchronize(s));
  }
  return MF_OK;
}

int mf_cnn_train(mf_cnn *net, int npairs, int n, const float *r, const float *e, int nsteps, int batch,
                 const int32_t *order, float lr, double *losses, void *stream) {
  if (!net || !r || !e || !order) return fail(MF_EINVAL, "mf_cnn_train: null argument");
  if (npairs < 1 || nsteps < 0 || !(lr > 0.0f)) return fail(MF_EINVAL, "mf_cnn_train: npairs / nsteps / lr");
  int rc = check_grid(batch, n, n, n, net->levels, "mf_cnn_train");
  if (rc) return rc;
  for (int64_t i = 0; i < (int64_t)nsteps * batch; i++)
    if (order[i] < 0 || order[i] >= npairs) return fail(MF_EINVAL, "mf_cnn_train: order index out of range");
  hipStream_t s = (hipStream_t)stream;
  const int64_t n3 = (int64_t)n * n * n;
  rc = grow(net->xb, (size_t)batch * n3 * 4);
  if (!rc) rc = grow(net->tb, (size_t)batch * n3 * 4);
  if (rc) return rc;
  DeviceBuffer lhist;
  if (nsteps > 0) {
    rc = lhist.alloc((size_t)nsteps * 8);
    if (rc) return rc;
  }
  const Grid3 g{batch, n, n, n};
  for (int st = 0; st < nsteps; st++) {
    for (int b = 0; b < batch; b++) {
      const int64_t k = order[(int64_t)st * batch + b];
      MF_HIP(hipMemcpyAsync(net->xb.as<float>() + b * n3, r + k * n3, (size_t)n3 * 4, hipMemcpyDeviceToDevice, s));
      MF_HIP(hipMemcpyAsync(net->tb.as<float>() + b * n3, e + k * n3, (size_t)n3 * 4, hipMemcpyDeviceToDevice, s));
    }
    rc = loss_grad(net, g, net->xb.as<float>(), net->tb.as<float>(), s);
    if (!rc) rc = adam(net, lr, s);
    if (rc) return rc;
    MF_HIP(hipMemcpyAsync(lhist.as<double>() + st, net->loss.ptr, 8, hipMemcpyDeviceToDevice, s));
  }
  if (losses && nsteps > 0) MF_HIP(hipMemcpyAsync(losses, lhist.ptr, (size_t)nsteps * 8, hipMemcpyDeviceToHost, s));
  MF_HIP(hipStreamSynchronize(s));
  return MF_OK;
}

// ------------------------------------------------------------------ preconditioner
int mf_precond_create_cnn(const mf_op *A, const mf_cnn *net, int nz, int ny, int nx, const int32_t *node_grid,
                          void *stream, mf_precond **out) {
  if (!A || !net || !node_grid || !out) return fail(MF_EINVAL, "mf_precond_create_cnn: null argument");
  if (A->ncomp != 1) return fail(MF_EUNSUPPORTED, "mf_precond_create_cnn: scalar spaces only");
  int rc = check_grid(1, nz, ny, nx, net->levels, "mf_precond_create_cnn");
  if (rc) return rc;
  const int64_t n = A->ndofs;
  if ((int64_t)nz * ny * nx != n) return fail(MF_EINVAL, "mf_precond_create_cnn: lattice size != number of nodes");
  // node_grid must be a bijection onto the lattice
  std::vector<uint8_t> seen((size_t)n, 0);
  for (int64_t i = 0; i < n; i++) {
    const int32_t gi = node_grid[i];
    if (gi < 0 || gi >= n || seen[gi]) return fail(MF_EINVAL, "mf_precond_create_cnn: node_grid is not a bijection");
    seen[gi] = 1;
  }
  hipStream_t s = (hipStream_t)stream;
  mf_precond *Pj = nullptr;
  rc = mf_precond_create_jacobi(A, stream, &Pj);
  if (rc) return rc;
  std::unique_ptr<mf_precond> P(Pj);
  P->kind = 1;
  P->net = net;
  P->gz = nz;
  P->gy = ny;
  P->gx = nx;
  // grid index per internal dof (internal node i is user node perm[i])
  std::vector<int32_t> gi((size_t)n);
  if (A->identity) {
    std::memcpy(gi.data(), node_grid, (size_t)n * 4);
  } else {
    MF_HIP(hipMemcpy(gi.data(), A->perm.ptr, (size_t)n * 4, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < n; i++) gi[i] = node_grid[gi[i]];
  }
  rc = P->gidx.alloc((size_t)n * 4);
  if (!rc) rc = P->sd.alloc((size_t)n * 8);
  if (!rc) rc = P->bc.alloc((size_t)n);
  if (!rc) rc = P->gin.alloc((size_t)n * 4);
  if (!rc) rc = P->gaux.alloc((size_t)n * 4);
  if (!rc) rc = P->acts.ensure(Grid3{1, nz, ny, nx}, net->C, net->levels);
  if (rc) return rc;
  MF_HIP(hipMemcpyAsync(P->gidx.ptr, gi.data(), (size_t)n * 4, hipMemcpyHostToDevice, s));
  MF_HIP(hipMemsetAsync(P->bc.ptr, 0, (size_t)n, s));
  if (A->n_bc_dofs > 0) rc = cnn_mark(A->bc_dofs.as<int32_t>(), A->n_bc_dofs, P->bc.as<uint8_t>(), s);
  if (!rc) rc = cg_sqrt(P->dinv.as<double>(), P->sd.as<double>(), n, s);
  if (rc) return rc;
  MF_HIP(hipStreamSynchronize(s));
  *out = P.release();
  return MF_OK;
}

}  // extern "C"

namespace mf {

// z = D^{-1/2} N(D^{-1/2} r) with constrained dofs passed through; internal numbering.
int precond_cnn_apply_internal(const mf_precond *P, const double *r, double *z, hipStream_t s) {
  int rc = cnn_to_grid(r, P->sd.as<double>(), +1, P->gidx.as<int32_t>(), P->gin.as<float>(), P->n, s);
  if (!rc) rc = cnn_forward(P->net->theta.as<float>(), P->net->L, P->gin.as<float>(), P->acts, s);
  if (!rc)
    rc = cnn_from_grid(P->acts.y.as<float>(), P->sd.as<double>(), P->gidx.as<int32_t>(), P->bc.as<uint8_t>(), r, z,
                       P->n, s);
  return rc;
}

}  // namespace mf

extern "C" {

int mf_precond_apply(const mf_precond *P, const double *r, double *z, void *stream) {
  if (!P || !r || !z) return fail(MF_EINVAL, "mf_precond_apply: null argument");
  hipStream_t s = (hipStream_t)stream;
  const int32_t *uoi = P->perm.as<int32_t>();
  const double *ri = r;
  double *zi = z;
  int rc = MF_OK;
  if (!P->identity) {
    rc = grow(P->wr, (size_t)P->n * 8);
    if (!rc) rc = grow(P->wz, (size_t)P->n * 8);
    if (!rc) rc = launch_to_internal<double>(uoi, P->nnodes, P->ncomp, r, P->wr.as<double>(), s);
    ri = P->wr.as<double>();
    zi = P->wz.as<double>();
  }
  if (rc) return rc;
  if (P->kind == 1) rc = precond_cnn_apply_internal(P, ri, zi, s);
  else rc = cg_scale(P->dinv.as<double>(), ri, zi, P->n, s);
  if (!rc && !P->identity) rc = launch_from_internal<double>(uoi, P->nnodes, P->ncomp, zi, z, false, s);
  return rc;
}

int mf_precond_harvest(const mf_precond *P, const double *r, const double *e, int ncrops, int n,
                       const int32_t *corners, float *r_out, float *e_out, void *stream) {
  if (!P || !r || !e || !corners || !r_out || !e_out) return fail(MF_EINVAL, "mf_precond_harvest: null argument");
  if (P->kind != 1) return fail(MF_EINVAL, "mf_precond_harvest: needs a lattice (learned) preconditioner");
  if (ncrops < 0 || n < 1) return fail(MF_EINVAL, "mf_precond_harvest: ncrops / n");
  for (int c = 0; c < ncrops; c++) {
    const int z = corners[3 * c], y = corners[3 * c + 1], x = corners[3 * c + 2];
    if (z < 0 || y < 0 || x < 0 || z + n > P->gz || y + n > P->gy || x + n > P->gx)
      return fail(MF_EINVAL, "mf_precond_harvest: crop outside the lattice");
  }
  if (ncrops == 0) return MF_OK;
  hipStream_t s = (hipStream_t)stream;
  DeviceBuffer dc;
  int rc = dc.alloc((size_t)ncrops * 3 * 4);
  if (rc) return rc;
  MF_HIP(hipMemcpyAsync(dc.ptr, corners, (size_t)ncrops * 3 * 4, hipMemcpyHostToDevice, s));
  const int32_t *uoi = P->perm.as<int32_t>();
  const double *ri = r, *ei = e;
  if (!P->identity) {
    rc = grow(P->wr, (size_t)P->n * 8);
    if (!rc) rc = grow(P->wz, (size_t)P->n * 8);
    if (!rc) rc = launch_to_internal<double>(uoi, P->nnodes, P->ncomp, r, P->wr.as<double>(), s);
    if (!rc) rc = launch_to_internal<double>(uoi, P->nnodes, P->ncomp, e, P->wz.as<double>(), s);
    ri = P->wr.as<double>();
    ei = P->wz.as<double>();
  }
  if (!rc) rc = cnn_to_grid(ri, P->sd.as<double>(), +1, P->gidx.as<int32_t>(), P->gin.as<float>(), P->n, s);
  if (!rc) rc = cnn_to_grid(ei, P->sd.as<double>(), -1, P->gidx.as<int32_t>(), P->gaux.as<float>(), P->n, s);
  if (!rc)
    rc = cnn_crops(P->gin.as<float>(), P->gaux.as<float>(), P->gz, P->gy, P->gx, dc.as<int32_t>(), ncrops, n, r_out,
                   e_out, s);
  if (rc) return rc;
  MF_HIP(hipStreamSynchronize(s));  // the corner buffer is freed on return
  return MF_OK;
}

}  // extern "C"

namespace mf {

// Workspaces of energy-loss training on a lattice preconditioner.
struct EnergyWork {
  DeviceBuffer z, Az, part, scal;
};

// One sample: r (FP64, internal numbering) -> loss into *loss_dev, gradient into net->grad.
static int energy_step(mf_cnn *net, const mf_precond *P, const mf_op *A, const double *ri, double *loss_dev,
                       EnergyWork &w, hipStream_t s) {
  const int64_t n = P->n;
  int rc = cnn_to_grid(ri, P->sd.as<double>(), +1, P->gidx.as<int32_t>(), P->gin.as<float>(), n, s);
  if (!rc) rc = cnn_forward(net->theta.as<float>(), net->L, P->gin.as<float>(), P->acts, s);
  if (!rc)
    rc = cnn_from_grid(P->acts.y.as<float>(), P->sd.as<double>(), P->gidx.as<int32_t>(), P->bc.as<uint8_t>(), ri,
                       w.z.as<double>(), n, s);
  if (!rc) rc = op_apply_internal(A, w.z.ptr, w.Az.ptr, s);
  if (!rc) rc = grow(net->gy, (size_t)n * 4);
  if (!rc)
    rc = cnn_energy(w.z.as<double>(), w.Az.as<double>(), ri, P->dinv.as<double>(), P->sd.as<double>(),
                    P->gidx.as<int32_t>(), P->bc.as<uint8_t>(), n, w.part.as<double>(), loss_dev,
                    w.scal.as<double>(), net->gy.as<float>(), s);
  if (!rc) rc = cnn_backward(net, P->acts, P->gin.as<float>(), net->gy.as<float>(), s);
  return rc;
}

static int energy_setup(mf_cnn *net, const mf_precond *P, const mf_op *A, EnergyWork &w, const char *who) {
  if (!net || !P || !A) return fail(MF_EINVAL, std::string(who) + ": null argument");
  if (P->kind != 1 || P->net != net)
    return fail(MF_EINVAL, std::string(who) + ": P must be a learned preconditioner built on this network");
  if (A->precision != MF_F64 || A->ndofs != P->n || A->numbering_id != P->numbering_id)
    return fail(MF_EINVAL, std::string(who) + ": A must be the FP64 operator P was built from");
  int rc = w.z.alloc((size_t)P->n * 8);
  if (!rc) rc = w.Az.alloc((size_t)P->n * 8);
  if (!rc) rc = w.part.alloc((size_t)cnn_energy_part_doubles() * 8);
  if (!rc) rc = w.scal.alloc(8);
  return rc;
}

// r (user numbering) -> internal numbering in P's workspace (or r itself)
static int to_internal_of(const mf_precond *P, const double *r, const double *&ri, hipStream_t s) {
  ri = r;
  if (P->identity) return MF_OK;
  int rc = grow(P->wr, (size_t)P->n * 8);
  if (!rc) rc = launch_to_internal<double>(P->perm.as<int32_t>(), P->nnodes, P->ncomp, r, P->wr.as<double>(), s);
  ri = P->wr.as<double>();
  return rc;
}

}  // namespace mf

extern "C" {

int mf_cnn_energy_loss_grad(mf_cnn *net, const mf_precond *P, const mf_op *A, const double *r, double *loss,
                            float *grad, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  EnergyWork w;
  int rc = energy_setup(net, P, A, w, "mf_cnn_energy_loss_grad");
  if (rc) return rc;
  if (!r) return fail(MF_EINVAL, "mf_cnn_energy_loss_grad: null r");
  DeviceBuffer ld;
  rc = ld.alloc(8);
  const double *ri = nullptr;
  if (!rc) rc = to_internal_of(P, r, ri, s);
  if (!rc) rc = energy_step(net, P, A, ri, ld.as<double>(), w, s);
  if (rc) return rc;
  if (grad) MF_HIP(hipMemcpyAsync(grad, net->grad.ptr, (size_t)net->L.nparams() * 4, hipMemcpyDeviceToDevice, s));
  if (loss) MF_HIP(hipMemcpyAsync(loss, ld.ptr, 8, hipMemcpyDeviceToHost, s));
  MF_HIP(hipStreamSynchronize(s));
  return MF_OK;
}

int mf_cnn_train_energy(mf_cnn *net, const mf_precond *P, const mf_op *A, int nsamples, const double *r,
                        int nsteps, const int32_t *order, float lr, double *losses, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  EnergyWork w;
  int rc = energy_setup(net, P, A, w, "mf_cnn_train_energy");
  if (rc) return rc;
  if (!r || !order || nsamples < 1 || nsteps < 0 || !(lr > 0.0f))
    return fail(MF_EINVAL, "mf_cnn_train_energy: r / order / nsamples / nsteps / lr");
  for (int i = 0; i < nsteps; i++)
    if (order[i] < 0 || order[i] >= nsamples) return fail(MF_EINVAL, "mf_cnn_train_energy: order index out of range");
  DeviceBuffer lhist;
  if (nsteps > 0) {
    rc = lhist.alloc((size_t)nsteps * 8);
    if (rc) return rc;
  }
  for (int st = 0; st < nsteps; st++) {
    const double *ri = nullptr;
    rc = to_internal_of(P, r + (int64_t)order[st] * P->n, ri, s);
    if (!rc) rc = energy_step(net, P, A, ri, lhist.as<double>() + st, w, s);
    if (!rc) rc = adam(net, lr, s);
    if (rc) return rc;
  }
  if (losses && nsteps > 0) MF_HIP(hipMemcpyAsync(losses, lhist.ptr, (size_t)nsteps * 8, hipMemcpyDeviceToHost, s));
  MF_HIP(hipStreamSynchronize(s));
  return MF_OK;
}

}  // extern "C"
