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

static bool lattice_ok(int n) { return n >= 5 && (n - 1) % 4 == 0; }

int CnnActs::ensure(const Grid3 &g, int c) {
  if (g.B == g0.B && g.Z == g0.Z && g.Y == g0.Y && g.X == g0.X && c == C && h0.ptr) return MF_OK;
  g0 = g;
  g1 = coarser(g0);
  g2 = coarser(g1);
  C = 0;  // set once every buffer is allocated
  const size_t f0 = (size_t)g0.points() * c * 4, f1 = (size_t)g1.points() * c * 4, f2 = (size_t)g2.points() * c * 4;
  int rc = MF_OK;
  for (auto pr : {std::make_pair(&h0, f0), std::make_pair(&u0, f0), std::make_pair(&c1, f1), std::make_pair(&h1, f1),
                  std::make_pair(&u1, f1), std::make_pair(&g1b, f1), std::make_pair(&c2, f2), std::make_pair(&h2, f2),
                  std::make_pair(&g2b, f2), std::make_pair(&y, (size_t)g0.points() * 4)}) {
    DeviceBuffer &b = *pr.first;
    if (b.ptr) {
      (void)hipFree(b.ptr);
      b.ptr = nullptr;
      b.bytes = 0;
    }
    if (!rc) rc = b.alloc(pr.second);
  }
  if (!rc) C = c;
  return rc;
}

static const float *layer(const float *theta, const CnnLayout &L, int l) { return theta + L.off[l]; }

int cnn_forward(const float *theta, const CnnLayout &L, const float *x, CnnActs &a, hipStream_t s) {
  const int C = L.C;
  int rc = cnn_conv(x, layer(theta, L, 0), a.h0.as<float>(), nullptr, a.g0, 1, C, true, false, s);
  if (!rc) rc = cnn_restrict(a.h0.as<float>(), a.c1.as<float>(), nullptr, 1.0f, a.g0, C, s);
  if (!rc) rc = cnn_conv(a.c1.as<float>(), layer(theta, L, 1), a.h1.as<float>(), nullptr, a.g1, C, C, true, false, s);
  if (!rc) rc = cnn_restrict(a.h1.as<float>(), a.c2.as<float>(), nullptr, 1.0f, a.g1, C, s);
  if (!rc) rc = cnn_conv(a.c2.as<float>(), layer(theta, L, 2), a.h2.as<float>(), nullptr, a.g2, C, C, true, false, s);
  if (!rc) rc = cnn_conv(a.h2.as<float>(), layer(theta, L, 3), a.g2b.as<float>(), nullptr, a.g2, C, C, true, false, s);
  if (!rc) rc = cnn_prolong_add(a.g2b.as<float>(), a.h1.as<float>(), a.u1.as<float>(), nullptr, 1.0f, a.g1, C, s);
  if (!rc) rc = cnn_conv(a.u1.as<float>(), layer(theta, L, 4), a.g1b.as<float>(), nullptr, a.g1, C, C, true, false, s);
  if (!rc) rc = cnn_prolong_add(a.g1b.as<float>(), a.h0.as<float>(), a.u0.as<float>(), nullptr, 1.0f, a.g0, C, s);
  if (!rc) rc = cnn_conv(a.u0.as<float>(), layer(theta, L, 5), a.y.as<float>(), nullptr, a.g0, C, 1, false, false, s);
  return rc;
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

// Loss of the batch (x, t) and the gradient of every weight into net->grad.
// x, t: [B][Z][Y][X]; the loss (FP64) is left in net->loss on the device.
static int loss_grad(mf_cnn *net, const Grid3 &g, const float *x, const float *t, hipStream_t s) {
  const int C = net->C;
  const CnnLayout &L = net->L;
  CnnActs &a = net->acts;
  int rc = a.ensure(g, C);
  if (rc) return rc;
  const size_t f0 = (size_t)a.g0.points() * C * 4, f1 = (size_t)a.g1.points() * C * 4;
  int64_t pf = 0;
  for (const Grid3 *gg : {&a.g0, &a.g1, &a.g2}) {
    const int64_t v = cnn_wgrad_part_floats(*gg, C, C);
    pf = v > pf ? v : pf;
  }
  if (!rc) rc = grow(net->gy, (size_t)a.g0.points() * 4);
  if (!rc) rc = grow(net->gA, f0);
  if (!rc) rc = grow(net->gB, f1);
  if (!rc) rc = grow(net->gC, f1);
  if (!rc) rc = grow(net->part, (size_t)pf * 4);
  if (!rc) rc = grow(net->lpart, (size_t)cnn_loss_part_doubles(g.B) * 8);
  if (!rc) rc = grow(net->loss, 8);
  if (rc) return rc;
  const float *th = net->theta.as<float>();
  float *gr = net->grad.as<float>();
  float *part = net->part.as<float>();
  rc = cnn_forward(th, L, x, a, s);
  if (!rc) rc = cnn_loss(a.y.as<float>(), t, net->gy.as<float>(), net->loss.as<double>(), net->lpart.as<double>(),
                         g.B, (int64_t)g.Z * g.Y * g.X, s);
  // y = F u0
  float *gu0 = net->gA.as<float>();  // becomes g(h0) after the skip contribution
  if (!rc) rc = cnn_wgrad(a.u0.as<float>(), net->gy.as<float>(), gr + L.off[5], part, a.g0, C, 1, s);
  if (!rc) rc = cnn_conv(net->gy.as<float>(), layer(th, L, 5), gu0, nullptr, a.g0, 1, C, false, true, s);
  // u0 = P g1 + h0, g1 = relu(E u1): g(g1) = 8 R g(u0) masked by g1 > 0
  float *gg1 = net->gB.as<float>();
  if (!rc) rc = cnn_restrict(gu0, gg1, a.g1b.as<float>(), 8.0f, a.g0, C, s);
  float *gu1 = net->gC.as<float>();  // becomes g(h1)
  if (!rc) rc = cnn_wgrad(a.u1.as<float>(), gg1, gr + L.off[4], part, a.g1, C, C, s);
  if (!rc) rc = cnn_conv(gg1, layer(th, L, 4), gu1, nullptr, a.g1, C, C, false, true, s);
  // u1 = P g2 + h1, g2 = relu(D h2): g(g2) = 8 R g(u1) masked by g2 > 0 (coarsest grid; reuse gB's head)
  float *gg2 = net->gB.as<float>();
  if (!rc) rc = cnn_restrict(gu1, gg2, a.g2b.as<float>(), 8.0f, a.g1, C, s);
  // h2 = relu(C c2): g(h2) = D^T g(g2) masked by h2 > 0
  float *gh2 = net->gB.as<float>() + (size_t)a.g2.points() * C;
  if (!rc) rc = cnn_wgrad(a.h2.as<float>(), gg2, gr + L.off[3], part, a.g2, C, C, s);
  if (!rc) rc = cnn_conv(gg2, layer(th, L, 3), gh2, a.h2.as<float>(), a.g2, C, C, false, true, s);
  float *gc2 = net->gB.as<float>();  // g(g2) no longer needed
  if (!rc) rc = cnn_wgrad(a.c2.as<float>(), gh2, gr + L.off[2], part, a.g2, C, C, s);
  if (!rc) rc = cnn_conv(gh2, layer(th, L, 2), gc2, nullptr, a.g2, C, C, false, true, s);
  // c2 = R h1: g(h1) += R^T g(c2) = P g(c2) / 8, then masked by h1 > 0
  if (!rc) rc = cnn_prolong_add(gc2, gu1, gu1, a.h1.as<float>(), 0.125f, a.g1, C, s);
  float *gc1 = net->gB.as<float>();
  if (!rc) rc = cnn_wgrad(a.c1.as<float>(), gu1, gr + L.off[1], part, a.g1, C, C, s);
  if (!rc) rc = cnn_conv(gu1, layer(th, L, 1), gc1, nullptr, a.g1, C, C, false, true, s);
  // c1 = R h0: g(h0) = g(u0) + P g(c1) / 8, masked by h0 > 0
  if (!rc) rc = cnn_prolong_add(gc1, gu0, gu0, a.h0.as<float>(), 0.125f, a.g0, C, s);
  if (!rc) rc = cnn_wgrad(x, gu0, gr + L.off[0], part, a.g0, 1, C, s);
  (void)f1;
  return rc;
}

static int adam(mf_cnn *net, float lr, hipStream_t s) {
  net->step += 1;
  const double b1 = 0.9, b2 = 0.999;
  const double bc1 = 1.0 - std::pow(b1, (double)net->step), bc2 = 1.0 - std::pow(b2, (double)net->step);
  return cnn_adam(net->theta.as<float>(), net->grad.as<float>(), net->m.as<float>(), net->v.as<float>(),
                  net->L.nparams(), lr, (float)b1, (float)b2, 1e-8f, (float)bc1, (float)bc2, s);
}

static int check_grid(int B, int nz, int ny, int nx, const char *who) {
  if (B < 1 || !lattice_ok(nz) || !lattice_ok(ny) || !lattice_ok(nx))
    return fail(MF_EINVAL, std::string(who) + ": lattice sizes must be 4m+1 (m >= 1) and batch >= 1");
  return MF_OK;
}

}  // namespace mf

using namespace mf;

struct CnnFileHeader {
  char magic[8];
  int32_t channels, pad;
  int64_t nparams;
};

extern "C" {

int64_t mf_cnn_nparams(int channels) {
  if (channels != 4 && channels != 8 && channels != 16) return -1;
  return CnnLayout(channels).nparams();
}

int mf_cnn_create(int channels, const float *theta, mf_cnn **out) {
  if (!out || !theta) return fail(MF_EINVAL, "mf_cnn_create: null argument");
  if (channels != 4 && channels != 8 && channels != 16)
    return fail(MF_EUNSUPPORTED, "mf_cnn_create: channels must be 4, 8 or 16");
  std::unique_ptr<mf_cnn> net(new (std::nothrow) mf_cnn);
  if (!net) return fail(MF_ENOMEM, "mf_cnn_create: host allocation");
  net->C = channels;
  net->L = CnnLayout(channels);
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
  std::memcpy(h.magic, "MFCNN01", 8);
  h.channels = net->C;
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
  bool ok = std::fread(&h, sizeof h, 1, f) == 1 && std::memcmp(h.magic, "MFCNN01", 8) == 0 &&
            (h.channels == 4 || h.channels == 8 || h.channels == 16) && h.nparams == CnnLayout(h.channels).nparams();
  std::vector<float> th;
  if (ok) {
    th.resize((size_t)h.nparams);
    ok = std::fread(th.data(), 4, th.size(), f) == th.size();
  }
  std::fclose(f);
  if (!ok) return fail(MF_EINVAL, std::string("mf_cnn_load: not a network file: ") + path);
  return mf_cnn_create(h.channels, th.data(), out);
}

void mf_cnn_destroy(mf_cnn *net) {
  if (!net) return;
  (void)hipDeviceSynchronize();
  delete net;
}

int mf_cnn_forward(mf_cnn *net, int batch, int nz, int ny, int nx, const float *x, float *y, void *stream) {
  if (!net || !x || !y) return fail(MF_EINVAL, "mf_cnn_forward: null argument");
  int rc = check_grid(batch, nz, ny, nx, "mf_cnn_forward");
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const Grid3 g{batch, nz, ny, nx};
  rc = net->acts.ensure(g, net->C);
  if (!rc) rc = cnn_forward(net->theta.as<float>(), net->L, x, net->acts, s);
  if (rc) return rc;
  MF_HIP(hipMemcpyAsync(y, net->acts.y.ptr, (size_t)g.points() * 4, hipMemcpyDeviceToDevice, s));
  return MF_OK;
}

int mf_cnn_loss_grad(mf_cnn *net, int batch, int nz, int ny, int nx, const float *x, const float *t, double *loss,
                     float *grad, void *stream) {
  if (!net || !x || !t) return fail(MF_EINVAL, "mf_cnn_loss_grad: null argument");
  int rc = check_grid(batch, nz, ny, nx, "mf_cnn_loss_grad");
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
  int rc = check_grid(batch, n, n, n, "mf_cnn_train");
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
  int rc = check_grid(1, nz, ny, nx, "mf_precond_create_cnn");
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
  if (!rc) rc = P->acts.ensure(Grid3{1, nz, ny, nx}, net->C);
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
