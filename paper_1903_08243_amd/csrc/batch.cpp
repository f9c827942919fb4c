// Batched solves: many hex operators of uneven size and degree solved together.
//
// Each CG iteration of the whole batch is a fixed sequence of launches: one
// persistent batched operator launch over a device work list of (operator,
// cell-batch range) items, then one launch per vector stage over the
// concatenated vectors of all systems with one-thread-per-system finalizes. A
// chunk of iterations is captured once into a hipGraph and replayed until all
// systems have stopped; stopped systems cost no operator work (their items are
// skipped) and their vector updates are no-ops.
//
// The launch form is a tuning parameter: the work-list kernel with its granularity
// (cell batches per item) and persistent grid size, or each live system's own
// operator kernels (its tile shape and scatter, as in a single solve; chunks are then
// launched directly, since the set of live systems changes); mf_batch_autotune times
// the candidates on the device and caches the winner in a text file.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <memory>
#include <sstream>
#include <string>

#include "batch_internal.h"

namespace mf {

static constexpr int BCHUNK = 8;              // CG iterations per graph replay
static constexpr int64_t VCH = 1 << 12;        // vector chunk length (16 elements per thread)

template <typename T> struct HostBatchOp {  // mirrors HexBatchOp<T> in hex_kernels.hip
  HexArgs<T> a;
  int N;
  int pad;
};
struct HostBatchItem {  // mirrors HexBatchItem
  int32_t op, pad;
  int64_t b0, b1;
};

}  // namespace mf

struct mf_batch {
  // all fields are set at creation; vectors are bound to the caller's pointers
  int nsys = 0, kind = 0;
  bool refine = false;
  std::vector<const mf_op *> A64, A32;
  std::vector<const mf_precond *> M;
  std::vector<int64_t> off;
  int64_t ntot = 0;
  std::vector<double *> b_user, x_user;
  mf::DeviceBuffer b, x, r, p, Ap, p32, Ap32, d, dinv, part, st, chunks, cptr;
  mf::DeviceBuffer ops64x, ops_in, items;  // op tables: FP64 residual (x -> Ap), inner (p -> Ap / p32 -> Ap32)
  int nch = 0, nitems = 0, grid = 0, items_per = 1;  // grid 0: one wavefront per item; -1: per-system kernels
  std::vector<char> live;                            // per-system launches: systems not yet stopped
  int64_t resident = 0;
  hipStream_t s = nullptr;
  hipEvent_t ev = nullptr;
  mf::CgState *host_st = nullptr;
  hipGraphExec_t exec = nullptr;
  ~mf_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (host_st) (void)hipHostFree(host_st);
    if (ev) (void)hipEventDestroy(ev);
    if (s) (void)hipStreamDestroy(s);
  }
};

namespace mf {

static BatchVec vec_desc(const mf_batch *B) {
  return BatchVec{B->chunks.as<VChunk>(), B->nch, B->cptr.as<int32_t>(), B->nsys, B->part.as<double>()};
}

template <typename T>
static HostBatchOp<T> batch_op(const mf_op *op, const void *x, void *y) {
  HostBatchOp<T> o{};
  o.a = HexArgs<T>{op->map.as<int32_t>(), op->geo.as<T>(), op->has_coef ? op->coef.as<T>() : nullptr,
                   (const T *)x, (T *)y, 0, op->ncells, op->ncomp, nullptr, 0, 0};
  o.N = op->degree + 1;
  return o;
}

template <typename T>
static int upload_ops(mf::DeviceBuffer &buf, const std::vector<HostBatchOp<T>> &v, hipStream_t s) {
  int rc = buf.alloc(v.size() * sizeof(HostBatchOp<T>));
  if (rc) return rc;
  MF_HIP(hipMemcpyAsync(buf.ptr, v.data(), v.size() * sizeof(HostBatchOp<T>), hipMemcpyHostToDevice, s));
  return MF_OK;
}

// Work list: every system's cell batches split into items of `per` batches. System
// after system for the one-wavefront-per-item launch (which hands each XCD a
// contiguous range, so an operator's neighbouring cells share one L2); interleaved
// across systems for the persistent launch, so concurrent wavefronts spread over
// the operators.
static int build_items(mf_batch *B, int per) {
  std::vector<std::vector<HostBatchItem>> lists(B->nsys);
  size_t longest = 0;
  for (int i = 0; i < B->nsys; i++) {
    const mf_op *op = B->A64[i];
    const int epb = hex_cells_per_batch(op->degree + 1);
    const int64_t nb = (op->ncells + epb - 1) / epb;
    for (int64_t b0 = 0; b0 < nb; b0 += per) lists[i].push_back(HostBatchItem{i, 0, b0, std::min(nb, b0 + per)});
    longest = std::max(longest, lists[i].size());
  }
  std::vector<HostBatchItem> items;
  if (B->grid == 0) {
    for (int i = 0; i < B->nsys; i++) items.insert(items.end(), lists[i].begin(), lists[i].end());
  } else {
    for (size_t j = 0; j < longest; j++)
      for (int i = 0; i < B->nsys; i++)
        if (j < lists[i].size()) items.push_back(lists[i][j]);
  }
  int rc = B->items.alloc(items.size() * sizeof(HostBatchItem));
  if (rc) return rc;
  MF_HIP(hipMemcpyAsync(B->items.ptr, items.data(), items.size() * sizeof(HostBatchItem), hipMemcpyHostToDevice, B->s));
  MF_HIP(hipStreamSynchronize(B->s));
  B->nitems = (int)items.size();
  B->items_per = per;
  return MF_OK;
}

// y = A x for all systems (x, y given by the op table); stopped systems skipped when st != null.
static int batch_apply(mf_batch *B, const mf::DeviceBuffer &ops, int precision, void *y, const CgState *st) {
  const int *stop = st ? (const int *)((const char *)st + offsetof(CgState, stop)) : nullptr;
  const int stride = (int)(sizeof(CgState) / sizeof(int));
  const BatchVec v = vec_desc(B);
  int rc;
  if (B->grid < 0) {
    // each live system's own operator kernels, accumulating into its cleared output
    const bool outer = &ops == &B->ops64x;
    rc = st ? (precision == MF_F64 ? batch_fill(v, (double *)y, st, B->s) : batch_fill(v, (float *)y, st, B->s))
            : (precision == MF_F64 ? launch_fill<double>((double *)y, 0.0, B->ntot, B->s)
                                   : launch_fill<float>((float *)y, 0.0f, B->ntot, B->s));
    for (int i = 0; i < B->nsys && !rc; i++) {
      if (st && !B->live[i]) continue;
      const int64_t o = B->off[i];
      if (precision == MF_F32) {
        rc = op_apply_internal_acc(B->A32[i], B->p32.as<float>() + o, (float *)y + o, B->s);
      } else {
        const double *in = (outer ? B->x.as<double>() : B->p.as<double>()) + o;
        rc = op_apply_internal_acc(B->A64[i], in, (double *)y + o, B->s);
      }
    }
    return rc;
  }
  if (precision == MF_F64) {
    rc = st ? batch_fill(v, (double *)y, st, B->s) : launch_fill<double>((double *)y, 0.0, B->ntot, B->s);
    if (!rc) rc = launch_hex_batch<double>(B->kind, ops.ptr, B->items.ptr, B->nitems, B->grid, stop, stride, B->s);
  } else {
    rc = st ? batch_fill(v, (float *)y, st, B->s) : launch_fill<float>((float *)y, 0.0f, B->ntot, B->s);
    if (!rc) rc = launch_hex_batch<float>(B->kind, ops.ptr, B->items.ptr, B->nitems, B->grid, stop, stride, B->s);
  }
  return rc;
}

static int read_states(mf_batch *B) {
  MF_HIP(hipMemcpyAsync(B->host_st, B->st.ptr, sizeof(CgState) * B->nsys, hipMemcpyDeviceToHost, B->s));
  MF_HIP(hipStreamSynchronize(B->s));
  return MF_OK;
}

static int write_states(mf_batch *B) {
  MF_HIP(hipMemcpyAsync(B->st.ptr, B->host_st, sizeof(CgState) * B->nsys, hipMemcpyHostToDevice, B->s));
  return MF_OK;
}

static int record_chunk(mf_batch *B) {
  const BatchVec v = vec_desc(B);
  const bool a32 = B->refine;
  CgState *st = B->st.as<CgState>();
  for (int j = 0; j < BCHUNK; j++) {
    int rc = batch_apply(B, B->ops_in, a32 ? MF_F32 : MF_F64, a32 ? B->Ap32.ptr : B->Ap.ptr, st);
    if (!rc)
      rc = batch_step_after_apply(v, B->x.as<double>(), B->r.as<double>(), B->p.as<double>(),
                                  a32 ? B->p32.as<float>() : nullptr, a32 ? B->Ap32.ptr : B->Ap.ptr, a32,
                                  B->dinv.ptr ? B->dinv.as<double>() : nullptr, st, B->s);
    if (rc) return rc;
  }
  return MF_OK;
}

static int ensure_graph(mf_batch *B) {
  if (B->exec) return MF_OK;
  hipGraph_t g = nullptr;
  MF_HIP(hipStreamBeginCapture(B->s, hipStreamCaptureModeThreadLocal));
  int rc = record_chunk(B);
  hipError_t e = hipStreamEndCapture(B->s, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(MF_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    B->exec = nullptr;
    return fail(MF_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  return MF_OK;
}

static int64_t batch_resident(mf_batch *B) {
  int dev = 0, cus = 256, per_cu = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  // one 64-thread workgroup per wavefront; query the occupancy of the widest kernel
  per_cu = 4;
  return (int64_t)cus * per_cu;
}

}  // namespace mf

using namespace mf;

extern "C" {

int mf_batch_create(int nsys, const mf_op *const *A64, const mf_op *const *A32, const mf_precond *const *M,
                    const double *const *b, double *const *x, void *stream, mf_batch **out) {
  if (nsys <= 0 || !A64 || !b || !x || !out) return fail(MF_EINVAL, "mf_batch_create: bad arguments");
  std::unique_ptr<mf_batch> B(new (std::nothrow) mf_batch);
  if (!B) return fail(MF_ENOMEM, "mf_batch_create: host allocation");
  B->nsys = nsys;
  B->refine = A32 != nullptr;
  B->kind = A64[0]->kind;
  B->off.assign(nsys + 1, 0);
  for (int i = 0; i < nsys; i++) {
    const mf_op *a = A64[i];
    if (!a || a->cell_type != MF_CELL_HEX || a->precision != MF_F64 || a->kind != B->kind || a->degree > 5 ||
        a->n_bc_dofs != 0 || a->ncomp != 1)
      return fail(MF_EUNSUPPORTED, "mf_batch_create: operators must be scalar FP64 hex operators of one kind, "
                                   "degree <= 5, without constraints");
    if (A32) {
      const mf_op *f = A32[i];
      if (!f || f->precision != MF_F32 || f->numbering_id != a->numbering_id || f->kind != a->kind)
        return fail(MF_EINVAL, "mf_batch_create: A32[i] must be the FP32 operator on A64[i]'s space");
    }
    if (M && M[i] && (M[i]->kind != 0 || M[i]->numbering_id != a->numbering_id))
      return fail(MF_EINVAL, "mf_batch_create: M[i] must be a Jacobi preconditioner of A64[i]");
    if (!b[i] || !x[i]) return fail(MF_EINVAL, "mf_batch_create: null vector");
    B->A64.push_back(a);
    B->A32.push_back(A32 ? A32[i] : nullptr);
    B->M.push_back(M ? M[i] : nullptr);
    B->b_user.push_back((double *)b[i]);
    B->x_user.push_back(x[i]);
    B->off[i + 1] = B->off[i] + a->ndofs;
  }
  B->ntot = B->off[nsys];
  if (sizeof(HostBatchOp<double>) != hex_batch_op_bytes(MF_F64) || sizeof(HostBatchOp<float>) != hex_batch_op_bytes(MF_F32) ||
      sizeof(HostBatchItem) != hex_batch_item_bytes())
    return fail(MF_EDEVICE, "mf_batch_create: work-list record layout mismatch");
  MF_HIP(hipStreamCreateWithFlags(&B->s, hipStreamNonBlocking));
  MF_HIP(hipEventCreateWithFlags(&B->ev, hipEventDisableTiming));
  MF_HIP(hipHostMalloc((void **)&B->host_st, sizeof(CgState) * nsys, hipHostMallocDefault));
  MF_HIP(hipEventRecord(B->ev, (hipStream_t)stream));
  MF_HIP(hipStreamWaitEvent(B->s, B->ev, 0));
  const size_t n8 = (size_t)B->ntot * 8, n4 = (size_t)B->ntot * 4;
  int rc = MF_OK;
  for (DeviceBuffer *buf : {&B->b, &B->x, &B->r, &B->p, &B->Ap, &B->d})
    if (!rc) rc = buf->alloc(n8);
  if (!rc && B->refine) rc = B->p32.alloc(n4);
  if (!rc && B->refine) rc = B->Ap32.alloc(n4);
  if (rc) return rc;
  // preconditioner: concatenated inverse diagonals (1 where a system has none)
  bool anyM = false;
  for (auto m : B->M) anyM |= m != nullptr;
  if (anyM) {
    rc = B->dinv.alloc(n8);
    if (rc) return rc;
    for (int i = 0; i < nsys; i++) {
      double *dst = B->dinv.as<double>() + B->off[i];
      if (B->M[i]) MF_HIP(hipMemcpyAsync(dst, B->M[i]->dinv.ptr, (size_t)B->A64[i]->ndofs * 8, hipMemcpyDeviceToDevice, B->s));
      else if ((rc = launch_fill<double>(dst, 1.0, B->A64[i]->ndofs, B->s))) return rc;
    }
  }
  // vector chunks
  std::vector<VChunk> ch;
  std::vector<int32_t> cp(nsys + 1, 0);
  for (int i = 0; i < nsys; i++) {
    for (int64_t s0 = B->off[i]; s0 < B->off[i + 1]; s0 += VCH)
      ch.push_back(VChunk{i, 0, s0, std::min(VCH, B->off[i + 1] - s0)});
    cp[i + 1] = (int32_t)ch.size();
  }
  B->nch = (int)ch.size();
  if ((rc = B->chunks.alloc(ch.size() * sizeof(VChunk))) || (rc = B->cptr.alloc(cp.size() * 4)) ||
      (rc = B->part.alloc((size_t)2 * B->nch * 8)) || (rc = B->st.alloc(sizeof(CgState) * nsys)))
    return rc;
  MF_HIP(hipMemcpyAsync(B->chunks.ptr, ch.data(), ch.size() * sizeof(VChunk), hipMemcpyHostToDevice, B->s));
  MF_HIP(hipMemcpyAsync(B->cptr.ptr, cp.data(), cp.size() * 4, hipMemcpyHostToDevice, B->s));
  // operator tables
  std::vector<HostBatchOp<double>> t64x, t64p;
  std::vector<HostBatchOp<float>> t32p;
  for (int i = 0; i < nsys; i++) {
    const int64_t o = B->off[i];
    t64x.push_back(batch_op<double>(B->A64[i], B->x.as<double>() + o, B->Ap.as<double>() + o));
    if (B->refine) t32p.push_back(batch_op<float>(B->A32[i], B->p32.as<float>() + o, B->Ap32.as<float>() + o));
    else t64p.push_back(batch_op<double>(B->A64[i], B->p.as<double>() + o, B->Ap.as<double>() + o));
  }
  if ((rc = upload_ops(B->ops64x, t64x, B->s))) return rc;
  rc = B->refine ? upload_ops(B->ops_in, t32p, B->s) : upload_ops(B->ops_in, t64p, B->s);
  if (rc) return rc;
  B->resident = batch_resident(B.get());
  B->grid = 0;
  if ((rc = build_items(B.get(), 1))) return rc;
  MF_HIP(hipStreamSynchronize(B->s));
  *out = B.release();
  return MF_OK;
}

void mf_batch_destroy(mf_batch *B) {
  if (!B) return;
  (void)hipDeviceSynchronize();
  delete B;
}

int mf_batch_get_tuning(const mf_batch *B, int *items_per, int *grid) {
  if (!B) return fail(MF_EINVAL, "mf_batch_get_tuning: null batch");
  if (items_per) *items_per = B->items_per;
  if (grid) *grid = B->grid;
  return MF_OK;
}

int mf_batch_set_tuning(mf_batch *B, int items_per, int grid) {
  if (!B || items_per < 1 || grid < -1 || (grid <= 0 && items_per != 1))
    return fail(MF_EINVAL, "mf_batch_set_tuning: items_per >= 1, grid >= -1 (grid 0 and -1 need items_per 1)");
  if (B->exec) {
    (void)hipGraphExecDestroy(B->exec);
    B->exec = nullptr;
  }
  B->grid = grid;
  return build_items(B, items_per);
}

int mf_batch_apply(mf_batch *B, int inner, void *stream) {
  if (!B) return fail(MF_EINVAL, "mf_batch_apply: null batch");
  MF_HIP(hipEventRecord(B->ev, (hipStream_t)stream));
  MF_HIP(hipStreamWaitEvent(B->s, B->ev, 0));
  int rc = inner ? batch_apply(B, B->ops_in, B->refine ? MF_F32 : MF_F64, B->refine ? B->Ap32.ptr : B->Ap.ptr, nullptr)
                 : batch_apply(B, B->ops64x, MF_F64, B->Ap.ptr, nullptr);
  if (rc) return rc;
  MF_HIP(hipEventRecord(B->ev, B->s));
  MF_HIP(hipStreamWaitEvent((hipStream_t)stream, B->ev, 0));
  return MF_OK;
}

int mf_batch_apply_user(mf_batch *B, int inner, const void *const *x, void *const *y, void *stream) {
  if (!B || !x || !y) return fail(MF_EINVAL, "mf_batch_apply_user: null argument");
  for (int i = 0; i < B->nsys; i++)
    if (!x[i] || !y[i]) return fail(MF_EINVAL, "mf_batch_apply_user: null vector");
  MF_HIP(hipEventRecord(B->ev, (hipStream_t)stream));
  MF_HIP(hipStreamWaitEvent(B->s, B->ev, 0));
  const bool f32 = inner && B->refine;
  // the operator table of the launch reads from and writes to these concatenated
  // internal buffers (see mf_batch_create)
  void *in = !inner ? B->x.ptr : (f32 ? B->p32.ptr : B->p.ptr);
  void *out = f32 ? B->Ap32.ptr : B->Ap.ptr;
  int rc = MF_OK;
  for (int i = 0; i < B->nsys && !rc; i++) {
    const mf_op *a = B->A64[i];
    const int64_t o = B->off[i];
    if (f32) {
      float *dst = (float *)in + o;
      if (a->identity) MF_HIP(hipMemcpyAsync(dst, x[i], (size_t)a->ndofs * 4, hipMemcpyDeviceToDevice, B->s));
      else rc = launch_to_internal<float>(a->perm.as<int32_t>(), a->nnodes, a->ncomp, (const float *)x[i], dst, B->s);
    } else {
      double *dst = (double *)in + o;
      if (a->identity) MF_HIP(hipMemcpyAsync(dst, x[i], (size_t)a->ndofs * 8, hipMemcpyDeviceToDevice, B->s));
      else rc = launch_to_internal<double>(a->perm.as<int32_t>(), a->nnodes, a->ncomp, (const double *)x[i], dst, B->s);
    }
  }
  if (rc) return rc;
  rc = inner ? batch_apply(B, B->ops_in, f32 ? MF_F32 : MF_F64, out, nullptr)
             : batch_apply(B, B->ops64x, MF_F64, out, nullptr);
  for (int i = 0; i < B->nsys && !rc; i++) {
    const mf_op *a = B->A64[i];
    const int64_t o = B->off[i];
    if (f32) {
      const float *src = (const float *)out + o;
      if (a->identity) MF_HIP(hipMemcpyAsync(y[i], src, (size_t)a->ndofs * 4, hipMemcpyDeviceToDevice, B->s));
      else rc = launch_from_internal<float>(a->perm.as<int32_t>(), a->nnodes, a->ncomp, src, (float *)y[i], false, B->s);
    } else {
      const double *src = (const double *)out + o;
      if (a->identity) MF_HIP(hipMemcpyAsync(y[i], src, (size_t)a->ndofs * 8, hipMemcpyDeviceToDevice, B->s));
      else rc = launch_from_internal<double>(a->perm.as<int32_t>(), a->nnodes, a->ncomp, src, (double *)y[i], false, B->s);
    }
  }
  if (rc) return rc;
  MF_HIP(hipEventRecord(B->ev, B->s));
  MF_HIP(hipStreamWaitEvent((hipStream_t)stream, B->ev, 0));
  return MF_OK;
}

int mf_batch_autotune(mf_batch *B, const char *cache_path, void *stream) {
  if (!B) return fail(MF_EINVAL, "mf_batch_autotune: null batch");
  // key: operator kind, precision of the inner action, device CU count, and the (degree, cells) multiset
  int dev = 0, cus = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  std::vector<std::pair<int, int64_t>> shape;
  for (auto a : B->A64) shape.push_back({a->degree, a->ncells});
  std::sort(shape.begin(), shape.end());
  uint64_t h = 1469598103934665603ull;
  for (auto &p : shape) {
    h = (h ^ (uint64_t)p.first) * 1099511628211ull;
    h = (h ^ (uint64_t)p.second) * 1099511628211ull;
  }
  char key[160];
  std::snprintf(key, sizeof key, "hexbatch kind=%d inner=%s cus=%d nsys=%d shape=%016llx", B->kind,
                B->refine ? "f32" : "f64", cus, B->nsys, (unsigned long long)h);
  if (cache_path) {
    std::ifstream f(cache_path);
    std::string line;
    while (std::getline(f, line)) {
      if (line.rfind(key, 0) == 0) {
        std::istringstream is(line.substr(std::strlen(key)));
        int per = 0, grid = 0;
        if (is >> per >> grid && per > 0 && grid >= -1) return mf_batch_set_tuning(B, per, grid);
      }
    }
  }
  (void)stream;
  const int pers[] = {1, 2, 4, 8, 16, 32};
  const int64_t grids[] = {-1, 0, B->resident, 2 * B->resident, 4 * B->resident};
  hipEvent_t e0, e1;
  MF_HIP(hipEventCreate(&e0));
  MF_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  int best_per = 1, best_grid = 0;
  const bool a32 = B->refine;
  for (int per : pers) {
    for (int64_t g : grids) {
      if (g <= 0 && per != 1) continue;
      B->grid = (int)g;
      int rc = build_items(B, per);
      if (rc) return rc;
      for (int w = 0; w < 2; w++)
        if ((rc = batch_apply(B, B->ops_in, a32 ? MF_F32 : MF_F64, a32 ? B->Ap32.ptr : B->Ap.ptr, nullptr))) return rc;
      MF_HIP(hipEventRecord(e0, B->s));
      for (int w = 0; w < 5; w++)
        if ((rc = batch_apply(B, B->ops_in, a32 ? MF_F32 : MF_F64, a32 ? B->Ap32.ptr : B->Ap.ptr, nullptr))) return rc;
      MF_HIP(hipEventRecord(e1, B->s));
      MF_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      MF_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) {
        best = ms;
        best_per = per;
        best_grid = (int)g;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  int rc = mf_batch_set_tuning(B, best_per, best_grid);
  if (rc) return rc;
  if (cache_path) {
    std::ofstream f(cache_path, std::ios::app);
    f << key << " " << best_per << " " << best_grid << " " << (best / 5.0f * 1000.0f) << " us\n";
  }
  return MF_OK;
}

int mf_batch_solve(mf_batch *B, double rtol, double inner_rtol, int maxit, mf_cg_info *infos, void *stream) {
  if (!B || !(rtol > 0.0) || maxit < 0) return fail(MF_EINVAL, "mf_batch_solve: bad arguments");
  const int ns = B->nsys;
  MF_HIP(hipEventRecord(B->ev, (hipStream_t)stream));
  MF_HIP(hipStreamWaitEvent(B->s, B->ev, 0));
  const BatchVec v = vec_desc(B);
  CgState *st = B->st.as<CgState>();
  const double *dinv = B->dinv.ptr ? B->dinv.as<double>() : nullptr;
  int rc = MF_OK;
  // user numbering -> internal numbering
  for (int i = 0; i < ns && !rc; i++) {
    const mf_op *a = B->A64[i];
    double *bi = B->b.as<double>() + B->off[i], *xi = B->x.as<double>() + B->off[i];
    if (a->identity) {
      MF_HIP(hipMemcpyAsync(bi, B->b_user[i], (size_t)a->ndofs * 8, hipMemcpyDeviceToDevice, B->s));
      MF_HIP(hipMemcpyAsync(xi, B->x_user[i], (size_t)a->ndofs * 8, hipMemcpyDeviceToDevice, B->s));
    } else {
      rc = launch_to_internal<double>(a->perm.as<int32_t>(), a->nnodes, a->ncomp, B->b_user[i], bi, B->s);
      if (!rc) rc = launch_to_internal<double>(a->perm.as<int32_t>(), a->nnodes, a->ncomp, B->x_user[i], xi, B->s);
    }
  }
  if (rc) return rc;
  // ||b||^2 per system
  if ((rc = launch_fill<double>(B->Ap.as<double>(), 0.0, B->ntot, B->s))) return rc;
  if ((rc = batch_residual(v, B->b.as<double>(), B->Ap.ptr, false, B->r.as<double>(), st, B->s))) return rc;
  if ((rc = read_states(B))) return rc;
  std::vector<double> bb(ns), rr(ns);
  std::vector<int> outer(ns, 0), inner(ns, 0), done(ns, 0);
  for (int i = 0; i < ns; i++) bb[i] = B->host_st[i].rr;
  // One preconditioned CG sequence per system, all systems in one launch sequence,
  // with reliable updates as in mf_cg_solve: whenever a live system's recursively
  // updated residual has dropped by delta since its last true residual, or a system
  // has newly stopped, the true residuals b - A64 x of all systems are formed in FP64
  // and replace r (r'z recomputed, search directions kept); a system whose true
  // residual misses the target resumes.
  const double delta = inner_rtol > 0.0 ? std::min(inner_rtol, 0.5) : 1e-3;
  int status = MF_OK;
  int nrel = 0;
  auto true_residuals = [&]() -> int {
    int r2 = batch_apply(B, B->ops64x, MF_F64, B->Ap.ptr, nullptr);
    if (!r2) r2 = batch_residual(v, B->b.as<double>(), B->Ap.ptr, false, B->r.as<double>(), st, B->s);
    return r2;
  };
  if ((rc = true_residuals())) return rc;
  if ((rc = read_states(B))) return rc;
  for (int i = 0; i < ns; i++) {
    CgState S{};
    S.tol2 = bb[i] == 0.0 ? DBL_MAX : rtol * rtol * bb[i];
    S.maxit = maxit;
    rr[i] = B->host_st[i].rr;
    B->host_st[i] = S;
  }
  if ((rc = write_states(B))) return rc;
  if ((rc = batch_init(v, B->r.as<double>(), dinv, B->p.as<double>(), B->refine ? B->p32.as<float>() : nullptr, st,
                       B->s)))
    return rc;
  // the accumulating inner action starts from a cleared output
  if (B->refine) {
    if ((rc = launch_fill<float>(B->Ap32.as<float>(), 0.0f, B->ntot, B->s))) return rc;
  } else if ((rc = launch_fill<double>(B->Ap.as<double>(), 0.0, B->ntot, B->s))) {
    return rc;
  }
  if ((rc = read_states(B))) return rc;
  std::vector<double> rr_ref(ns);
  std::vector<int> stopped(ns);
  for (int i = 0; i < ns; i++) {
    rr_ref[i] = B->host_st[i].rr;
    stopped[i] = B->host_st[i].stop;
  }
  bool all_stop = true;
  for (int i = 0; i < ns; i++) all_stop &= stopped[i] != 0;
  const bool direct = B->grid < 0;  // per-system kernels: the live set changes, no graph
  B->live.assign(ns, 1);
  if (!all_stop && !direct && (rc = ensure_graph(B))) return rc;
  while (!all_stop) {
    if (direct) {
      for (int i = 0; i < ns; i++) B->live[i] = B->host_st[i].stop ? 0 : 1;
      if ((rc = record_chunk(B))) return rc;
    } else {
      MF_HIP(hipGraphLaunch(B->exec, B->s));
    }
    if ((rc = read_states(B))) return rc;
    bool due = false, brk = false;
    all_stop = true;
    for (int i = 0; i < ns; i++) {
      const CgState &S = B->host_st[i];
      brk |= S.breakdown != 0;
      all_stop &= S.stop != 0;
      due |= (S.stop && !stopped[i]) || (!S.stop && S.rr < delta * rr_ref[i]);
    }
    if (brk) {
      status = fail(MF_EBREAKDOWN, "batched CG breakdown in at least one system");
      break;
    }
    if (!due && !all_stop) continue;
    // reliable update of every system (the accumulating inner action's output was
    // cleared by the last search-direction update)
    if ((rc = true_residuals())) return rc;
    if ((rc = batch_reliable(v, B->r.as<double>(), dinv, st, B->s))) return rc;
    if ((rc = read_states(B))) return rc;
    nrel++;
    all_stop = true;
    for (int i = 0; i < ns; i++) {
      rr_ref[i] = B->host_st[i].rr;
      stopped[i] = B->host_st[i].stop;
      all_stop &= stopped[i] != 0;
      brk |= B->host_st[i].breakdown != 0;
    }
    if (brk) {
      status = fail(MF_EBREAKDOWN, "batched CG breakdown in at least one system");
      break;
    }
  }
  for (int i = 0; i < ns; i++) {
    rr[i] = B->host_st[i].rr;
    outer[i] = 1 + nrel;
    inner[i] = B->host_st[i].iters;
  }
  // back to user numbering
  for (int i = 0; i < ns && !rc; i++) {
    const mf_op *a = B->A64[i];
    const double *xi = B->x.as<double>() + B->off[i];
    if (a->identity) MF_HIP(hipMemcpyAsync(B->x_user[i], xi, (size_t)a->ndofs * 8, hipMemcpyDeviceToDevice, B->s));
    else rc = launch_from_internal<double>(a->perm.as<int32_t>(), a->nnodes, a->ncomp, xi, B->x_user[i], false, B->s);
  }
  if (rc) return rc;
  MF_HIP(hipStreamSynchronize(B->s));
  bool all_conv = true;
  for (int i = 0; i < ns; i++) {
    if (infos) infos[i] = mf_cg_info{outer[i], inner[i], 0, bb[i] > 0 ? std::sqrt(rr[i] / bb[i]) : 0.0};
    all_conv &= bb[i] == 0.0 || rr[i] <= rtol * rtol * bb[i];
  }
  if (status == MF_OK && !all_conv) status = fail(MF_ENOTCONV, "batched CG: not every system reached the tolerance");
  return status;
}

}  // extern "C"
