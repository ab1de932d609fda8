// C ABI of the batched apply: a list of operators (uneven meshes, degrees and
// column counts) applied in one persistent launch, optionally captured once in
// a HIP graph and replayed.
#include <algorithm>
#include <cstring>
#include <new>
#include <numeric>

#include "mf_internal.h"
#include "sf_common.h"

namespace mf {

struct Batch {
  int device = 0;
  int prec = MF_FP64;
  int cfg = 0;
  int nops = 0;
  std::vector<Operator*> ops;  // in the caller's order
  std::vector<int> nvec;
  std::vector<int> perm;       // work-list position -> caller index
  BatchOp* d_ops = nullptr;    // in work-list order
  int* d_counter = nullptr;
  int64_t total_items = 0, total_lines = 0;
  int grid[kBatchCfgs] = {0, 0, 0};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

static int batch_tile_rt(int prec, int cfg, int p) {
  // runtime mirror of batch_tile for kinds q = p + 1
  switch (cfg) {
    case 0: return batch_tile(prec, 0, p + 1, p + 1);
    case 1: return batch_tile(prec, 1, p + 1, p + 1);
    default: return batch_tile(prec, 2, p + 1, p + 1);
  }
}

// Build the device op table for launch shape `cfg` (tiles depend on it).
static int build_table(Batch* b, int cfg) {
  std::vector<BatchOp> host(b->nops);
  int64_t items = 0, lines = 0;
  for (int k = 0; k < b->nops; ++k) {
    const int i = b->perm[k];
    const Operator* op = b->ops[i];
    const int B = batch_tile_rt(b->prec, cfg, op->p);
    BatchOp& d = host[k];
    d.map = op->d_map;
    d.order = op->d_order;
    d.geo = op->d_geo;
    d.vq = op->d_vq;
    d.ncells = op->ncells;
    d.ntiles = (b->nvec[i] + B - 1) / B;
    d.p = op->p;
    for (int j = 0; j < 3; ++j) d.nodes[j] = (int)op->nodes[j];
    d.item_begin = items;
    d.line_begin = lines;
    d.grid = op->grid;
    items += op->ncells * d.ntiles;
    lines += op->nodes[1] * op->nodes[2];
  }
  if (items >= ((int64_t)1 << 31)) return fail(MF_ERR_UNSUPPORTED, "more than 2^31 work items");
  hipError_t err = hipMemcpy(b->d_ops, host.data(), host.size() * sizeof(BatchOp),
                             hipMemcpyHostToDevice);
  if (err != hipSuccess) return hip_fail(err, "hipMemcpy");
  b->total_items = items;
  b->total_lines = lines;
  b->cfg = cfg;
  return MF_OK;
}

static int fill_ptrs(const Batch* b, const double* const* X, double* const* Y, const int64_t* ldx,
                     const int64_t* ldy, BatchPtrs& p) {
  if (!X || !Y) return fail(MF_ERR_ARG, "X and Y arrays must be non-NULL");
  std::memset(&p, 0, sizeof(p));
  for (int k = 0; k < b->nops; ++k) {
    const int i = b->perm[k];
    const int64_t lx = ldx ? ldx[i] : b->nvec[i], ly = ldy ? ldy[i] : b->nvec[i];
    if (!X[i] || !Y[i]) return fail(MF_ERR_ARG, "NULL multivector in the batch");
    if (lx < b->nvec[i] || ly < b->nvec[i]) return fail(MF_ERR_ARG, "ld < nvec in the batch");
    p.X[k] = X[i];
    p.Y[k] = Y[i];
    p.ldx[k] = lx;
    p.ldy[k] = ly;
    p.nvec[k] = b->nvec[i];
  }
  // outputs must not overlap each other or any input
  for (int k = 0; k < b->nops; ++k) {
    const int64_t nd = b->ops[b->perm[k]]->ndofs;
    const char* y0 = reinterpret_cast<const char*>(p.Y[k]);
    const char* y1 = y0 + ((nd - 1) * p.ldy[k] + p.nvec[k]) * sizeof(double);
    for (int j = 0; j < b->nops; ++j) {
      const int64_t nj = b->ops[b->perm[j]]->ndofs;
      const char* x0 = reinterpret_cast<const char*>(p.X[j]);
      const char* x1 = x0 + ((nj - 1) * p.ldx[j] + p.nvec[j]) * sizeof(double);
      if (y0 < x1 && x0 < y1) return fail(MF_ERR_ARG, "an output overlaps an input of the batch");
      if (j != k) {
        const char* z0 = reinterpret_cast<const char*>(p.Y[j]);
        const char* z1 = z0 + ((nj - 1) * p.ldy[j] + p.nvec[j]) * sizeof(double);
        if (y0 < z1 && z0 < y1) return fail(MF_ERR_ARG, "two outputs of the batch overlap");
      }
    }
  }
  return MF_OK;
}

static int enqueue(Batch* b, const BatchPtrs& p, hipStream_t s) {
  hipError_t err = launch_reset_counter(b->d_counter, s);
  if (err == hipSuccess) err = launch_batch_zero(b->d_ops, b->nops, p, b->total_lines, s);
  if (err == hipSuccess)
    err = launch_batched(b->prec, b->cfg, b->d_ops, b->nops, b->total_items, b->d_counter, p,
                         b->grid[b->cfg], s);
  if (err != hipSuccess) return hip_fail(err, "batched launch");
  return MF_OK;
}

}  // namespace mf

using namespace mf;

extern "C" {

int mf_batch_create(int nops, mf_operator* const* ops, const int* nvec, int prec, mf_batch** out) {
  if (!out) return fail(MF_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (nops < 1 || nops > kMaxBatch) return fail(MF_ERR_ARG, "nops must be in [1, 64]");
  if (!ops || !nvec) return fail(MF_ERR_ARG, "ops and nvec must be non-NULL");
  if (prec != MF_FP64 && prec != MF_FP32_MFMA && prec != MF_BF16_MFMA)
    return fail(MF_ERR_UNSUPPORTED, "unknown precision");
  Batch* b = new (std::nothrow) Batch();
  if (!b) return fail(MF_ERR_OOM, "host allocation failed");
  b->prec = prec;
  b->nops = nops;
  for (int i = 0; i < nops; ++i) {
    Operator* op = reinterpret_cast<Operator*>(ops[i]);
    if (!op) {
      delete b;
      return fail(MF_ERR_ARG, "NULL operator in the batch");
    }
    if (op->p < kBatchMinP || op->p > kBatchMaxP || op->q != op->p + 1 || !op->box) {
      delete b;
      return fail(MF_ERR_UNSUPPORTED,
                  "batched kinds: axis-aligned cells, q = p + 1, p in [2, 8]");
    }
    if (nvec[i] < 1) {
      delete b;
      return fail(MF_ERR_ARG, "nvec must be >= 1");
    }
    b->ops.push_back(op);
    b->nvec.push_back(nvec[i]);
  }
  // heaviest items first: degree, then cells x columns
  b->perm.resize(nops);
  std::iota(b->perm.begin(), b->perm.end(), 0);
  std::stable_sort(b->perm.begin(), b->perm.end(), [&](int a, int c) {
    if (b->ops[a]->p != b->ops[c]->p) return b->ops[a]->p > b->ops[c]->p;
    return b->ops[a]->ncells * b->nvec[a] > b->ops[c]->ncells * b->nvec[c];
  });
  hipError_t err = hipGetDevice(&b->device);
  int cus = 0;
  if (err == hipSuccess) err = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device);
  if (err == hipSuccess) err = hipMalloc(&b->d_ops, nops * sizeof(BatchOp));
  if (err == hipSuccess) err = hipMalloc(&b->d_counter, sizeof(int));
  if (err != hipSuccess) {
    mf_batch_destroy(reinterpret_cast<mf_batch*>(b));
    return hip_fail(err, "batch setup");
  }
  for (int c = 0; c < kBatchCfgs; ++c) {
    const int per_cu = batched_blocks_per_cu(prec, c);
    b->grid[c] = std::max(1, per_cu) * cus;
  }
  if (int s = build_table(b, 0)) {
    mf_batch_destroy(reinterpret_cast<mf_batch*>(b));
    return s;
  }
  *out = reinterpret_cast<mf_batch*>(b);
  return MF_OK;
}

void mf_batch_destroy(mf_batch* handle) {
  if (!handle) return;
  Batch* b = reinterpret_cast<Batch*>(handle);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->d_ops) (void)hipFree(b->d_ops);
  if (b->d_counter) (void)hipFree(b->d_counter);
  delete b;
}

int mf_batch_set_launch(mf_batch* handle, int cfg) {
  if (!handle) return fail(MF_ERR_ARG, "batch is NULL");
  if (cfg < 0 || cfg >= kBatchCfgs) return fail(MF_ERR_ARG, "cfg out of range");
  Batch* b = reinterpret_cast<Batch*>(handle);
  return build_table(b, cfg);
}

int mf_batch_apply(mf_batch* handle, const double* const* X, double* const* Y, const int64_t* ldx,
                   const int64_t* ldy, void* stream) {
  if (!handle) return fail(MF_ERR_ARG, "batch is NULL");
  Batch* b = reinterpret_cast<Batch*>(handle);
  BatchPtrs p;
  if (int s = fill_ptrs(b, X, Y, ldx, ldy, p)) return s;
  return enqueue(b, p, static_cast<hipStream_t>(stream));
}

int mf_batch_capture(mf_batch* handle, const double* const* X, double* const* Y,
                     const int64_t* ldx, const int64_t* ldy, void* stream) {
  if (!handle) return fail(MF_ERR_ARG, "batch is NULL");
  if (!stream) return fail(MF_ERR_ARG, "capture needs a non-null stream");
  Batch* b = reinterpret_cast<Batch*>(handle);
  BatchPtrs p;
  if (int s = fill_ptrs(b, X, Y, ldx, ldy, p)) return s;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (b->exec) {
    (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  if (b->graph) {
    (void)hipGraphDestroy(b->graph);
    b->graph = nullptr;
  }
  hipError_t err = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (err != hipSuccess) return hip_fail(err, "hipStreamBeginCapture");
  const int st = enqueue(b, p, s);
  hipGraph_t g = nullptr;
  err = hipStreamEndCapture(s, &g);
  if (st) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (err != hipSuccess) return hip_fail(err, "hipStreamEndCapture");
  b->graph = g;
  err = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
  if (err != hipSuccess) return hip_fail(err, "hipGraphInstantiate");
  return MF_OK;
}

int mf_batch_replay(mf_batch* handle, void* stream) {
  if (!handle) return fail(MF_ERR_ARG, "batch is NULL");
  Batch* b = reinterpret_cast<Batch*>(handle);
  if (!b->exec) return fail(MF_ERR_ARG, "no captured graph: call mf_batch_capture first");
  hipError_t err = hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream));
  if (err != hipSuccess) return hip_fail(err, "hipGraphLaunch");
  return MF_OK;
}

int mf_batch_info(const mf_batch* handle, int64_t* items, int* cfg, int* grid) {
  if (!handle) return fail(MF_ERR_ARG, "batch is NULL");
  const Batch* b = reinterpret_cast<const Batch*>(handle);
  if (items) *items = b->total_items;
  if (cfg) *cfg = b->cfg;
  if (grid) *grid = b->grid[b->cfg];
  return MF_OK;
}

}  // extern "C"
