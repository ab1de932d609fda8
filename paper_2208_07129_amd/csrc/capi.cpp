// C ABI of libmfmv: argument checking, operator setup and kernel dispatch.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <utility>

#include "mf_internal.h"
#include "sf_common.h"
#include "sf_tables.h"

namespace mf {

static thread_local std::string g_last_error;

int fail(int status, const std::string& msg) {
  g_last_error = msg;
  return status;
}

int hip_fail(hipError_t err, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(err);
  return MF_ERR_HIP;
}

hipError_t kernel_facts(const void* kernel, int nt, size_t lds, KernelFacts& out) {
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, KernelFacts> known;
  int dev = 0;
  hipError_t err = hipGetDevice(&dev);
  if (err != hipSuccess) return err;
  std::lock_guard<std::mutex> lock(mu);
  auto it = known.find({kernel, dev});
  if (it != known.end()) {
    out = it->second;
    return hipSuccess;
  }
  KernelFacts f;
  if (lds > 64 * 1024) {
    err = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
  }
  int n = 0;
  err = hipDeviceGetAttribute(&f.cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (err == hipSuccess) err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, nt, lds);
  if (err != hipSuccess) return err;
  f.per_cu = n < 1 ? 1 : n;
  known[{kernel, dev}] = f;
  out = f;
  return hipSuccess;
}

static int check_degree(int p) {
  if (p < 1 || p > kMaxP) return fail(MF_ERR_UNSUPPORTED, "p must be in [1, 10]");
  return MF_OK;
}

static int check_pq(int p, int q) {
  if (int s = check_degree(p)) return s;
  if (q < p + 1 || q > p + kMaxQExtra)
    return fail(MF_ERR_UNSUPPORTED,
                "q must be in [p+1, p+3]: the collocation factorisation needs q >= p+1");
  return MF_OK;
}

}  // namespace mf

using namespace mf;

extern "C" {

const char* mf_last_error(void) { return g_last_error.c_str(); }

int mf_num_cells(const mf_box_mesh* mesh, int64_t* ncells) {
  if (int s = validate_mesh(mesh)) return s;
  if (!ncells) return fail(MF_ERR_ARG, "ncells is NULL");
  *ncells = (int64_t)mesh->n[0] * mesh->n[1] * mesh->n[2];
  return MF_OK;
}

int mf_num_dofs(const mf_box_mesh* mesh, int p, int64_t* ndofs) {
  if (int s = validate_mesh(mesh)) return s;
  if (int s = check_degree(p)) return s;
  if (!ndofs) return fail(MF_ERR_ARG, "ndofs is NULL");
  *ndofs = nodes_per_dir(*mesh, p, 0) * nodes_per_dir(*mesh, p, 1) * nodes_per_dir(*mesh, p, 2);
  return MF_OK;
}

int mf_constrained_mask(const mf_box_mesh* mesh, int p, uint8_t* mask) {
  int64_t nd;
  if (int s = mf_num_dofs(mesh, p, &nd)) return s;
  if (!mask) return fail(MF_ERR_ARG, "mask is NULL");
  const int64_t Nx = nodes_per_dir(*mesh, p, 0), Ny = nodes_per_dir(*mesh, p, 1),
                Nz = nodes_per_dir(*mesh, p, 2);
  const bool dir = mesh->bc == MF_BC_DIRICHLET0;
  for (int64_t gz = 0; gz < Nz; ++gz)
    for (int64_t gy = 0; gy < Ny; ++gy)
      for (int64_t gx = 0; gx < Nx; ++gx) {
        const bool b = gx == 0 || gx == Nx - 1 || gy == 0 || gy == Ny - 1 || gz == 0 || gz == Nz - 1;
        mask[gx + Nx * (gy + Ny * gz)] = (dir && b) ? 1 : 0;
      }
  return MF_OK;
}

int mf_quad_points(const mf_box_mesh* mesh, int q, double* xq) {
  if (int s = validate_mesh(mesh)) return s;
  if (q < 1 || q > kMaxP + 1 + kMaxQExtra) return fail(MF_ERR_UNSUPPORTED, "q out of range");
  if (!xq) return fail(MF_ERR_ARG, "xq is NULL");
  Rule1D g = gauss_rule(q);
  double L[9];
  lin_matrix(*mesh, L);
  double h[3];
  for (int d = 0; d < 3; ++d) h[d] = (mesh->hi[d] - mesh->lo[d]) / mesh->n[d];
  int64_t idx = 0;
  for (int cz = 0; cz < mesh->n[2]; ++cz)
    for (int cy = 0; cy < mesh->n[1]; ++cy)
      for (int cx = 0; cx < mesh->n[0]; ++cx)
        for (int a3 = 0; a3 < q; ++a3)
          for (int a2 = 0; a2 < q; ++a2)
            for (int a1 = 0; a1 < q; ++a1) {
              const double y[3] = {mesh->lo[0] + h[0] * (cx + 0.5 * (g.x[a1] + 1.0)),
                                   mesh->lo[1] + h[1] * (cy + 0.5 * (g.x[a2] + 1.0)),
                                   mesh->lo[2] + h[2] * (cz + 0.5 * (g.x[a3] + 1.0))};
              for (int r = 0; r < 3; ++r)
                xq[idx * 3 + r] = L[3 * r] * y[0] + L[3 * r + 1] * y[1] + L[3 * r + 2] * y[2];
              ++idx;
            }
  return MF_OK;
}

int mf_basis_1d(int p, int q, double* xq, double* wq, double* xn, double* N, double* D, double* Dt) {
  if (int s = check_pq(p, q)) return s;
  Tables1D t = make_tables(p, q);
  auto put = [](double* dst, const std::vector<double>& v) {
    if (dst) std::memcpy(dst, v.data(), v.size() * sizeof(double));
  };
  put(xq, t.xq);
  put(wq, t.wq);
  put(xn, t.xn);
  put(N, t.N);
  put(D, t.D);
  put(Dt, t.Dt);
  return MF_OK;
}

int mf_create_operator(const mf_box_mesh* mesh, int p, int q, double mu, const double* Vq,
                       double sigma, mf_operator** out) {
  if (!out) return fail(MF_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (int s = validate_mesh(mesh)) return s;
  if (int s = check_pq(p, q)) return s;
  if (!std::isfinite(mu) || !std::isfinite(sigma)) return fail(MF_ERR_ARG, "mu and sigma must be finite");
  if (!apply_f64_supported(p, q)) return fail(MF_ERR_UNSUPPORTED, "no kernel built for this (p, q)");

  Operator* op = new (std::nothrow) Operator();
  if (!op) return fail(MF_ERR_OOM, "host allocation failed");
  op->p = p;
  op->q = q;
  op->np = p + 1;
  op->nq = q;
  op->mu = mu;
  op->sigma = sigma;
  op->cfg = -1;
  op->t = make_tables(p, q);
  const int np = op->np, nq = op->nq, np3 = np * np * np, nq3 = nq * nq * nq;
  const int64_t Nx = nodes_per_dir(*mesh, p, 0), Ny = nodes_per_dir(*mesh, p, 1),
                Nz = nodes_per_dir(*mesh, p, 2);
  op->ndofs = Nx * Ny * Nz;
  op->nodes[0] = Nx;
  op->nodes[1] = Ny;
  op->nodes[2] = Nz;
  for (int d = 0; d < 3; ++d) {
    op->grid.n[d] = mesh->n[d];
    op->grid.N[d] = (int)op->nodes[d];
  }
  op->grid.p = p;
  op->grid.dirichlet = mesh->bc == MF_BC_DIRICHLET0 ? 1 : 0;
  op->ncells = (int64_t)mesh->n[0] * mesh->n[1] * mesh->n[2];
  if (op->ndofs >= (int64_t)1 << 31) {
    delete op;
    return fail(MF_ERR_UNSUPPORTED, "more than 2^31-1 nodes");
  }
  const int64_t E = op->ncells;

  // Cell-to-node map (extraction Q of Sec. 3.2.3) with zero-Dirichlet nodes
  // marked -1: reading them as zero and skipping them on assembly is the
  // action of C and C^T for constraints with empty masters (Sec. 3.2.2).
  std::vector<int32_t> map(E * np3);
  std::vector<uint8_t> mask(op->ndofs);
  mf_constrained_mask(mesh, p, mask.data());
  const bool per = mesh->bc == MF_BC_PERIODIC;
  for (int64_t e = 0; e < E; ++e) {
    const int64_t cx = e % mesh->n[0], cy = (e / mesh->n[0]) % mesh->n[1],
                  cz = e / ((int64_t)mesh->n[0] * mesh->n[1]);
    for (int i3 = 0; i3 < np; ++i3)
      for (int i2 = 0; i2 < np; ++i2)
        for (int i1 = 0; i1 < np; ++i1) {
          int64_t gx = cx * p + i1, gy = cy * p + i2, gz = cz * p + i3;
          if (per) {
            gx %= Nx;
            gy %= Ny;
            gz %= Nz;
          }
          const int64_t g = gx + Nx * (gy + Ny * gz);
          map[e * np3 + i1 + np * (i2 + np * i3)] = mask[g] ? -1 : (int32_t)g;
        }
  }

  // Geometry (eq. sjacobian / eq. mjacobian): the cell map is affine, so J is
  // constant per cell: J = lin * diag(h/2).
  double L[9];
  lin_matrix(*mesh, L);
  double h[3];
  for (int d = 0; d < 3; ++d) h[d] = (mesh->hi[d] - mesh->lo[d]) / mesh->n[d];
  double G6[6];
  const double detJ = cell_factor(L, h, mu, G6);
  // axis-aligned cells: the off-diagonal entries vanish exactly (J diagonal)
  op->box = G6[1] == 0.0 && G6[2] == 0.0 && G6[4] == 0.0;
  // lumped (GLL) mass data: det J and the GLL weights 2 / (p (p+1) P_p(x_i)^2)
  op->detj = detJ;
  {
    const std::vector<double> xg = gll_points(p);
    for (int i = 0; i <= p; ++i) {
      double P = 0.0, dP = 0.0, ddP = 0.0;
      ct::legendre(p, xg[i], P, dP, ddP);
      op->wgll[i] = 2.0 / (p * (p + 1.0) * P * P);
    }
  }
  std::vector<double> geo(E * 6);
  for (int64_t e = 0; e < E; ++e)
    for (int k = 0; k < 6; ++k) geo[e * 6 + k] = G6[k];
  std::vector<double> vq(E * nq3);
  for (int64_t k = 0; k < E * nq3; ++k) {
    const double v = Vq ? Vq[k] : 0.0;
    if (!std::isfinite(v)) {
      delete op;
      return fail(MF_ERR_ARG, "Vq holds a non-finite value");
    }
    vq[k] = detJ * (v + sigma);
  }

  hipError_t err = hipGetDevice(&op->device);
  if (err != hipSuccess) {
    delete op;
    return hip_fail(err, "hipGetDevice");
  }
  auto alloc_copy = [&](void** dst, const void* src, size_t bytes) -> int {
    hipError_t e2 = hipMalloc(dst, bytes);
    if (e2 != hipSuccess) {
      *dst = nullptr;
      return e2 == hipErrorOutOfMemory ? fail(MF_ERR_OOM, "hipMalloc failed") : hip_fail(e2, "hipMalloc");
    }
    e2 = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
    if (e2 != hipSuccess) return hip_fail(e2, "hipMemcpy");
    return MF_OK;
  };
  const int nn[3] = {mesh->n[0], mesh->n[1], mesh->n[2]};
  std::vector<int32_t> order = cell_order(nn);
  int s = alloc_copy((void**)&op->d_map, map.data(), map.size() * sizeof(int32_t));
  if (!s) s = alloc_copy((void**)&op->d_order, order.data(), order.size() * sizeof(int32_t));
  if (!s) s = alloc_copy((void**)&op->d_geo, geo.data(), geo.size() * sizeof(double));
  if (!s) s = alloc_copy((void**)&op->d_vq, vq.data(), vq.size() * sizeof(double));
  if (!s) {
    // 1D sums of the diagonal (mf_diagonal): [w N^2 (nq x np) | a | b | c]
    const Tables1D& t = op->t;
    std::vector<double> tab((size_t)q * np + 3 * np, 0.0);
    for (int a = 0; a < q; ++a)
      for (int i = 0; i < np; ++i) {
        const double n = t.N[a * np + i], d = t.D[a * np + i], w = t.wq[a];
        tab[a * np + i] = w * n * n;
        tab[q * np + i] += w * d * d;
        tab[q * np + np + i] += w * n * n;
        tab[q * np + 2 * np + i] += w * d * n;
      }
    s = alloc_copy((void**)&op->d_dtab, tab.data(), tab.size() * sizeof(double));
  }
  if (s) {
    mf_destroy_operator(reinterpret_cast<mf_operator*>(op));
    return s;
  }
  *out = reinterpret_cast<mf_operator*>(op);
  return MF_OK;
}

void mf_destroy_operator(mf_operator* handle) {
  if (!handle) return;
  Operator* op = reinterpret_cast<Operator*>(handle);
  batch_cache_forget(op);
  if (op->d_map) (void)hipFree(op->d_map);
  if (op->d_order) (void)hipFree(op->d_order);
  if (op->d_colour_order) (void)hipFree(op->d_colour_order);
  for (hipEvent_t e : op->ev) (void)hipEventDestroy(e);
  if (op->d_geo) (void)hipFree(op->d_geo);
  if (op->d_vq) (void)hipFree(op->d_vq);
  if (op->d_dtab) (void)hipFree(op->d_dtab);
  if (op->d_sets) (void)hipFree(op->d_sets);
  if (op->d_cidx) (void)hipFree(op->d_cidx);
  if (op->d_cw) (void)hipFree(op->d_cw);
  if (op->d_zrows) (void)hipFree(op->d_zrows);
  if (op->d_detj) (void)hipFree(op->d_detj);
  delete op;
}

int mf_operator_info(const mf_operator* handle, int64_t* ndofs, int64_t* ncells, int* p, int* q) {
  if (!handle) return fail(MF_ERR_ARG, "operator is NULL");
  const Operator* op = reinterpret_cast<const Operator*>(handle);
  if (ndofs) *ndofs = op->ndofs;
  if (ncells) *ncells = op->ncells;
  if (p) *p = op->p;
  if (q) *q = op->q;
  return MF_OK;
}

int mf_cell_order(const mf_operator* handle, int32_t* order) {
  if (!handle) return fail(MF_ERR_ARG, "operator is NULL");
  if (!order) return fail(MF_ERR_ARG, "order is NULL");
  const Operator* op = reinterpret_cast<const Operator*>(handle);
  if (op->refined) return fail(MF_ERR_UNSUPPORTED, "a refined operator has no grid cell order");
  const std::vector<int32_t> o = cell_order(op->grid.n);
  std::memcpy(order, o.data(), o.size() * sizeof(int32_t));
  return MF_OK;
}

int mf_fma_probe(int blocks, int64_t iters, double* out, void* stream) {
  if (!out) return fail(MF_ERR_ARG, "out is NULL");
  if (blocks < 1 || iters < 1) return fail(MF_ERR_ARG, "need blocks, iters >= 1");
  hipError_t err = launch_fma_probe(blocks, iters, out, static_cast<hipStream_t>(stream));
  if (err != hipSuccess) return hip_fail(err, "FMA probe launch");
  return MF_OK;
}

int mf_set_deterministic(mf_operator* handle, int on) {
  if (!handle) return fail(MF_ERR_ARG, "operator is NULL");
  Operator* op = reinterpret_cast<Operator*>(handle);
  if (!on) {
    op->deterministic = false;
    return MF_OK;
  }
  if (!op->box)
    return fail(MF_ERR_UNSUPPORTED,
                "the deterministic assembly is built for box meshes of axis-aligned cells");
  if (!op->d_colour_order) {
    bool periodic[3];
    for (int d = 0; d < 3; ++d) periodic[d] = op->grid.N[d] == op->grid.n[d] * op->p;
    const std::vector<int> col = cell_colours(op->grid.n, periodic);
    if (col.empty())
      return fail(MF_ERR_UNSUPPORTED,
                  "a periodic direction with one cell: the cell meets itself (no colouring)");
    // the processing order, stably sorted by colour
    const std::vector<int32_t> order = cell_order(op->grid.n);
    std::vector<int32_t> sorted;
    sorted.reserve(order.size());
    std::vector<int64_t> off(1, 0);
    for (int c = 0; c < 27; ++c) {
      for (int32_t e : order)
        if (col[e] == c) sorted.push_back(e);
      if ((int64_t)sorted.size() > off.back()) off.push_back((int64_t)sorted.size());
    }
    const size_t bytes = sorted.size() * sizeof(int32_t);
    hipError_t err = hipMalloc((void**)&op->d_colour_order, bytes);
    if (err != hipSuccess) {
      op->d_colour_order = nullptr;
      return err == hipErrorOutOfMemory ? fail(MF_ERR_OOM, "hipMalloc (colour order)")
                                        : hip_fail(err, "hipMalloc");
    }
    err = hipMemcpy(op->d_colour_order, sorted.data(), bytes, hipMemcpyHostToDevice);
    if (err != hipSuccess) {
      (void)hipFree(op->d_colour_order);
      op->d_colour_order = nullptr;
      return hip_fail(err, "hipMemcpy (colour order)");
    }
    op->coff = off;
  }
  op->deterministic = true;
  return MF_OK;
}

static bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes) {
  const char* ca = static_cast<const char*>(a);
  const char* cb = static_cast<const char*>(b);
  return ca < cb + bbytes && cb < ca + abytes;
}

}  // extern "C"

int mf::apply_dispatch(mf_operator* handle, const double* X, double* Y, int nvec, int64_t ldx,
                       int64_t ldy, int prec, void* stream, bool accumulate) {
  if (!handle) return fail(MF_ERR_ARG, "operator is NULL");
  if (!X || !Y) return fail(MF_ERR_ARG, "X and Y must be non-NULL device pointers");
  if (nvec < 1) return fail(MF_ERR_ARG, "nvec must be >= 1");
  if (ldx < nvec || ldy < nvec) return fail(MF_ERR_ARG, "ldx and ldy must be >= nvec");
  Operator* op = reinterpret_cast<Operator*>(handle);
  const size_t xb = ((op->ndofs - 1) * ldx + nvec) * sizeof(double);
  const size_t yb = ((op->ndofs - 1) * ldy + nvec) * sizeof(double);
  if (overlaps(X, xb, Y, yb)) return fail(MF_ERR_ARG, "X and Y overlap");
  if (prec != MF_FP64 && prec != MF_FP32 && prec != MF_BF16)
    return fail(MF_ERR_UNSUPPORTED, "unknown precision");
  const bool mixed = prec != MF_FP64;
  // mixed precision: axis-aligned cells; on a refined map FP32 vector only
  const bool map32 = mixed && op->map_box && prec == MF_FP32;
  if (mixed && !op->box && !map32)
    return fail(MF_ERR_UNSUPPORTED,
                "mixed precision is built for axis-aligned cells only (FP32 on refined meshes)");
  hipStream_t s = static_cast<hipStream_t>(stream);

  ApplyLaunch a{};
  a.grid = op->grid;
  a.map = op->d_map;
  a.order = op->d_order;
  a.geo = op->d_geo;
  a.vq = op->d_vq;
  a.X = X;
  a.Y = Y;
  a.ldx = ldx;
  a.ldy = ldy;
  a.ncells = op->ncells;
  a.nvec = nvec;
  a.threads = 256;
  a.vtile = choose_vtile_f64(op->np, op->nq, nvec);
  a.cfg = mixed ? op->mcfg : op->cfg;
  if (a.cfg < 0) {
    const auto it = op->tuned.find({prec, nvec});
    if (it != op->tuned.end())
      a.cfg = it->second;
    else
      a.cfg = mixed ? choose_cfg_mixed(op->np, op->nq, nvec, prec)
                    : choose_cfg_box(op->np, op->nq, nvec);
  }
  if (mixed && a.cfg >= kMixedMfmaCfgs && !box_pairs_ok(X, Y, nvec, ldx, ldy))
    a.cfg = vec32_cfg_single(a.cfg);
  if (!mixed && op->box && !box_pairs_ok(X, Y, nvec, ldx, ldy))
    a.cfg = box_cfg_single(op->np, op->nq, a.cfg);
  a.accumulate = accumulate;

  hipEvent_t* ev = nullptr;
  if (op->ev_slots > 0) {
    ev = &op->ev[3 * op->ev_next];
    op->ev_next = (op->ev_next + 1) % op->ev_slots;
    if (op->ev_count < op->ev_slots) ++op->ev_count;
    (void)hipEventRecord(ev[0], s);
  }
  hipError_t err = hipSuccess;
  if (!accumulate) {
    // the box kernels store cell-interior rows and add to the others
    err = op->box       ? launch_zero_shared_rows(Y, op->nodes, op->p, nvec, ldy, s)
        : op->map_box ? launch_zero_listed_rows(Y, op->d_zrows, op->nzrows, nvec, ldy, s)
                      : launch_zero_rows(Y, op->ndofs, nvec, ldy, s);
    if (err != hipSuccess) return hip_fail(err, "zero kernel launch");
  }
  if (ev) (void)hipEventRecord(ev[1], s);
  auto launch = [&]() {
    return map32   ? launch_apply_box_map32(*op, a, s)
           : mixed ? launch_apply_mixed(*op, a, prec, s)
                 : (op->box       ? (a.cfg == kBoxMfmaCfg ? launch_apply_mfma(*op, a, s)
                                                            : launch_apply_box(*op, a, s))
                    : op->map_box ? launch_apply_box_map(*op, a, s)
                                  : launch_apply_f64(*op, a, s));
  };
  if (op->deterministic && op->box) {
    // one launch per colour, in colour order: within a launch every shared row
    // receives at most one atomic addition per column, so its sum is formed in
    // a fixed order
    for (size_t c = 0; c + 1 < op->coff.size() && err == hipSuccess; ++c) {
      a.order = op->d_colour_order + op->coff[c];
      a.ncells = op->coff[c + 1] - op->coff[c];
      err = launch();
    }
  } else {
    err = launch();
  }
  if (err != hipSuccess) return hip_fail(err, "apply kernel launch");
  if (ev) (void)hipEventRecord(ev[2], s);
  return MF_OK;
}

extern "C" {

int mf_apply(mf_operator* handle, const double* X, double* Y, int nvec, int64_t ldx, int64_t ldy,
             int prec, void* stream) {
  return apply_dispatch(handle, X, Y, nvec, ldx, ldy, prec, stream, /*accumulate=*/false);
}

int mf_apply_add(mf_operator* handle, const double* X, double* Y, int nvec, int64_t ldx,
                 int64_t ldy, int prec, void* stream) {
  return apply_dispatch(handle, X, Y, nvec, ldx, ldy, prec, stream, /*accumulate=*/true);
}

int mf_set_launch(mf_operator* handle, int general, int cfg) {
  if (!handle) return fail(MF_ERR_ARG, "operator is NULL");
  Operator* op = reinterpret_cast<Operator*>(handle);
  if (cfg < -1 || cfg >= kBoxCfgs) return fail(MF_ERR_ARG, "cfg out of range");
  if (cfg >= 0 && !apply_box_supported(op->p, op->q, cfg))
    return fail(MF_ERR_UNSUPPORTED, "launch shape does not fit this (p, q)");
  if (general) {  // the general kernel takes cells in index order: no colour order
    op->box = false;
    op->map_box = false;
    op->deterministic = false;
  }
  op->cfg = cfg;
  return MF_OK;
}

int mf_set_launch_mixed(mf_operator* handle, int cfg) {
  if (!handle) return fail(MF_ERR_ARG, "operator is NULL");
  Operator* op = reinterpret_cast<Operator*>(handle);
  if (cfg < -1 || cfg >= kMixedCfgs) return fail(MF_ERR_ARG, "cfg out of range");
  if (cfg >= 0 && !apply_mixed_supported(op->p, op->q, cfg))
    return fail(MF_ERR_UNSUPPORTED, "launch shape does not fit this (p, q)");
  op->mcfg = cfg;
  return MF_OK;
}

int mf_timing(mf_operator* handle, int slots) {
  if (!handle) return fail(MF_ERR_ARG, "operator is NULL");
  if (slots < 0 || slots > 100000) return fail(MF_ERR_ARG, "slots out of range");
  Operator* op = reinterpret_cast<Operator*>(handle);
  for (hipEvent_t e : op->ev) (void)hipEventDestroy(e);
  op->ev.assign(3 * (size_t)slots, nullptr);
  for (auto& e : op->ev) {
    hipError_t err = hipEventCreate(&e);
    if (err != hipSuccess) {
      op->ev_slots = 0;
      return hip_fail(err, "hipEventCreate");
    }
  }
  op->ev_slots = slots;
  op->ev_next = 0;
  op->ev_count = 0;
  return MF_OK;
}

int mf_timing_read(mf_operator* handle, int* count, double* zero_ms, double* kernel_ms) {
  if (!handle) return fail(MF_ERR_ARG, "operator is NULL");
  Operator* op = reinterpret_cast<Operator*>(handle);
  double z = 0.0, k = 0.0;
  for (int i = 0; i < op->ev_count; ++i) {
    hipError_t err = hipEventSynchronize(op->ev[3 * i + 2]);
    if (err != hipSuccess) return hip_fail(err, "hipEventSynchronize");
    float a = 0.f, b = 0.f;
    err = hipEventElapsedTime(&a, op->ev[3 * i], op->ev[3 * i + 1]);
    if (err == hipSuccess) err = hipEventElapsedTime(&b, op->ev[3 * i + 1], op->ev[3 * i + 2]);
    if (err != hipSuccess) return hip_fail(err, "hipEventElapsedTime");
    z += a;
    k += b;
  }
  if (count) *count = op->ev_count;
  if (zero_ms) *zero_ms = z;
  if (kernel_ms) *kernel_ms = k;
  op->ev_count = 0;
  op->ev_next = 0;
  return MF_OK;
}

int mf_timing_samples(mf_operator* handle, int cap, double* zero_ms, double* kernel_ms, int* count) {
  if (!handle || !count) return fail(MF_ERR_ARG, "operator and count must be non-NULL");
  if (cap < 0 || (cap > 0 && (!zero_ms || !kernel_ms))) return fail(MF_ERR_ARG, "bad output arrays");
  Operator* op = reinterpret_cast<Operator*>(handle);
  // the ring holds the last ev_count applies; the oldest is at ev_next when full
  const int n = op->ev_count;
  const int first = n < op->ev_slots ? 0 : op->ev_next;
  int w = 0;
  for (int i = 0; i < n; ++i) {
    const int j = (first + i) % op->ev_slots;
    hipError_t err = hipEventSynchronize(op->ev[3 * j + 2]);
    float a = 0.f, b = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&a, op->ev[3 * j], op->ev[3 * j + 1]);
    if (err == hipSuccess) err = hipEventElapsedTime(&b, op->ev[3 * j + 1], op->ev[3 * j + 2]);
    if (err != hipSuccess) return hip_fail(err, "hipEvent timing");
    if (w < cap) {
      zero_ms[w] = a;
      kernel_ms[w] = b;
      ++w;
    }
  }
  *count = w;
  op->ev_count = 0;
  op->ev_next = 0;
  return MF_OK;
}

int mf_zero(double* Y, int64_t nrows, int ncols, int64_t ld, void* stream) {
  if (!Y) return fail(MF_ERR_ARG, "Y is NULL");
  if (nrows < 0 || ncols < 1 || ld < ncols) return fail(MF_ERR_ARG, "need nrows >= 0, 1 <= ncols <= ld");
  if (nrows == 0) return MF_OK;
  hipError_t err = launch_zero_rows(Y, nrows, ncols, ld, static_cast<hipStream_t>(stream));
  if (err != hipSuccess) return hip_fail(err, "zero kernel launch");
  return MF_OK;
}

}  // extern "C"
