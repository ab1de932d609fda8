// Dispatch of the fused apply by polynomial degree, and the zero-fill kernel.
#include "mf_internal.h"
#include "sf_common.h"

namespace mf {

namespace {

// Y rows [0, nrows) x columns [0, ncols) := 0.  A kernel rather than a memset
// so that it also clears strided (ld > ncols) outputs and can be captured in a
// graph.
__global__ void zero_rows_kernel(double* __restrict__ Y, int64_t nrows, int ncols, int64_t ld) {
  const int64_t total = nrows * ncols;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / ncols, c = i % ncols;
    Y[r * ld + c] = 0.0;
  }
}

// X[i] := a fixed pseudo-random value in [-1, 1) (an integer hash of i): the
// input the launch-shape tuner times the kernels on.
__global__ void fill_pattern_kernel(double* __restrict__ X, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t h = (uint64_t)i * 0x9E3779B97F4A7C15ull;
    h ^= h >> 29;
    X[i] = (double)(h >> 44) * (1.0 / (1 << 19)) - 1.0;
  }
}

// FP64 FMA issue-rate probe: every thread runs `iters` rounds of 8
// independent FMA chains (no loads), then writes their sum so nothing is
// dropped.  8 iters x 2 flops per thread and round.
__global__ void __launch_bounds__(256) fma_probe_kernel(int64_t iters, double seed, double* out) {
  double v[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) v[c] = seed + c + threadIdx.x * 1e-3;
  const double a = 0.999999, b = 1e-7;
#pragma unroll 4
  for (int64_t i = 0; i < iters; ++i)
#pragma unroll
    for (int c = 0; c < 8; ++c) v[c] = fma(v[c], a, b);
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < 8; ++c) s += v[c];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// Node lines (gy, gz) of the Nx x Ny x Nz grid, each taken whole by one
// workgroup (a grid-stride loop when the grid is smaller than the line count).
// A line on a cell-face plane (gy or gz a multiple of p) is zeroed whole;
// otherwise only the rows gx = 0, p, 2p, ... are.  Threads form (row, column)
// pairs, the columns of a row on cw = 2^cw_log2 consecutive lanes (the next
// power of two >= ncols, at most 64), so narrow multivectors keep every lane
// busy and wide ones store 64 contiguous columns at a time.  Rows of
// cell-interior nodes are skipped: the box kernel writes them.
__global__ void zero_shared_rows_kernel(double* __restrict__ Y, int Nx, int Ny, int p, int ncols,
                                        int64_t ld, int64_t lines, int cw_log2) {
  const int cw = 1 << cw_log2;
  const int c0 = threadIdx.x & (cw - 1);
  const int r0 = threadIdx.x >> cw_log2, rstep = blockDim.x >> cw_log2;
  for (int64_t line = blockIdx.x; line < lines; line += gridDim.x) {
    const int gy = (int)(line % Ny), gz = (int)(line / Ny);
    const bool full = (gy % p == 0) || (gz % p == 0);
    const int step = full ? 1 : p;
    const int nrows = full ? Nx : (Nx + p - 1) / p;
    double* base = Y + line * Nx * ld;
    for (int r = r0; r < nrows; r += rstep) {
      double* row = base + (int64_t)r * step * ld;
      for (int c = c0; c < ncols; c += cw) row[c] = 0.0;
    }
  }
}

// Chebyshev step initialisation: the face rows of the zero fill's line walk
// (cell-interior rows are written by the fused kernel) get b Y + c Xp, and
// constrained rows (the boundary of a zero-Dirichlet mesh) 0.
__global__ void cheb_init_kernel(const double* __restrict__ Y, const double* Xp, double* Out,
                                 int Nx, int Ny, int Nz, int p, int dirichlet, int ncols,
                                 int64_t ld, double b, double c) {
  const int line = blockIdx.x;
  const int gy = line % Ny, gz = line / Ny;
  const bool full = (gy % p == 0) || (gz % p == 0);
  const bool yz_bnd = dirichlet && (gy == 0 || gy == Ny - 1 || gz == 0 || gz == Nz - 1);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int step = full ? 1 : p;
  for (int gx = wave * step; gx < Nx; gx += nw * step) {
    const int64_t row = ((int64_t)line * Nx + gx) * ld;
    const bool cons = yz_bnd || (dirichlet && (gx == 0 || gx == Nx - 1));
    for (int j = lane; j < ncols; j += 64) {
      double v = 0.0;
      if (!cons) {
        v = b * Y[row + j];
        if (Xp) v = fma(c, Xp[row + j], v);
      }
      Out[row + j] = v;
    }
  }
}

// GLL-lumped mass: per cell and local node, w_a w_b w_c det J added to the
// node's row (the GLL rule of the element's own nodes makes the mass
// diagonal).
struct GllWeights {
  double w[kMaxP + 1];
};
__global__ void gll_mass_kernel(GridDesc g, int np, GllWeights wt, double detj,
                                double* __restrict__ m) {
  const int e = blockIdx.x;
  const int cx = e % g.n[0], cy = (e / g.n[0]) % g.n[1], cz = e / (g.n[0] * g.n[1]);
  const int F = np * np * np;
  for (int i = threadIdx.x; i < F; i += blockDim.x) {
    const int i1 = i % np, i2 = (i / np) % np, i3 = i / (np * np);
    const int node = grid_node(g, cx, cy, cz, i1, i2, i3);
    if (node >= 0) unsafeAtomicAdd(m + node, wt.w[i1] * wt.w[i2] * wt.w[i3] * detj);
  }
}
__global__ void inv_sqrt_kernel(double* __restrict__ m, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    m[i] = m[i] > 0.0 ? 1.0 / sqrt(m[i]) : 0.0;
}

// Batched form: kBatchZeroSplit workgroups per node plane gz of any operator of
// the batch, each taking a contiguous share of the plane's face rows
// (per-line workgroups are too small for the batch's small meshes and column
// counts).  A plane on a cell face (gz a multiple of p) is zeroed whole;
// otherwise its face rows are enumerated as k = 0 .. n-1: first the lines
// gy = 0, p, 2p, ... whole, then the rows gx = 0, p, 2p, ... of the other
// lines.  Lanes take columns in groups of the next power of two >= ncols (up
// to 64), so a wavefront stores 64 / group rows at a time.
constexpr int kBatchZeroSplit = 16;

__global__ void batch_zero_kernel(const BatchOp* __restrict__ ops,
                                  const uint8_t* __restrict__ plane_op, BatchPtrs ptrs,
                                  int64_t first) {
  const int64_t g = first + blockIdx.x;
  const int o = plane_op[g];
  const BatchOp& op = ops[o];
  const int gz = (int)(g - op.plane_begin);
  const int Nx = op.nodes[0], Ny = op.nodes[1], p = op.p;
  const int64_t ld = ptrs.ldy[o];
  const int ncols = ptrs.nvec[o];
  double* base = ptrs.Y[o] + (int64_t)gz * Nx * Ny * ld;
  const bool full = p == 1 || gz % p == 0;
  const int nyf = (Ny + p - 1) / p, nxf = (Nx + p - 1) / p;
  const int64_t nrows = full ? (int64_t)Nx * Ny : (int64_t)nyf * Nx + (int64_t)(Ny - nyf) * nxf;
  int lpr = 1;
  while (lpr < ncols && lpr < 64) lpr *= 2;
  const int rpw = 64 / lpr;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int sub = lane / lpr, c0 = lane % lpr;
  const int64_t k0 = nrows * blockIdx.y / gridDim.y, k1 = nrows * (blockIdx.y + 1) / gridDim.y;
  for (int64_t k = k0 + (int64_t)wave * rpw + sub; k < k1; k += (int64_t)nw * rpw) {
    int64_t row;
    if (full) {
      row = k;
    } else if (k < (int64_t)nyf * Nx) {
      row = (k / Nx) * p * (int64_t)Nx + k % Nx;
    } else {
      const int64_t kk = k - (int64_t)nyf * Nx;
      const int64_t j = kk / nxf;
      row = (j + j / (p - 1) + 1) * (int64_t)Nx + (kk % nxf) * p;
    }
    double* dst = base + row * ld;
    for (int c = c0; c < ncols; c += lpr) dst[c] = 0.0;
  }
}

}  // namespace

hipError_t launch_batch_zero(const BatchOp* ops, const uint8_t* plane_op, const BatchPtrs& ptrs,
                             int64_t first, int64_t planes, hipStream_t s) {
  if (planes < 1) return hipSuccess;
  hipLaunchKernelGGL(batch_zero_kernel, dim3((unsigned)planes, kBatchZeroSplit), dim3(256), 0, s,
                     ops, plane_op, ptrs, first);
  return hipGetLastError();
}

hipError_t launch_batched(int prec, int bcfg, const BatchOp* ops, const uint8_t* item_op,
                          const int64_t* bounds, const BatchPtrs& ptrs, int grid, hipStream_t s) {
#define MF_BATCH_CASE(P, C)                                                                  \
  if (prec == P && bcfg == C)                                                                \
    return launch_batched_kernel<P, C>(ops, item_op, bounds, ptrs, grid, s);
  MF_BATCH_CASE(MF_FP64, 0) MF_BATCH_CASE(MF_FP64, 1) MF_BATCH_CASE(MF_FP64, 2)
  MF_BATCH_CASE(MF_FP32, 0) MF_BATCH_CASE(MF_FP32, 1) MF_BATCH_CASE(MF_FP32, 2)
  MF_BATCH_CASE(MF_BF16, 0) MF_BATCH_CASE(MF_BF16, 1) MF_BATCH_CASE(MF_BF16, 2)
#undef MF_BATCH_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_batched_kind_any(int prec, int p, bool loop, const BatchOp* ops,
                                   const uint8_t* item_op,
                                   const int64_t* bounds, const BatchPtrs& ptrs, int grid,
                                   hipStream_t s) {
  if (prec == MF_FP64)
    return launch_batched_kind<MF_FP64>(p, loop, ops, item_op, bounds, ptrs, grid, s);
  if (prec == MF_FP32)
    return launch_batched_kind<MF_FP32>(p, loop, ops, item_op, bounds, ptrs, grid, s);
  if (prec == MF_BF16)
    return launch_batched_kind<MF_BF16>(p, loop, ops, item_op, bounds, ptrs, grid, s);
  return hipErrorInvalidValue;
}

int batched_kind_blocks_per_cu(int prec, int p) {
  if (prec == MF_FP64) return batched_kind_occupancy<MF_FP64>(p);
  if (prec == MF_FP32) return batched_kind_occupancy<MF_FP32>(p);
  if (prec == MF_BF16) return batched_kind_occupancy<MF_BF16>(p);
  return 0;
}

int batched_blocks_per_cu(int prec, int bcfg) {
#define MF_BATCH_CASE(P, C) \
  if (prec == P && bcfg == C) return batched_occupancy<P, C>();
  MF_BATCH_CASE(MF_FP64, 0) MF_BATCH_CASE(MF_FP64, 1) MF_BATCH_CASE(MF_FP64, 2)
  MF_BATCH_CASE(MF_FP32, 0) MF_BATCH_CASE(MF_FP32, 1) MF_BATCH_CASE(MF_FP32, 2)
  MF_BATCH_CASE(MF_BF16, 0) MF_BATCH_CASE(MF_BF16, 1) MF_BATCH_CASE(MF_BF16, 2)
#undef MF_BATCH_CASE
  return 0;
}

hipError_t launch_zero_shared_rows(double* Y, const int64_t nodes[3], int p, int ncols, int64_t ld,
                                   hipStream_t s) {
  const int64_t lines = nodes[1] * nodes[2];
  if (lines < 1 || ncols < 1) return hipSuccess;
  int cw_log2 = 0;
  while (cw_log2 < 6 && (1 << cw_log2) < ncols) ++cw_log2;
  // about 2048 grid elements per workgroup (some 7 KB of face rows), at least
  // one workgroup per CU, at most one per line
  int64_t wgs = nodes[0] * lines * ncols / 2048;
  if (wgs < 256) wgs = 256;
  if (wgs > lines) wgs = lines;
  hipLaunchKernelGGL(zero_shared_rows_kernel, dim3((unsigned)wgs), dim3(256), 0, s, Y,
                     (int)nodes[0], (int)nodes[1], p, ncols, ld, lines, cw_log2);
  return hipGetLastError();
}

hipError_t launch_cheb_init(const Operator& op, const double* Y, const double* Xp, double* Out,
                            int64_t ld, int nvec, double b, double c, hipStream_t s) {
  const int64_t lines = op.nodes[1] * op.nodes[2];
  if (lines < 1) return hipSuccess;
  hipLaunchKernelGGL(cheb_init_kernel, dim3((unsigned)lines), dim3(256), 0, s, Y, Xp, Out,
                     (int)op.nodes[0], (int)op.nodes[1], (int)op.nodes[2], op.p, op.grid.dirichlet,
                     nvec, ld, b, c);
  return hipGetLastError();
}

// The same over an explicit map with a det J per cell (refined meshes).
__global__ void gll_mass_map_kernel(const int32_t* __restrict__ map,
                                    const double* __restrict__ detj, int np, GllWeights wt,
                                    double* __restrict__ m) {
  const int64_t e = blockIdx.x;
  const int F = np * np * np;
  const double dj = detj[e];
  for (int i = threadIdx.x; i < F; i += blockDim.x) {
    const int i1 = i % np, i2 = (i / np) % np, i3 = i / (np * np);
    const int node = map[e * F + i];
    if (node >= 0) unsafeAtomicAdd(m + node, wt.w[i1] * wt.w[i2] * wt.w[i3] * dj);
  }
}

// Row-major elementwise passes over n rows x nvec columns: one row per
// wavefront step, lane = column (no per-element division).
__global__ void scale_rows_kernel(int64_t n, int nvec, const double* __restrict__ D,
                                  const double* __restrict__ Y, int64_t ld,
                                  double* __restrict__ W) {
  const int lane = threadIdx.x % 64;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / 64);
  for (int64_t r = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64; r < n; r += waves) {
    const double d = D[r];
    for (int j = lane; j < nvec; j += 64) W[r * nvec + j] = d * Y[r * ld + j];
  }
}

// Xp may alias Out: each element is read before it is written, by one thread.
__global__ void cheb_combine_kernel(int64_t n, int nvec, const double* __restrict__ D,
                                    const double* __restrict__ V, const double* __restrict__ Y,
                                    const double* Xp, double* Out, int64_t ld, double a, double b,
                                    double c) {
  const int lane = threadIdx.x % 64;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / 64);
  for (int64_t r = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64; r < n; r += waves) {
    const double d = D[r];
    for (int j = lane; j < nvec; j += 64) {
      const int64_t at = r * ld + j;
      double v = 0.0;
      if (d != 0.0) {
        v = a * d * V[r * nvec + j] + b * Y[at];
        if (Xp) v += c * Xp[at];
      }
      Out[at] = v;
    }
  }
}

static unsigned grid_1d(int64_t total) {
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  return (unsigned)(blocks < 1 ? 1 : blocks);
}

hipError_t launch_gll_mass_map(const Operator& op, double* out, hipStream_t s) {
  hipLaunchKernelGGL(zero_rows_kernel, dim3(grid_1d(op.ndofs)), dim3(256), 0, s, out, op.ndofs, 1,
                     (int64_t)1);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  GllWeights wt{};
  for (int i = 0; i < op.np && i <= kMaxP; ++i) wt.w[i] = op.wgll[i];
  hipLaunchKernelGGL(gll_mass_map_kernel, dim3((unsigned)op.ncells), dim3(256), 0, s, op.d_map,
                     op.d_detj, op.np, wt, out);
  return hipGetLastError();
}

hipError_t launch_inv_sqrt(double* m, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(inv_sqrt_kernel, dim3(grid_1d(n)), dim3(256), 0, s, m, n);
  return hipGetLastError();
}

// four rows per 256-thread workgroup step, at most 65536 workgroups
static unsigned grid_rows(int64_t n) {
  int64_t blocks = (n + 3) / 4;
  if (blocks > 65536) blocks = 65536;
  return (unsigned)(blocks < 1 ? 1 : blocks);
}

hipError_t launch_scale_rows(int64_t n, int nvec, const double* D, const double* Y, int64_t ld,
                             double* W, hipStream_t s) {
  hipLaunchKernelGGL(scale_rows_kernel, dim3(grid_rows(n)), dim3(256), 0, s, n, nvec, D, Y, ld, W);
  return hipGetLastError();
}

hipError_t launch_cheb_combine(int64_t n, int nvec, const double* D, const double* V,
                               const double* Y, const double* Xp, double* Out, int64_t ld,
                               double a, double b, double c, hipStream_t s) {
  hipLaunchKernelGGL(cheb_combine_kernel, dim3(grid_rows(n)), dim3(256), 0, s, n, nvec, D, V, Y,
                     Xp, Out, ld, a, b, c);
  return hipGetLastError();
}

hipError_t launch_gll_mass(const Operator& op, int inv_sqrt, double* out, hipStream_t s) {
  const int64_t n = op.ndofs;
  unsigned blocks = (unsigned)((n + 255) / 256 > 65536 ? 65536 : (n + 255) / 256);
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(zero_rows_kernel, dim3(blocks), dim3(256), 0, s, out, n, 1, (int64_t)1);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  GllWeights wt{};
  for (int i = 0; i < op.np && i <= kMaxP; ++i) wt.w[i] = op.wgll[i];
  hipLaunchKernelGGL(gll_mass_kernel, dim3((unsigned)op.ncells), dim3(256), 0, s, op.grid, op.np,
                     wt, op.detj, out);
  err = hipGetLastError();
  if (err != hipSuccess || !inv_sqrt) return err;
  hipLaunchKernelGGL(inv_sqrt_kernel, dim3(blocks), dim3(256), 0, s, out, n);
  return hipGetLastError();
}

hipError_t launch_apply_cheb(const Operator& op, const double* Y, double* Out, int64_t ld,
                             int nvec, const ChebArgs& ca, hipStream_t s) {
  switch (op.p) {
    case 1: return launch_cheb_p<1>(op, Y, Out, ld, nvec, ca, s);
    case 2: return launch_cheb_p<2>(op, Y, Out, ld, nvec, ca, s);
    case 3: return launch_cheb_p<3>(op, Y, Out, ld, nvec, ca, s);
    case 4: return launch_cheb_p<4>(op, Y, Out, ld, nvec, ca, s);
    case 5: return launch_cheb_p<5>(op, Y, Out, ld, nvec, ca, s);
    case 6: return launch_cheb_p<6>(op, Y, Out, ld, nvec, ca, s);
    case 7: return launch_cheb_p<7>(op, Y, Out, ld, nvec, ca, s);
    case 8: return launch_cheb_p<8>(op, Y, Out, ld, nvec, ca, s);
    case 9: return launch_cheb_p<9>(op, Y, Out, ld, nvec, ca, s);
    case 10: return launch_cheb_p<10>(op, Y, Out, ld, nvec, ca, s);
    default: return hipErrorInvalidValue;
  }
}

bool apply_box_supported(int p, int q, int cfg) {
  if (p < 1 || p > kMaxP || q < p + 1 || q > p + kMaxQExtra || cfg < 0 || cfg >= kBoxCfgs)
    return false;
  if (cfg == kBoxMfmaCfg) return q == p + 1 && q <= kMfmaMaxN;
  return box_cfg(p + 1, q, cfg).B > 0;
}

int choose_cfg_box(int np, int nq, int nvec) {
  // the default shape, unless the columns fill a smaller tile better
  const int b0 = box_cfg(np, nq, 0).B;
  if (nvec >= b0) return 0;
  int best = 0, bestB = b0;
  for (int c = 1; c < kBoxCfgs; ++c) {
    if (c == kBoxMfmaCfg) continue;
    const int b = box_cfg(np, nq, c).B;
    if (b >= nvec && b < bestB) {
      best = c;
      bestB = b;
    }
  }
  return best;
}

bool apply_mixed_supported(int p, int q, int cfg) {
  if (p < 1 || p > kMaxP || q < p + 1 || q > p + kMaxQExtra || cfg < 0 || cfg >= kMixedCfgs)
    return false;
  if (cfg >= kMixedMfmaCfgs) return vec32_cfg(p + 1, q, cfg).B > 0;
  return mixed_cfg(p + 1, q, cfg).B > 0;
}

int choose_cfg_mixed(int np, int nq, int nvec, int prec) {
  if (prec == MF_FP32) {
    // FP32: the vector shapes measured fastest (p = 6: 0.42 vs 0.50 ms for the
    // matrix-core shape at nvec 64; p = 8: 0.42 vs 0.61 ms): 16 columns, one per
    // thread, where the workgroup fits, else 8; 8 for narrow multivectors.
    if (nvec > 8 && vec32_cfg(np, nq, 6).B > 0) return 6;
    if (vec32_cfg(np, nq, 5).B > 0) return 5;
  }
  const int b0 = mixed_cfg(np, nq, 0).B;
  if (nvec >= b0) return 0;
  int best = 0, bestB = b0;
  for (int c = 1; c < kMixedMfmaCfgs; ++c) {
    const int b = mixed_cfg(np, nq, c).B;
    if (b >= nvec && b < bestB) {
      best = c;
      bestB = b;
    }
  }
  return best;
}

hipError_t launch_apply_mixed(const Operator& op, const ApplyLaunch& a, int prec, hipStream_t s) {
  switch (op.p) {
    case 1: return launch_apply_mixed_p<1>(op, a, prec, s);
    case 2: return launch_apply_mixed_p<2>(op, a, prec, s);
    case 3: return launch_apply_mixed_p<3>(op, a, prec, s);
    case 4: return launch_apply_mixed_p<4>(op, a, prec, s);
    case 5: return launch_apply_mixed_p<5>(op, a, prec, s);
    case 6: return launch_apply_mixed_p<6>(op, a, prec, s);
    case 7: return launch_apply_mixed_p<7>(op, a, prec, s);
    case 8: return launch_apply_mixed_p<8>(op, a, prec, s);
    case 9: return launch_apply_mixed_p<9>(op, a, prec, s);
    case 10: return launch_apply_mixed_p<10>(op, a, prec, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_apply_box(const Operator& op, const ApplyLaunch& a, hipStream_t s) {
  switch (op.p) {
    case 1: return launch_apply_box_p<1>(op, a, s);
    case 2: return launch_apply_box_p<2>(op, a, s);
    case 3: return launch_apply_box_p<3>(op, a, s);
    case 4: return launch_apply_box_p<4>(op, a, s);
    case 5: return launch_apply_box_p<5>(op, a, s);
    case 6: return launch_apply_box_p<6>(op, a, s);
    case 7: return launch_apply_box_p<7>(op, a, s);
    case 8: return launch_apply_box_p<8>(op, a, s);
    case 9: return launch_apply_box_p<9>(op, a, s);
    case 10: return launch_apply_box_p<10>(op, a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_apply_mfma(const Operator& op, const ApplyLaunch& a, hipStream_t s) {
  switch (op.p) {
    case 1: return launch_apply_mfma_p<1>(op, a, s);
    case 2: return launch_apply_mfma_p<2>(op, a, s);
    case 3: return launch_apply_mfma_p<3>(op, a, s);
    case 4: return launch_apply_mfma_p<4>(op, a, s);
    case 5: return launch_apply_mfma_p<5>(op, a, s);
    case 6: return launch_apply_mfma_p<6>(op, a, s);
    case 7: return launch_apply_mfma_p<7>(op, a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_apply_box_map(const Operator& op, const ApplyLaunch& a, hipStream_t s) {
  switch (op.p) {
    case 1: return launch_apply_box_map_p<1>(op, a, s);
    case 2: return launch_apply_box_map_p<2>(op, a, s);
    case 3: return launch_apply_box_map_p<3>(op, a, s);
    case 4: return launch_apply_box_map_p<4>(op, a, s);
    case 5: return launch_apply_box_map_p<5>(op, a, s);
    case 6: return launch_apply_box_map_p<6>(op, a, s);
    case 7: return launch_apply_box_map_p<7>(op, a, s);
    case 8: return launch_apply_box_map_p<8>(op, a, s);
    case 9: return launch_apply_box_map_p<9>(op, a, s);
    case 10: return launch_apply_box_map_p<10>(op, a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_apply_box_map32(const Operator& op, const ApplyLaunch& a, hipStream_t s) {
  switch (op.p) {
    case 1: return launch_apply_box_map32_p<1>(op, a, s);
    case 2: return launch_apply_box_map32_p<2>(op, a, s);
    case 3: return launch_apply_box_map32_p<3>(op, a, s);
    case 4: return launch_apply_box_map32_p<4>(op, a, s);
    case 5: return launch_apply_box_map32_p<5>(op, a, s);
    case 6: return launch_apply_box_map32_p<6>(op, a, s);
    case 7: return launch_apply_box_map32_p<7>(op, a, s);
    case 8: return launch_apply_box_map32_p<8>(op, a, s);
    case 9: return launch_apply_box_map32_p<9>(op, a, s);
    case 10: return launch_apply_box_map32_p<10>(op, a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_zero_rows(double* Y, int64_t nrows, int ncols, int64_t ld, hipStream_t s) {
  const int64_t total = nrows * ncols;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(zero_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, s, Y, nrows, ncols, ld);
  return hipGetLastError();
}

hipError_t launch_fma_probe(int blocks, int64_t iters, double* out, hipStream_t s) {
  hipLaunchKernelGGL(fma_probe_kernel, dim3((unsigned)blocks), dim3(256), 0, s, iters, 1.0, out);
  return hipGetLastError();
}

hipError_t launch_fill_pattern(double* X, int64_t n, hipStream_t s) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(fill_pattern_kernel, dim3((unsigned)blocks), dim3(256), 0, s, X, n);
  return hipGetLastError();
}

bool apply_f64_supported(int p, int q) {
  if (p < 1 || p > kMaxP || q < p + 1 || q > p + kMaxQExtra) return false;
  return f64_bmax(p + 1, q) >= 1;
}

int choose_vtile_f64(int np, int nq, int nvec) {
  // the default tile, or for fewer columns the smallest built tile covering them
  const int bd = f64_bdef(np, nq);
  if (nvec >= bd) return bd;
  for (int b = 1; b <= bd; ++b)
    if (b >= nvec && f64_tile_built(np, nq, b)) return b;
  return bd;
}

hipError_t launch_apply_f64(const Operator& op, const ApplyLaunch& a, hipStream_t s) {
  switch (op.p) {
    case 1: return launch_apply_f64_p<1>(op, a, s);
    case 2: return launch_apply_f64_p<2>(op, a, s);
    case 3: return launch_apply_f64_p<3>(op, a, s);
    case 4: return launch_apply_f64_p<4>(op, a, s);
    case 5: return launch_apply_f64_p<5>(op, a, s);
    case 6: return launch_apply_f64_p<6>(op, a, s);
    case 7: return launch_apply_f64_p<7>(op, a, s);
    case 8: return launch_apply_f64_p<8>(op, a, s);
    case 9: return launch_apply_f64_p<9>(op, a, s);
    case 10: return launch_apply_f64_p<10>(op, a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mf
