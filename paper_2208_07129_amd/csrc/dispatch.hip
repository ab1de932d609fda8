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

// One workgroup per node line (gy, gz) of the Nx x Ny x Nz grid.  A line on a
// cell-face plane (gy or gz a multiple of p) is zeroed whole; otherwise only the
// rows gx = 0, p, 2p, ... are.  Each wavefront takes rows, lanes take columns,
// so stores are contiguous and no per-element index arithmetic is needed.
// Rows of cell-interior nodes are skipped: the box kernel writes them.
__global__ void zero_shared_rows_kernel(double* __restrict__ Y, int Nx, int Ny, int p, int ncols,
                                        int64_t ld) {
  const int line = blockIdx.x;
  const int gy = line % Ny, gz = line / Ny;
  const bool full = (gy % p == 0) || (gz % p == 0);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  double* base = Y + (int64_t)line * Nx * ld;
  const int step = full ? 1 : p;
  for (int gx = wave * step; gx < Nx; gx += nw * step) {
    double* row = base + (int64_t)gx * ld;
    for (int c = lane; c < ncols; c += 64) row[c] = 0.0;
  }
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
  MF_BATCH_CASE(MF_FP32_MFMA, 0) MF_BATCH_CASE(MF_FP32_MFMA, 1) MF_BATCH_CASE(MF_FP32_MFMA, 2)
  MF_BATCH_CASE(MF_BF16_MFMA, 0) MF_BATCH_CASE(MF_BF16_MFMA, 1) MF_BATCH_CASE(MF_BF16_MFMA, 2)
#undef MF_BATCH_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_batched_kind_any(int prec, int p, bool loop, const BatchOp* ops,
                                   const uint8_t* item_op,
                                   const int64_t* bounds, const BatchPtrs& ptrs, int grid,
                                   hipStream_t s) {
  if (prec == MF_FP64)
    return launch_batched_kind<MF_FP64>(p, loop, ops, item_op, bounds, ptrs, grid, s);
  if (prec == MF_FP32_MFMA)
    return launch_batched_kind<MF_FP32_MFMA>(p, loop, ops, item_op, bounds, ptrs, grid, s);
  if (prec == MF_BF16_MFMA)
    return launch_batched_kind<MF_BF16_MFMA>(p, loop, ops, item_op, bounds, ptrs, grid, s);
  return hipErrorInvalidValue;
}

int batched_kind_blocks_per_cu(int prec, int p) {
  if (prec == MF_FP64) return batched_kind_occupancy<MF_FP64>(p);
  if (prec == MF_FP32_MFMA) return batched_kind_occupancy<MF_FP32_MFMA>(p);
  if (prec == MF_BF16_MFMA) return batched_kind_occupancy<MF_BF16_MFMA>(p);
  return 0;
}

int batched_blocks_per_cu(int prec, int bcfg) {
#define MF_BATCH_CASE(P, C) \
  if (prec == P && bcfg == C) return batched_occupancy<P, C>();
  MF_BATCH_CASE(MF_FP64, 0) MF_BATCH_CASE(MF_FP64, 1) MF_BATCH_CASE(MF_FP64, 2)
  MF_BATCH_CASE(MF_FP32_MFMA, 0) MF_BATCH_CASE(MF_FP32_MFMA, 1) MF_BATCH_CASE(MF_FP32_MFMA, 2)
  MF_BATCH_CASE(MF_BF16_MFMA, 0) MF_BATCH_CASE(MF_BF16_MFMA, 1) MF_BATCH_CASE(MF_BF16_MFMA, 2)
#undef MF_BATCH_CASE
  return 0;
}

hipError_t launch_zero_shared_rows(double* Y, const int64_t nodes[3], int p, int ncols, int64_t ld,
                                   hipStream_t s) {
  const int64_t lines = nodes[1] * nodes[2];
  if (lines < 1) return hipSuccess;
  hipLaunchKernelGGL(zero_shared_rows_kernel, dim3((unsigned)lines), dim3(256), 0, s, Y,
                     (int)nodes[0], (int)nodes[1], p, ncols, ld);
  return hipGetLastError();
}

bool apply_box_supported(int p, int q, int cfg) {
  if (p < 1 || p > kMaxP || q < p + 1 || q > p + kMaxQExtra || cfg < 0 || cfg >= kBoxCfgs)
    return false;
  return box_cfg(p + 1, q, cfg).B > 0;
}

int choose_cfg_box(int np, int nq, int nvec) {
  // the default shape, unless the columns fill a smaller tile better
  const int b0 = box_cfg(np, nq, 0).B;
  if (nvec >= b0) return 0;
  int best = 0, bestB = b0;
  for (int c = 1; c < kBoxCfgs; ++c) {
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
  if (prec == MF_FP32_MFMA) {
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

hipError_t launch_zero_rows(double* Y, int64_t nrows, int ncols, int64_t ld, hipStream_t s) {
  const int64_t total = nrows * ncols;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(zero_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, s, Y, nrows, ncols, ld);
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
