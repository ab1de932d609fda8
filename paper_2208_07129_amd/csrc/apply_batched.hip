// Batched apply: Y_i := A_i X_i for a list of operators of different meshes,
// degrees and column counts, in ONE persistent launch (the generalisation of
// the single launch over every (cell, batch) pair of eq. basempigpu).
//
// The work list is the concatenation, operator by operator (heaviest degree
// first), of each operator's (cell, column tile) items in its XCD-blocked
// Morton cell order.  The host cuts the list into one contiguous range per XCD
// of equal estimated cost; the resident workgroups of an XCD take that range
// in an interleaved order (static: no shared counter, whose device-scope
// atomics from every XCD serialise), so cells sharing nodes run close in time
// on one XCD's L2.  A byte table gives each item's operator in one uniform
// load.  Each item runs the fused body of its (p, q) kind (box_cell_tile or
// mixed_cell_tile, selected by a switch that is uniform over the workgroup);
// every workgroup leaves when its range is exhausted.
//
// Compiled once per (precision, launch shape); kinds are q = p + 1 for
// p = 2 .. 8.
#include "box_body.h"
#include "mixed_body.h"

#ifndef MF_BPREC
#error "compile with -DMF_BPREC=<precision> -DMF_BCFG=<shape>"
#endif

namespace mf {
namespace {

template <int BCFG, int PREC>
struct Shape {
  static constexpr int NT = batch_threads(BCFG);
};

template <int NP, int BCFG, int PREC>
__device__ __forceinline__ void run_kind(double* lds, const BatchOp& op, const BatchPtrs& ptrs,
                                         int o, int64_t local) {
  constexpr int NQ = NP;  // q = p + 1
  constexpr int B = batch_tile(PREC, BCFG, NP, NQ);
  constexpr int NT = Shape<BCFG, PREC>::NT;
  const int64_t e = op.order[local / op.ntiles];
  const int v0 = (int)(local % op.ntiles) * B;
  if constexpr (PREC == MF_FP64)
    box_cell_tile<NP, NQ, B, 1, NT, false>(lds, op.grid, op.geo, op.vq, ptrs.X[o], ptrs.Y[o],
                                         ptrs.ldx[o], ptrs.ldy[o], ptrs.nvec[o], e, v0);
  else
    mixed_cell_tile<NP, NQ, B, NT, false, PREC>(lds, op.map, op.geo, op.vq, ptrs.X[o], ptrs.Y[o],
                                                ptrs.ldx[o], ptrs.ldy[o], ptrs.nvec[o], e, v0);
}

// Waves per SIMD the register allocation leaves room for: the workgroups per
// CU that the LDS allows (the largest kind's tile sets the LDS size).  The
// mixed body needs more registers than that occupancy leaves (its single-
// operator kernel runs at 2-3 waves per SIMD), so it gets no budget.
template <int BCFG, int PREC>
constexpr int batch_waves_per_eu() {
  if (PREC != MF_FP64) return 1;
  const size_t l = batch_lds_bytes(PREC, BCFG);
  int wg = (int)(kLdsMax / (l > 0 ? l : 1));
  if (wg < 1) wg = 1;
  int w = (wg * (batch_threads(BCFG) / 64) + 3) / 4;
  return w < 1 ? 1 : (w > 8 ? 8 : w);
}

template <int BCFG, int PREC>
__global__ void __attribute__((amdgpu_flat_work_group_size(1, batch_threads(BCFG)),
                               amdgpu_waves_per_eu(batch_waves_per_eu<BCFG, PREC>())))
batched_kernel(const BatchOp* __restrict__ ops, const uint8_t* __restrict__ item_op,
               const int64_t* __restrict__ bounds, BatchPtrs ptrs) {
  extern __shared__ double lds[];
  const int64_t W = gridDim.x / kXcds;  // workgroups per XCD
  const int x = blockIdx.x % kXcds;
  const int64_t end = bounds[x + 1];
  for (int64_t item = bounds[x] + blockIdx.x / kXcds; item < end; item += W) {
    const int o = item_op[item];
    const BatchOp& op = ops[o];
    const int64_t local = item - op.item_begin;
    switch (op.p) {
      case 2: run_kind<3, BCFG, PREC>(lds, op, ptrs, o, local); break;
      case 3: run_kind<4, BCFG, PREC>(lds, op, ptrs, o, local); break;
      case 4: run_kind<5, BCFG, PREC>(lds, op, ptrs, o, local); break;
      case 5: run_kind<6, BCFG, PREC>(lds, op, ptrs, o, local); break;
      case 6: run_kind<7, BCFG, PREC>(lds, op, ptrs, o, local); break;
      case 7: run_kind<8, BCFG, PREC>(lds, op, ptrs, o, local); break;
      case 8: run_kind<9, BCFG, PREC>(lds, op, ptrs, o, local); break;
      default: break;
    }
    __syncthreads();  // every thread is done with this item's LDS
  }
}

#if MF_BCFG == 0
// One kind per launch (shapes 3 and 4): the kind's own tile and workgroup
// size, the register budget of the occupancy its LDS allows; same static
// per-XCD ranges (bounds of this kind's items only).  Shape 3 launches the
// resident grid, shape 4 eight times the longest range (one item each).
template <int NP, int PREC>
struct KindShape {
  static constexpr BoxCfg c = batch_kind_shape(PREC, NP, NP);
  static constexpr int B = c.B, NT = c.NT;
  // FP64 and FP32 run the box body (double / float cell arrays), BF16 the
  // matrix-core body
  static constexpr bool BOX = PREC != MF_BF16;
  static constexpr size_t LDS = PREC == MF_FP64        ? box_lds_bytes(NP, NP, B)
                                : PREC == MF_FP32 ? box_lds_bytes_t<float>(NP, NP, B)
                                                       : mixed_lds_bytes(NP, NP, B);
  static constexpr int WG = (int)(kLdsMax / LDS) < 1 ? 1 : (int)(kLdsMax / LDS);
  static constexpr int W0 = (WG * (NT / 64) + 3) / 4;
  // box bodies: the LDS-limited occupancy; matrix-core body: no budget (see
  // batch_waves_per_eu)
  static constexpr int WAVES = !BOX ? 1 : (W0 < 1 ? 1 : (W0 > 8 ? 8 : W0));
};

template <int NP, int PREC>
__device__ __forceinline__ void kind_item(double* lds, const BatchOp& op, const BatchPtrs& ptrs,
                                          int o, int64_t local) {
  constexpr int B = KindShape<NP, PREC>::B, NT = KindShape<NP, PREC>::NT;
  const int64_t e = op.order[local / op.ntiles];
  const int v0 = (int)(local % op.ntiles) * B;
  if constexpr (PREC == MF_FP64)
    box_cell_tile<NP, NP, B, 1, NT, false>(lds, op.grid, op.geo, op.vq, ptrs.X[o], ptrs.Y[o],
                                           ptrs.ldx[o], ptrs.ldy[o], ptrs.nvec[o], e, v0);
  else if constexpr (PREC == MF_FP32)
    box_cell_tile<NP, NP, B, 1, NT, false, float>(reinterpret_cast<float*>(lds), op.grid, op.geo,
                                                  op.vq, ptrs.X[o], ptrs.Y[o], ptrs.ldx[o],
                                                  ptrs.ldy[o], ptrs.nvec[o], e, v0);
  else
    mixed_cell_tile<NP, NP, B, NT, false, PREC>(lds, op.map, op.geo, op.vq, ptrs.X[o], ptrs.Y[o],
                                                ptrs.ldx[o], ptrs.ldy[o], ptrs.nvec[o], e, v0);
}

// LOOP: resident grid, each workgroup takes items j, j + W, ... of its XCD's
// range; otherwise one item per workgroup (no loop, so nothing that is
// invariant across items is kept live in registers).
template <int NP, int PREC, bool LOOP>
__global__ void __attribute__((amdgpu_flat_work_group_size(1, KindShape<NP, PREC>::NT),
                               amdgpu_waves_per_eu(KindShape<NP, PREC>::WAVES)))
batched_kind_kernel(const BatchOp* __restrict__ ops, const uint8_t* __restrict__ item_op,
                    const int64_t* __restrict__ bounds, BatchPtrs ptrs) {
  extern __shared__ double lds[];
  const int x = blockIdx.x % kXcds;
  const int64_t end = bounds[x + 1];
  int64_t item = bounds[x] + blockIdx.x / kXcds;
  if constexpr (LOOP) {
    const int64_t W = gridDim.x / kXcds;
    for (; item < end; item += W) {
      const int o = item_op[item];
      kind_item<NP, PREC>(lds, ops[o], ptrs, o, item - ops[o].item_begin);
      __syncthreads();
    }
  } else {
    if (item >= end) return;
    const int o = item_op[item];
    kind_item<NP, PREC>(lds, ops[o], ptrs, o, item - ops[o].item_begin);
  }
}

template <int NP, int PREC>
void* kind_kernel_ptr(bool loop, size_t& lds, int& nt) {
  lds = KindShape<NP, PREC>::LDS;
  nt = KindShape<NP, PREC>::NT;
  return loop ? reinterpret_cast<void*>(batched_kind_kernel<NP, PREC, true>)
              : reinterpret_cast<void*>(batched_kind_kernel<NP, PREC, false>);
}

template <int PREC>
void* kind_kernel(int p, bool loop, size_t& lds, int& nt) {
  switch (p) {
    case 2: return kind_kernel_ptr<3, PREC>(loop, lds, nt);
    case 3: return kind_kernel_ptr<4, PREC>(loop, lds, nt);
    case 4: return kind_kernel_ptr<5, PREC>(loop, lds, nt);
    case 5: return kind_kernel_ptr<6, PREC>(loop, lds, nt);
    case 6: return kind_kernel_ptr<7, PREC>(loop, lds, nt);
    case 7: return kind_kernel_ptr<8, PREC>(loop, lds, nt);
    case 8: return kind_kernel_ptr<9, PREC>(loop, lds, nt);
    default: return nullptr;
  }
}
#endif

}  // namespace

#if MF_BCFG == 0
template <>
hipError_t launch_batched_kind<MF_BPREC>(int p, bool loop, const BatchOp* ops,
                                         const uint8_t* item_op, const int64_t* bounds,
                                         const BatchPtrs& ptrs, int grid, hipStream_t s) {
  size_t lds = 0;
  int nt = 0;
  void* k = kind_kernel<MF_BPREC>(p, loop, lds, nt);
  if (!k) return hipErrorInvalidValue;
  if (lds > 64 * 1024) {
    hipError_t err = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
  }
  void* args[] = {(void*)&ops, (void*)&item_op, (void*)&bounds, (void*)&ptrs};
  return hipLaunchKernel(k, dim3(grid), dim3(nt), args, lds, s);
}

template <>
int batched_kind_occupancy<MF_BPREC>(int p) {
  size_t lds = 0;
  int nt = 0;
  void* k = kind_kernel<MF_BPREC>(p, true, lds, nt);
  if (!k) return 0;
  if (lds > 64 * 1024)
    (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, nt, lds) != hipSuccess) return 0;
  return n;
}
#endif

template <>
hipError_t launch_batched_kernel<MF_BPREC, MF_BCFG>(const BatchOp* ops, const uint8_t* item_op,
                                                    const int64_t* bounds, const BatchPtrs& ptrs,
                                                    int grid, hipStream_t s) {
  constexpr size_t lds = batch_lds_bytes(MF_BPREC, MF_BCFG);
  auto k = batched_kernel<MF_BCFG, MF_BPREC>;
  if (lds > 64 * 1024) {
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
  }
  hipLaunchKernelGGL(k, dim3(grid), dim3(Shape<MF_BCFG, MF_BPREC>::NT), lds, s, ops, item_op,
                     bounds, ptrs);
  return hipGetLastError();
}

template <>
int batched_occupancy<MF_BPREC, MF_BCFG>() {
  constexpr size_t lds = batch_lds_bytes(MF_BPREC, MF_BCFG);
  auto k = batched_kernel<MF_BCFG, MF_BPREC>;
  if (lds > 64 * 1024)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, Shape<MF_BCFG, MF_BPREC>::NT, lds) !=
      hipSuccess)
    return 0;
  return n;
}

}  // namespace mf
