// Batched apply: Y_i := A_i X_i for a list of operators of different meshes,
// degrees and column counts, in ONE persistent launch (the generalisation of
// the single launch over every (cell, batch) pair of eq. basempigpu).
//
// The work list is the concatenation, operator by operator (heaviest degree
// first), of each operator's (cell, column tile) items in its XCD-blocked
// Morton cell order.  A grid sized to the resident capacity of the device
// pulls items from one global counter; each item runs the fused body of its
// (p, q) kind (box_cell_tile or mixed_cell_tile, selected by a switch that is
// uniform over the workgroup).  Every workgroup leaves the loop once the
// counter passes the item count, so the grid always drains.
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

template <int BCFG, int PREC>
__global__ void __launch_bounds__(batch_threads(BCFG))
batched_kernel(const BatchOp* __restrict__ ops, int nops, int64_t total, int* __restrict__ counter,
               BatchPtrs ptrs) {
  extern __shared__ double lds[];
  __shared__ int s_item, s_op;
  for (;;) {
    if (threadIdx.x == 0) {
      const int it = atomicAdd(counter, 1);
      int o = 0;
      while (o + 1 < nops && ops[o + 1].item_begin <= it) ++o;
      s_item = it;
      s_op = o;
    }
    __syncthreads();  // also: every thread has finished the previous item's LDS use
    const int item = s_item, o = s_op;
    __syncthreads();  // s_item / s_op read before thread 0 overwrites them
    if (item >= total) break;
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
  }
}

}  // namespace

template <>
hipError_t launch_batched_kernel<MF_BPREC, MF_BCFG>(const BatchOp* ops, int nops, int64_t total,
                                                    int* counter, const BatchPtrs& ptrs, int grid,
                                                    hipStream_t s) {
  constexpr size_t lds = batch_lds_bytes(MF_BPREC, MF_BCFG);
  auto k = batched_kernel<MF_BCFG, MF_BPREC>;
  if (lds > 64 * 1024) {
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
  }
  hipLaunchKernelGGL(k, dim3(grid), dim3(Shape<MF_BCFG, MF_BPREC>::NT), lds, s, ops, nops, total,
                     counter, ptrs);
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
