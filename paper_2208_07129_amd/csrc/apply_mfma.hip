// FP64 fused apply on the matrix cores for axis-aligned (box) cells with
// q = p + 1 <= 8 points per direction: one launch over (cell, column tile)
// work items, the per-item body mfma_cell_tile (mfma_body.h).  Work items are
// taken in the cell order `order` (XCD-blocked, Morton inside a block), item
// i on XCD i mod 8 as in the vector kernel.
#include "mfma_body.h"

#ifndef MF_P
#error "compile with -DMF_P=<degree>"
#endif

namespace mf {
namespace {

// Three workgroups fit a CU's LDS at N = 7, so the register budget is that of
// three wavefronts per SIMD.
template <int N, bool ACCUM>
__global__ void __attribute__((amdgpu_flat_work_group_size(1, MfmaShape<N>::NT),
                               amdgpu_waves_per_eu(mfma_waves_per_eu<N>())))
apply_mfma_kernel(const GridDesc grid, const int32_t* __restrict__ order,
                  const double* __restrict__ geo, const double* __restrict__ vq,
                  const double* __restrict__ X, double* __restrict__ Y, int64_t ldx, int64_t ldy,
                  int nvec, int ntiles, int nitems, int chunk) {
  extern __shared__ double lds[];
  const int wg = blockIdx.x;
  const int item = (wg % kXcds) * chunk + wg / kXcds;
  if (item >= nitems) return;
  const int e = order[item / ntiles];
  const int v0 = (item % ntiles) * 8;
  mfma_cell_tile<N, ACCUM>(lds, grid, geo, vq, X, Y, ldx, ldy, nvec, e, v0);
}

template <int N, bool ACCUM>
hipError_t launch_mfma(const ApplyLaunch& a, hipStream_t s) {
  using S = MfmaShape<N>;
  constexpr size_t lds = mfma_lds_bytes<N>();
  static_assert(lds <= kLdsMax, "LDS");
  const int ntiles = (a.nvec + 7) / 8;
  const int64_t nitems = a.ncells * ntiles;
  if (nitems >= ((int64_t)1 << 31) - 8) return hipErrorInvalidValue;
  const int chunk = (int)((nitems + kXcds - 1) / kXcds);
  auto k = apply_mfma_kernel<N, ACCUM>;
  KernelFacts f;  // raises the dynamic LDS limit on this device if needed
  hipError_t err = kernel_facts(reinterpret_cast<const void*>(k), S::NT, lds, f);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k, dim3((unsigned)chunk * kXcds), dim3(S::NT), lds, s, a.grid, a.order, a.geo,
                     a.vq, a.X, a.Y, a.ldx, a.ldy, a.nvec, ntiles, (int)nitems, chunk);
  return hipGetLastError();
}

}  // namespace

template <>
hipError_t launch_apply_mfma_p<MF_P>(const Operator& op, const ApplyLaunch& a, hipStream_t s) {
  constexpr int N = MF_P + 1;
  if constexpr (N <= kMfmaMaxN) {
    if (op.q != N) return hipErrorInvalidValue;
    if (a.cfg == kBoxMfmaCfg)
      return a.accumulate ? launch_mfma<N, true>(a, s) : launch_mfma<N, false>(a, s);
  }
  (void)op;
  (void)a;
  (void)s;
  return hipErrorInvalidValue;
}

}  // namespace mf
