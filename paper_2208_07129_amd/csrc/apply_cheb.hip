// Fused Chebyshev filter step for axis-aligned cells (box_cell_tile_cheb):
// one launch over (cell, 8-column tile) work items, the box kernel's default
// one-shot shape (4-column tiles where two 8-column buffers exceed the LDS).
#include "box_body.h"

#ifndef MF_P
#error "compile with -DMF_P=<degree>"
#endif

namespace mf {
namespace {

template <int NP, int NQ, int B, int NT>
__global__ void __attribute__((amdgpu_flat_work_group_size(1, NT),
                               amdgpu_waves_per_eu(box_waves_per_eu(NP, NQ, B, NT))))
apply_cheb_kernel(const GridDesc grid, const int32_t* __restrict__ order,
                  const double* __restrict__ geo, const double* __restrict__ vq,
                  const double* __restrict__ Y, double* Out, int64_t ld, int nvec, int ntiles,
                  int64_t nitems, int64_t chunk, ChebArgs ca) {
  extern __shared__ double lds[];
  const int64_t item = xcd_item(blockIdx.x, chunk);
  if (item >= nitems) return;
  const int64_t e = order[item / ntiles];
  const int v0 = (int)(item % ntiles) * B;
  box_cell_tile_cheb<NP, NQ, B, NT>(lds, grid, geo, vq, Y, Out, ld, nvec, e, v0, ca);
}

template <int NP, int NQ>
hipError_t launch_cheb_pq(const Operator& op, const double* Y, double* Out, int64_t ld, int nvec,
                          const ChebArgs& ca, hipStream_t s) {
  constexpr int B = box_lds_bytes(NP, NQ, 8) <= kLdsMax ? 8 : 4;
  constexpr int NT = (NQ * NQ * B + 63) / 64 * 64 > 1024 ? 1024 : (NQ * NQ * B + 63) / 64 * 64;
  constexpr size_t lds = box_lds_bytes(NP, NQ, B);
  static_assert(lds <= kLdsMax, "LDS");
  const int ntiles = (nvec + B - 1) / B;
  const int64_t nitems = op.ncells * ntiles;
  const int64_t chunk = (nitems + kXcds - 1) / kXcds;
  auto k = apply_cheb_kernel<NP, NQ, B, NT>;
  if (lds > 64 * 1024) {
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
  }
  hipLaunchKernelGGL(k, dim3((unsigned)(chunk * kXcds)), dim3(NT), lds, s, op.grid, op.d_order,
                     op.d_geo, op.d_vq, Y, Out, ld, nvec, ntiles, nitems, chunk, ca);
  return hipGetLastError();
}

}  // namespace

template <>
hipError_t launch_cheb_p<MF_P>(const Operator& op, const double* Y, double* Out, int64_t ld,
                               int nvec, const ChebArgs& ca, hipStream_t s) {
  switch (op.q - MF_P) {
    case 1: return launch_cheb_pq<MF_P + 1, MF_P + 1>(op, Y, Out, ld, nvec, ca, s);
    case 2: return launch_cheb_pq<MF_P + 1, MF_P + 2>(op, Y, Out, ld, nvec, ca, s);
    case 3: return launch_cheb_pq<MF_P + 1, MF_P + 3>(op, Y, Out, ld, nvec, ca, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mf
