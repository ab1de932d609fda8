// FP64 fused apply for axis-aligned (box) cells: one launch over (cell, column
// tile) work items.  The per-item body is box_cell_tile (box_body.h).
//
// Work item = (cell, tile of B columns); cells are taken in the order given by
// `order` (XCD-blocked, Morton inside a block) so that cells sharing nodes run
// close in time on the same XCD.
#include "box_body.h"

#ifndef MF_P
#error "compile with -DMF_P=<degree>"
#endif

namespace mf {
namespace {

template <int NP, int NQ, int B, int C, int NT, bool ACCUM>
__global__ void __attribute__((amdgpu_flat_work_group_size(1, NT),
                               amdgpu_waves_per_eu(box_waves_per_eu(NP, NQ, B, NT))))
apply_box_kernel(const GridDesc grid, const int32_t* __restrict__ order,
                 const double* __restrict__ geo, const double* __restrict__ vq,
                 const double* __restrict__ X, double* __restrict__ Y, int64_t ldx, int64_t ldy,
                 int nvec, int ntiles, int64_t nitems, int64_t chunk) {
  extern __shared__ double lds[];
  const int64_t item = xcd_item(blockIdx.x, chunk);
  if (item >= nitems) return;
  const int64_t e = order[item / ntiles];
  const int v0 = (int)(item % ntiles) * B;
  box_cell_tile<NP, NQ, B, C, NT, ACCUM>(lds, grid, geo, vq, X, Y, ldx, ldy, nvec, e, v0);
}

// Persistent grid: the workgroups of each XCD take that XCD's contiguous item
// range in an interleaved order (box_items), so cells sharing nodes still run
// close in time on one XCD.
template <int NP, int NQ, int B, int C, int NT, bool ACCUM>
__global__ void __attribute__((amdgpu_flat_work_group_size(1, NT),
                               amdgpu_waves_per_eu(box_waves_per_eu(NP, NQ, B, NT))))
apply_box_pers_kernel(const GridDesc grid, const int32_t* __restrict__ order,
                      const double* __restrict__ geo, const double* __restrict__ vq,
                      const double* __restrict__ X, double* __restrict__ Y, int64_t ldx,
                      int64_t ldy, int nvec, int ntiles, int64_t nitems, int64_t chunk) {
  extern __shared__ double lds[];
  const int64_t W = gridDim.x / kXcds;  // workgroups per XCD
  const int64_t xcd = blockIdx.x % kXcds, j = blockIdx.x / kXcds;
  const int64_t begin = xcd * chunk;
  const int64_t end = begin + chunk < nitems ? begin + chunk : nitems;
  box_items<NP, NQ, B, C, NT, ACCUM>(lds, grid, order, geo, vq, X, Y, ldx, ldy, nvec, ntiles,
                                      begin + j, end, W);
}

template <int NP, int NQ, int B, int C, int NT, bool ACCUM, bool PERS>
hipError_t launch_box(const ApplyLaunch& a, hipStream_t s) {
  const int ntiles = (a.nvec + B - 1) / B;
  const int64_t nitems = a.ncells * ntiles;
  const int64_t chunk = (nitems + kXcds - 1) / kXcds;
  constexpr size_t lds = box_lds_bytes(NP, NQ, B);
  static_assert(lds <= kLdsMax, "LDS");
  using Kern = void (*)(const GridDesc, const int32_t*, const double*, const double*,
                       const double*, double*, int64_t, int64_t, int, int, int64_t, int64_t);
  Kern k;
  if constexpr (PERS) k = apply_box_pers_kernel<NP, NQ, B, C, NT, ACCUM>;
  else k = apply_box_kernel<NP, NQ, B, C, NT, ACCUM>;
  KernelFacts f;
  hipError_t err = kernel_facts(reinterpret_cast<const void*>(k), NT, lds, f);
  if (err != hipSuccess) return err;
  int64_t blocks = chunk * kXcds;
  if (PERS) {
    int64_t resident = (int64_t)f.per_cu * f.cus;
    resident -= resident % kXcds;
    if (resident < kXcds) resident = kXcds;
    if (resident < blocks) blocks = resident;
  }
  hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(NT), lds, s, a.grid, a.order, a.geo, a.vq,
                     a.X, a.Y, a.ldx, a.ldy, a.nvec, ntiles, nitems, chunk);
  return hipGetLastError();
}

template <int NP, int NQ, int CFG>
hipError_t try_cfg(const ApplyLaunch& a, hipStream_t s, bool& done) {
  constexpr BoxCfg c = box_cfg(NP, NQ, CFG);
  if constexpr (c.B > 0) {
    if (a.cfg == CFG) {
      done = true;
      return a.accumulate ? launch_box<NP, NQ, c.B, c.C, c.NT, true, c.pers>(a, s)
                          : launch_box<NP, NQ, c.B, c.C, c.NT, false, c.pers>(a, s);
    }
  }
  return hipSuccess;
}

template <int NP, int NQ>
hipError_t launch_pq(const ApplyLaunch& a, hipStream_t s) {
  bool done = false;
  hipError_t err = hipSuccess;
  if (!done) err = try_cfg<NP, NQ, 0>(a, s, done);
  if (!done) err = try_cfg<NP, NQ, 1>(a, s, done);
  if (!done) err = try_cfg<NP, NQ, 2>(a, s, done);
  if (!done) err = try_cfg<NP, NQ, 3>(a, s, done);
  if (!done) err = try_cfg<NP, NQ, 4>(a, s, done);
  if (!done) err = try_cfg<NP, NQ, 5>(a, s, done);
  if (!done) err = try_cfg<NP, NQ, 6>(a, s, done);
  if (!done) err = try_cfg<NP, NQ, 7>(a, s, done);
  if (!done) err = try_cfg<NP, NQ, 8>(a, s, done);
  if (!done) err = try_cfg<NP, NQ, 9>(a, s, done);
  if (!done) err = try_cfg<NP, NQ, 11>(a, s, done);
  if (!done) err = try_cfg<NP, NQ, 12>(a, s, done);
  return done ? err : hipErrorInvalidValue;
}

}  // namespace

template <>
hipError_t launch_apply_box_p<MF_P>(const Operator& op, const ApplyLaunch& a, hipStream_t s) {
  switch (op.q - MF_P) {
    case 1: return launch_pq<MF_P + 1, MF_P + 1>(a, s);
    case 2: return launch_pq<MF_P + 1, MF_P + 2>(a, s);
    case 3: return launch_pq<MF_P + 1, MF_P + 3>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mf
