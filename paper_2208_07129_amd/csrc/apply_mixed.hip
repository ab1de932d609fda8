// Mixed-precision fused apply for axis-aligned cells: one launch over (cell,
// column tile) work items.  Shapes 0 .. 3: the per-item body is mixed_cell_tile
// (mixed_body.h): FP32 / BF16 matrix-core contractions, FP64 assembly.
// Shapes 4 .. 6 (FP32 only): box_cell_tile on float cell arrays, the even-odd
// vector contractions of the FP64 box kernel at half the LDS per column.
#include "box_body.h"
#include "mixed_body.h"

#ifndef MF_P
#error "compile with -DMF_P=<degree>"
#endif

namespace mf {
namespace {

template <int NP, int NQ, int B, int NT, bool ACCUM, int PREC>
__global__ void __launch_bounds__(NT)
apply_mixed_kernel(const int32_t* __restrict__ cmap, const int32_t* __restrict__ order,
                   const double* __restrict__ geo, const double* __restrict__ vq,
                   const double* __restrict__ X, double* __restrict__ Y, int64_t ldx,
                   int64_t ldy, int nvec, int ntiles, int64_t nitems, int64_t chunk) {
  extern __shared__ double lds_d[];
  const int64_t item = xcd_item(blockIdx.x, chunk);
  if (item >= nitems) return;
  const int64_t e = order[item / ntiles];
  const int v0 = (int)(item % ntiles) * B;
  mixed_cell_tile<NP, NQ, B, NT, ACCUM, PREC>(lds_d, cmap, geo, vq, X, Y, ldx, ldy, nvec, e, v0);
}

template <int NP, int NQ, int B, int NT, bool ACCUM, int PREC>
hipError_t launch_mixed(const ApplyLaunch& a, hipStream_t s) {
  const int ntiles = (a.nvec + B - 1) / B;
  const int64_t nitems = a.ncells * ntiles;
  const int64_t chunk = (nitems + kXcds - 1) / kXcds;
  constexpr size_t lds = mixed_lds_bytes(NP, NQ, B);
  static_assert(lds <= kLdsMax, "LDS");
  auto k = apply_mixed_kernel<NP, NQ, B, NT, ACCUM, PREC>;
  if (lds > 64 * 1024) {
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
  }
  hipLaunchKernelGGL(k, dim3((unsigned)(chunk * kXcds)), dim3(NT), lds, s, a.map, a.order, a.geo,
                     a.vq, a.X, a.Y, a.ldx, a.ldy, a.nvec, ntiles, nitems, chunk);
  return hipGetLastError();
}

template <int NP, int NQ, int B, int C, int NT, bool ACCUM>
__global__ void __attribute__((amdgpu_flat_work_group_size(1, NT),
                               amdgpu_waves_per_eu(vec32_waves_per_eu(NP, NQ, B, NT))))
apply_vec32_kernel(const GridDesc grid, const int32_t* __restrict__ order,
                   const double* __restrict__ geo, const double* __restrict__ vq,
                   const double* __restrict__ X, double* __restrict__ Y, int64_t ldx,
                   int64_t ldy, int nvec, int ntiles, int64_t nitems, int64_t chunk) {
  extern __shared__ double lds_d[];
  const int64_t item = xcd_item(blockIdx.x, chunk);
  if (item >= nitems) return;
  const int64_t e = order[item / ntiles];
  const int v0 = (int)(item % ntiles) * B;
  box_cell_tile<NP, NQ, B, C, NT, ACCUM, float>(reinterpret_cast<float*>(lds_d), grid, geo, vq, X,
                                                Y, ldx, ldy, nvec, e, v0);
}

template <int NP, int NQ, int B, int C, int NT, bool ACCUM>
hipError_t launch_vec32(const ApplyLaunch& a, hipStream_t s) {
  const int ntiles = (a.nvec + B - 1) / B;
  const int64_t nitems = a.ncells * ntiles;
  const int64_t chunk = (nitems + kXcds - 1) / kXcds;
  constexpr size_t lds = box_lds_bytes_t<float>(NP, NQ, B);
  static_assert(lds <= kLdsMax, "LDS");
  auto k = apply_vec32_kernel<NP, NQ, B, C, NT, ACCUM>;
  if (lds > 64 * 1024) {
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
  }
  hipLaunchKernelGGL(k, dim3((unsigned)(chunk * kXcds)), dim3(NT), lds, s, a.grid, a.order, a.geo,
                     a.vq, a.X, a.Y, a.ldx, a.ldy, a.nvec, ntiles, nitems, chunk);
  return hipGetLastError();
}

template <int NP, int NQ, int CFG>
hipError_t try_vec32(const ApplyLaunch& a, hipStream_t s, bool& done) {
  constexpr BoxCfg c = vec32_cfg(NP, NQ, CFG);
  if constexpr (c.B > 0) {
    if (a.cfg == CFG) {
      done = true;
      return a.accumulate ? launch_vec32<NP, NQ, c.B, c.C, c.NT, true>(a, s)
                          : launch_vec32<NP, NQ, c.B, c.C, c.NT, false>(a, s);
    }
  }
  return hipSuccess;
}

template <int NP, int NQ, int CFG, int PREC>
hipError_t try_cfg(const ApplyLaunch& a, hipStream_t s, bool& done) {
  constexpr BoxCfg c = mixed_cfg(NP, NQ, CFG);
  if constexpr (c.B > 0) {
    if (a.cfg == CFG) {
      done = true;
      return a.accumulate ? launch_mixed<NP, NQ, c.B, c.NT, true, PREC>(a, s)
                          : launch_mixed<NP, NQ, c.B, c.NT, false, PREC>(a, s);
    }
  }
  return hipSuccess;
}

template <int NP, int NQ, int PREC>
hipError_t launch_pq(const ApplyLaunch& a, hipStream_t s) {
  bool done = false;
  hipError_t err = hipSuccess;
  if (!done) err = try_cfg<NP, NQ, 0, PREC>(a, s, done);
  if (!done) err = try_cfg<NP, NQ, 1, PREC>(a, s, done);
  if (!done) err = try_cfg<NP, NQ, 2, PREC>(a, s, done);
  if (!done) err = try_cfg<NP, NQ, 3, PREC>(a, s, done);
  if constexpr (PREC == MF_FP32) {
    if (!done) err = try_vec32<NP, NQ, 4>(a, s, done);
    if (!done) err = try_vec32<NP, NQ, 5>(a, s, done);
    if (!done) err = try_vec32<NP, NQ, 6>(a, s, done);
  } else if (!done && a.cfg >= kMixedMfmaCfgs) {
    // the FP32 vector shapes have no BF16 form: BF16 runs its default shape
    ApplyLaunch a0 = a;
    a0.cfg = 0;
    err = try_cfg<NP, NQ, 0, PREC>(a0, s, done);
  }
  return done ? err : hipErrorInvalidValue;
}

template <int NP, int NQ>
hipError_t launch_pq_prec(const ApplyLaunch& a, int prec, hipStream_t s) {
  if (prec == MF_FP32) return launch_pq<NP, NQ, MF_FP32>(a, s);
  if (prec == MF_BF16) return launch_pq<NP, NQ, MF_BF16>(a, s);
  return hipErrorInvalidValue;
}

}  // namespace

template <>
hipError_t launch_apply_mixed_p<MF_P>(const Operator& op, const ApplyLaunch& a, int prec,
                                      hipStream_t s) {
  switch (op.q - MF_P) {
    case 1: return launch_pq_prec<MF_P + 1, MF_P + 1>(a, prec, s);
    case 2: return launch_pq_prec<MF_P + 1, MF_P + 2>(a, prec, s);
    case 3:
      if constexpr (mixed_cfg(MF_P + 1, MF_P + 3, 0).B > 0)
        return launch_pq_prec<MF_P + 1, MF_P + 3>(a, prec, s);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mf
