// Fused apply (FP64, or FP32 cell arrays) for axis-aligned cells given by an
// explicit cell-to-node map (the refined meshes of include/mfrefine.h: cells of two sizes, node
// numbers that no grid formula gives).  The per-item body is the box kernel's
// (box_body.h: even-odd contractions, collapsed diagonal 3x3 factor, plain
// stores on cell-interior rows and FP64 atomics on shared rows); only the node
// numbers come from the map instead of the structured-grid arithmetic.
//
// Work item = (cell, tile of B columns), one workgroup per item, items spread
// over the XCDs in contiguous chunks (cells of one chunk are neighbours in the
// numbering, so they share nodes within one L2).
#include "box_body.h"
#include "mf_internal.h"

#ifndef MF_P
#error "compile with -DMF_P=<degree>"
#endif

namespace mf {
namespace {

// Node numbers of the thread's tasks from row e of the map (local node
// i1 + np (i2 + np i3), pencil pen = i2 + np i3; -1 = zero-Dirichlet).
template <int NP, int B, int C, int NT, typename T>
__device__ __forceinline__ void load_map(BoxGather<NP, B, C, NT, T>& Gt,
                                         const int32_t* __restrict__ map, int64_t e, int tid) {
  using GT = BoxGather<NP, B, C, NT, T>;
  const int32_t* row = map + e * (NP * NP * NP);
#pragma unroll
  for (int k = 0; k < GT::R1; ++k) {
    const int pen = GT::TK::clamp(tid + k * NT) / GT::G;
#pragma unroll
    for (int i = 0; i < NP; ++i) Gt.node[k][i] = row[pen * NP + i];
  }
}

constexpr int map_tile(int np, int nq) { return box_lds_bytes(np, nq, 8) <= kLdsMax ? 8 : 4; }
constexpr int map_threads(int nq, int B) {
  const int t = (nq * nq * B + 63) / 64 * 64;  // fewest whole wavefronts over the widest phase
  return t > 1024 ? 1024 : t;
}
template <typename T>
constexpr int map_waves(int np, int nq, int B, int NT) {
  return std::is_same<T, float>::value ? vec32_waves_per_eu(np, nq, B, NT)
                                       : box_waves_per_eu(np, nq, B, NT);
}

// T = double: FP64 throughout.  T = float: the cell arrays of the FP32 vector
// apply (power-of-two scaling per cell and column, FP64 assembly).
template <int NP, int NQ, int B, int NT, bool ACCUM, typename T>
__global__ void __attribute__((amdgpu_flat_work_group_size(1, NT),
                               amdgpu_waves_per_eu(map_waves<T>(NP, NQ, B, NT))))
apply_box_map_kernel(const int32_t* __restrict__ map, const double* __restrict__ geo,
                     const double* __restrict__ vq, const double* __restrict__ X,
                     double* __restrict__ Y, int64_t ldx, int64_t ldy, int nvec, int ntiles,
                     int64_t nitems, int64_t chunk) {
  extern __shared__ double lds_raw[];
  const int64_t item = xcd_item(blockIdx.x, chunk);
  if (item >= nitems) return;
  const int64_t e = item / ntiles;
  const int v0 = (int)(item % ntiles) * B;
  constexpr int NQ3 = NQ * NQ * NQ;
  T* bA = reinterpret_cast<T*>(lds_raw);
  T* bB = bA + NQ3 * B;
  T* svq = bB + NQ3 * B;
  const int tid = threadIdx.x;
  BoxGather<NP, B, 1, NT, T> Gt;
  load_map(Gt, map, e, tid);
  for (int i = tid; i < NQ3; i += NT) svq[i] = (T)vq[e * NQ3 + i];
  const T g0 = (T)geo[e * 6 + 0], g1 = (T)geo[e * 6 + 3], g2 = (T)geo[e * 6 + 5];
  Gt.load_x(X, ldx, nvec, v0, tid);
  if constexpr (std::is_same<T, float>::value)
    Gt.scale(reinterpret_cast<int*>(bB), tid);  // B is first written in P2
  box_p1<NP, NQ, B, 1, NT, T>(bA, Gt, tid);
  __syncthreads();
  box_mid<NP, NQ, B, 1, NT, T>(bA, bB, svq, g0, g1, g2, tid);
  box_p8<NP, NQ, B, 1, NT, ACCUM, T>(bB, Gt, Y, ldy, nvec, v0, tid);
}

template <int NP, int NQ, int B, bool ACCUM, typename T>
hipError_t launch_map(const ApplyLaunch& a, hipStream_t s) {
  constexpr int NT = map_threads(NQ, B);
  constexpr size_t lds = box_lds_bytes_t<T>(NP, NQ, B);
  static_assert(lds <= kLdsMax, "LDS");
  const int ntiles = (a.nvec + B - 1) / B;
  const int64_t nitems = a.ncells * ntiles;
  const int64_t chunk = (nitems + kXcds - 1) / kXcds;
  auto k = apply_box_map_kernel<NP, NQ, B, NT, ACCUM, T>;
  KernelFacts f;  // raises the dynamic LDS limit on this device
  hipError_t err = kernel_facts(reinterpret_cast<const void*>(k), NT, lds, f);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k, dim3((unsigned)(chunk * kXcds)), dim3(NT), lds, s, a.map, a.geo, a.vq,
                     a.X, a.Y, a.ldx, a.ldy, a.nvec, ntiles, nitems, chunk);
  return hipGetLastError();
}

template <int NP, int NQ>
hipError_t launch_map_pq(const ApplyLaunch& a, hipStream_t s) {
  constexpr int B = map_tile(NP, NQ);
  return a.accumulate ? launch_map<NP, NQ, B, true, double>(a, s)
                      : launch_map<NP, NQ, B, false, double>(a, s);
}

// FP32: 16 columns per item when more than 8 are asked for and the tile fits,
// else 8 (the FP32 vector shapes of the uniform mesh, one column per thread).
template <int NP, int NQ>
hipError_t launch_map32_pq(const ApplyLaunch& a, hipStream_t s) {
  constexpr bool b16 = vec32_cfg(NP, NQ, 6).B > 0;
  constexpr bool b8 = vec32_cfg(NP, NQ, 5).B > 0;
  if constexpr (b16) {
    if (a.nvec > 8 || !b8)
      return a.accumulate ? launch_map<NP, NQ, 16, true, float>(a, s)
                          : launch_map<NP, NQ, 16, false, float>(a, s);
  }
  if constexpr (b8)
    return a.accumulate ? launch_map<NP, NQ, 8, true, float>(a, s)
                        : launch_map<NP, NQ, 8, false, float>(a, s);
  return hipErrorInvalidValue;
}

}  // namespace

template <>
hipError_t launch_apply_box_map32_p<MF_P>(const Operator& op, const ApplyLaunch& a,
                                          hipStream_t s) {
  switch (op.q - MF_P) {
    case 1: return launch_map32_pq<MF_P + 1, MF_P + 1>(a, s);
    case 2: return launch_map32_pq<MF_P + 1, MF_P + 2>(a, s);
    case 3: return launch_map32_pq<MF_P + 1, MF_P + 3>(a, s);
    default: return hipErrorInvalidValue;
  }
}

template <>
hipError_t launch_apply_box_map_p<MF_P>(const Operator& op, const ApplyLaunch& a, hipStream_t s) {
  switch (op.q - MF_P) {
    case 1: return launch_map_pq<MF_P + 1, MF_P + 1>(a, s);
    case 2: return launch_map_pq<MF_P + 1, MF_P + 2>(a, s);
    case 3: return launch_map_pq<MF_P + 1, MF_P + 3>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mf
