// Building blocks of the sum-factorisation kernels.
//
// Cell arrays live in LDS as [point][vector]: point index x + S0*(y + S1*z)
// (first reference direction fastest, Sec. 3.2.3), with the B vectors of the
// workgroup's tile innermost so that the lanes of a wavefront that work on the
// same pencil for consecutive vectors touch consecutive LDS words.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "mf_internal.h"

namespace mf {

constexpr int kXcds = 8;  // MI355X: workgroups are dealt round-robin to 8 XCDs

// Map a launch-order workgroup index to a work item so that every XCD gets a
// contiguous range of items (neighbouring cells share nodes, and the tiles of
// one cell share its map and geometry: keeping them on one XCD keeps the
// reuse inside that XCD's L2).
__device__ inline int64_t xcd_item(int64_t wg, int64_t chunk) {
  return (wg % kXcds) * chunk + wg / kXcds;
}

// Weight-folded 1D matrices passed by value in the kernel-argument segment:
// every lane reads the same entry at the same time, so the compiler serves them
// with scalar loads.  N[a*NP + i], D[a*NQ + b].
template <int NP, int NQ>
struct Mats {
  double N[NQ * NP];
  double D[NQ * NQ];
};

// out[o] = sum_i M(o, i) in[i]; M(o, i) = M[o*LD + i], or M[i*LD + o] if TR.
template <int NOUT, int NIN, bool TR, int LD, typename T>
__device__ __forceinline__ void matvec(const double* __restrict__ M, const T (&in)[NIN],
                                       T (&out)[NOUT]) {
#pragma unroll
  for (int o = 0; o < NOUT; ++o) {
    T acc = T(0);
#pragma unroll
    for (int i = 0; i < NIN; ++i) acc = fma(T(TR ? M[i * LD + o] : M[o * LD + i]), in[i], acc);
    out[o] = acc;
  }
}

// Pencil geometry of an (S0, S1, S2) array for a contraction along DIR.
template <int DIR, int S0, int S1, int S2>
struct Pencils {
  static constexpr int L = DIR == 0 ? S0 : (DIR == 1 ? S1 : S2);
  static constexpr int COUNT = (S0 * S1 * S2) / L;
  static constexpr int STRIDE = DIR == 0 ? 1 : (DIR == 1 ? S0 : S0 * S1);
  __device__ static inline int base(int pen) {
    if constexpr (DIR == 0) return pen * S0;
    else if constexpr (DIR == 1) return (pen / S0) * S0 * S1 + (pen % S0);
    else return pen;
  }
};

// One 1D contraction stage over every (vector, pencil) work item of the tile:
// dst (extent NOUT along DIR) = M applied along DIR to src (extents S0,S1,S2).
template <int DIR, int S0, int S1, int S2, int NOUT, bool TR, int LD, typename T>
__device__ __forceinline__ void stage(const T* __restrict__ src, T* __restrict__ dst,
                                      const double* __restrict__ M, int B, int tid, int nthr) {
  using PI = Pencils<DIR, S0, S1, S2>;
  using PO = Pencils<DIR, DIR == 0 ? NOUT : S0, DIR == 1 ? NOUT : S1, DIR == 2 ? NOUT : S2>;
  constexpr int NIN = PI::L;
  for (int w = tid; w < PI::COUNT * B; w += nthr) {
    const int b = w % B, pen = w / B;
    const int bi = PI::base(pen), bo = PO::base(pen);
    T r[NIN], o[NOUT];
#pragma unroll
    for (int i = 0; i < NIN; ++i) r[i] = src[(bi + i * PI::STRIDE) * B + b];
    matvec<NOUT, NIN, TR, LD>(M, r, o);
#pragma unroll
    for (int i = 0; i < NOUT; ++i) dst[(bo + i * PO::STRIDE) * B + b] = o[i];
  }
}

// LDS bytes of the FP64 kernel: three cell buffers, the scaled potential and the map.
inline size_t f64_lds_bytes(int np, int nq, int vtile) {
  const size_t nq3 = (size_t)nq * nq * nq, np3 = (size_t)np * np * np;
  return (3 * nq3 * vtile + nq3) * sizeof(double) + np3 * sizeof(int);
}

template <int P>
hipError_t launch_apply_f64_p(const Operator& op, const ApplyLaunch& a, hipStream_t s);

}  // namespace mf
