// Building blocks of the sum-factorisation kernels.
//
// Cell arrays live in LDS as [point][vector]: point index x + S0*(y + S1*z)
// (first reference direction fastest, Sec. 3.2.3), with the B vectors of the
// workgroup's tile innermost so that the lanes of a wavefront that work on the
// same pencil for consecutive vectors touch consecutive LDS words.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <utility>

#include "mf_internal.h"
#include "sf_tables.h"

namespace mf {

constexpr int kXcds = 8;  // MI355X: workgroups are dealt round-robin to 8 XCDs

// Map a launch-order workgroup index to a work item so that every XCD gets a
// contiguous range of items (neighbouring cells share nodes, and the tiles of
// one cell share its map and geometry: keeping them on one XCD keeps the
// reuse inside that XCD's L2).
__device__ inline int64_t xcd_item(int64_t wg, int64_t chunk) {
  return (wg % kXcds) * chunk + wg / kXcds;
}

// Grid node of local node (i1, i2, i3) of cell (cx, cy, cz) on a structured
// box mesh (periodic wrap; -1 for a zero-Dirichlet boundary node).
__device__ inline int grid_node(const GridDesc& g, int cx, int cy, int cz, int i1, int i2, int i3) {
  int gx = cx * g.p + i1, gy = cy * g.p + i2, gz = cz * g.p + i3;
  if (gx == g.N[0]) gx = 0;
  if (gy == g.N[1]) gy = 0;
  if (gz == g.N[2]) gz = 0;
  if (g.dirichlet && (gx == 0 || gx == g.N[0] - 1 || gy == 0 || gy == g.N[1] - 1 || gz == 0 ||
                      gz == g.N[2] - 1))
    return -1;
  return gx + g.N[0] * (gy + g.N[1] * gz);
}

// Compile-time coefficient sources: M::at<K> is the K-th entry of a 1D matrix
// as a constant expression, so contractions are emitted with literal
// coefficients (uniform operands, nothing loaded or held in registers).
template <int NP, int NQ>
struct MatN {  // folded N1D, NQ x NP, row-major
  template <int K>
  static constexpr double at = Tab<NP, NQ>::v.Nf[K];
  static constexpr double get(int k) { return Tab<NP, NQ>::v.Nf[k]; }
};
template <int NP, int NQ>
struct MatD {  // folded Dt, NQ x NQ, row-major
  template <int K>
  static constexpr double at = Tab<NP, NQ>::v.Dtf[K];
  static constexpr double get(int k) { return Tab<NP, NQ>::v.Dtf[k]; }
};

template <int NP, int NQ>
struct MatL {  // Dtf^T Dtf, NQ x NQ, symmetric
  template <int K>
  static constexpr double at = Tab<NP, NQ>::v.Lf[K];
  static constexpr double get(int k) { return Tab<NP, NQ>::v.Lf[k]; }
};

// ------------------------------------------------------------ even-odd form
// Points and nodes of the 1D rules are symmetric about the cell centre, so the
// folded interpolation matrix N (and its transpose) is centrosymmetric,
// M(m-1-o, n-1-i) = M(o, i), the folded derivative Dt is anti-centrosymmetric
// and Lf = Dt^T Dt is centrosymmetric again.  For such an m x n matrix,
//   y_o +- y_{m-1-o} = sum_{i < n/2} (M(o,i) +- M(o,n-1-i)) (x_i +- x_{n-1-i})
//                      [+ 2 M(o, n/2) x_{n/2} in the sum, odd n]
// and the middle row (odd m) sees only the even part.  This halves the
// coefficient uses of a contraction and cuts its arithmetic by about a
// quarter (the Kronecker structure itself is unchanged).
template <class M, bool TR, int LD>
constexpr double mco(int o, int i) {
  return M::get(TR ? i * LD + o : o * LD + i);
}
template <class M, int NOUT, int NIN, bool TR, int LD>
constexpr bool centrosymmetric() {
  for (int o = 0; o < NOUT; ++o)
    for (int i = 0; i < NIN; ++i) {
      const double a = mco<M, TR, LD>(o, i), b = mco<M, TR, LD>(NOUT - 1 - o, NIN - 1 - i);
      const double d = a - b, s = (a < 0 ? -a : a) + 1.0;
      if ((d < 0 ? -d : d) > 1e-13 * s) return false;
    }
  return true;
}
template <int N, class F, int... I>
__device__ __forceinline__ void sfor_(F& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
// compile-time loop: f(std::integral_constant<int, i>) for i = 0 .. N-1
template <int N, class F>
__device__ __forceinline__ void sfor(F&& f) {
  sfor_<N>(f, std::make_integer_sequence<int, N>{});
}

// Coefficients of the even / odd half-problems of an NOUT x NIN matrix.
template <class M, int NOUT, int NIN, bool TR, int LD>
struct EoMat {
  static constexpr int HI = NIN / 2, HO = NOUT / 2;
  static constexpr int MI = NIN % 2, MO = NOUT % 2;
  // even part of row o (o < HO, or the middle row o = HO of an odd NOUT) on
  // folded column i (i < HI: x_i + x_{n-1-i}; i = HI of an odd NIN: x_mid)
  static constexpr double e(int o, int i) {
    if (2 * i + 1 == NIN || 2 * o + 1 == NOUT) return mco<M, TR, LD>(o, i);
    return 0.5 * (mco<M, TR, LD>(o, i) + mco<M, TR, LD>(o, NIN - 1 - i));
  }
  // odd part of row o < HO on folded column i < HI (x_i - x_{n-1-i})
  static constexpr double d(int o, int i) {
    return 0.5 * (mco<M, TR, LD>(o, i) - mco<M, TR, LD>(o, NIN - 1 - i));
  }
  static constexpr int first_e(int o) {
    for (int i = 0; i < HI + MI; ++i)
      if (e(o, i) != 0.0) return i;
    return -1;
  }
  static constexpr int first_d(int o) {
    for (int i = 0; i < HI; ++i)
      if (d(o, i) != 0.0) return i;
    return -1;
  }
};

// y[r] = M x[r] for RN right-hand sides in even-odd form.  x is folded in
// place (x[r][i] <- x_i + x_{n-1-i}, x[r][n-1-i] <- x_i - x_{n-1-i}) and is
// not usable afterwards.  Every coefficient is a literal used RN times back to
// back; exact zeros are skipped.
template <class M, int NOUT, int NIN, bool TR, int LD, int RN, typename T>
__device__ __forceinline__ void eo_matvec(T (&x)[RN][NIN], T (&y)[RN][NOUT]) {
  using E = EoMat<M, NOUT, NIN, TR, LD>;
  static_assert(centrosymmetric<M, NOUT, NIN, TR, LD>(), "matrix is not centrosymmetric");
#pragma unroll
  for (int r = 0; r < RN; ++r)
#pragma unroll
    for (int i = 0; i < E::HI; ++i) {
      const T a = x[r][i], b = x[r][NIN - 1 - i];
      x[r][i] = a + b;
      x[r][NIN - 1 - i] = a - b;
    }
  sfor<E::HO + E::MO>([&](auto O) {
    constexpr int o = decltype(O)::value;
    T ev[RN], od[RN];
    constexpr int fe = E::first_e(o);
    if constexpr (fe < 0) {
#pragma unroll
      for (int r = 0; r < RN; ++r) ev[r] = T(0);
    } else {
      sfor<E::HI + E::MI>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr T c = (T)E::e(o, i);
        if constexpr (i == fe) {
#pragma unroll
          for (int r = 0; r < RN; ++r) ev[r] = c * x[r][i];
        } else if constexpr (i > fe && c != T(0)) {
#pragma unroll
          for (int r = 0; r < RN; ++r) ev[r] = fma(c, x[r][i], ev[r]);
        }
      });
    }
    if constexpr (o == E::HO) {  // middle row of an odd NOUT
#pragma unroll
      for (int r = 0; r < RN; ++r) y[r][o] = ev[r];
    } else {
      constexpr int fd = E::first_d(o);
      if constexpr (fd < 0) {
#pragma unroll
        for (int r = 0; r < RN; ++r) {
          y[r][o] = ev[r];
          y[r][NOUT - 1 - o] = ev[r];
        }
      } else {
        sfor<E::HI>([&](auto I) {
          constexpr int i = decltype(I)::value;
          constexpr T c = (T)E::d(o, i);
          if constexpr (i == fd) {
#pragma unroll
            for (int r = 0; r < RN; ++r) od[r] = c * x[r][NIN - 1 - i];
          } else if constexpr (i > fd && c != T(0)) {
#pragma unroll
            for (int r = 0; r < RN; ++r) od[r] = fma(c, x[r][NIN - 1 - i], od[r]);
          }
        });
#pragma unroll
        for (int r = 0; r < RN; ++r) {
          y[r][o] = ev[r] + od[r];
          y[r][NOUT - 1 - o] = ev[r] - od[r];
        }
      }
    }
  });
}

template <class M, bool TR, int LD, int O, typename T, int NIN, int... I>
__device__ __forceinline__ T mrow(const T (&in)[NIN], std::integer_sequence<int, I...>) {
  T acc = T(0);
  // entries that are exactly zero (a Gauss point on a GLL node) are skipped
  ((M::template at<(TR ? I * LD + O : O * LD + I)> != 0.0
        ? (void)(acc = fma(T(M::template at<(TR ? I * LD + O : O * LD + I)>), in[I], acc))
        : (void)0),
   ...);
  return acc;
}

template <class M, bool TR, int LD, typename T, int NIN, int NOUT, int... O>
__device__ __forceinline__ void mvec(const T (&in)[NIN], T (&out)[NOUT],
                                     std::integer_sequence<int, O...>) {
  ((out[O] = mrow<M, TR, LD, O>(in, std::make_integer_sequence<int, NIN>{})), ...);
}

// out[o] = sum_i M(o, i) in[i]; M(o, i) = M[o*LD + i], or M[i*LD + o] if TR.
template <class M, int NOUT, int NIN, bool TR, int LD, typename T>
__device__ __forceinline__ void matvec(const T (&in)[NIN], T (&out)[NOUT]) {
  mvec<M, TR, LD>(in, out, std::make_integer_sequence<int, NOUT>{});
}

// Multi-right-hand-side form: out[r][o] = sum_i M(o, i) in[r][i] for R pencils.
// Each coefficient is formed once and used R times back to back (the R
// accumulation chains are independent), which keeps the scalar constants
// short-lived instead of parked in registers for the whole phase.
template <class M, bool TR, int LD, int O, int I>
constexpr double coef() {
  return M::template at<(TR ? I * LD + O : O * LD + I)>;
}
template <class M, bool TR, int LD, int R, int O, int I, int FIRST, typename T, int NIN, int NOUT>
__device__ __forceinline__ void mrhs_term(const T (&in)[R][NIN], T (&out)[R][NOUT]) {
  constexpr double c = coef<M, TR, LD, O, I>();
  if constexpr (I == FIRST) {
#pragma unroll
    for (int r = 0; r < R; ++r) out[r][O] = T(c) * in[r][I];
  } else if constexpr (c != 0.0) {
#pragma unroll
    for (int r = 0; r < R; ++r) out[r][O] = fma(T(c), in[r][I], out[r][O]);
  }
}
template <class M, bool TR, int LD, int O, int... I>
constexpr int first_nonzero(std::integer_sequence<int, I...>) {
  constexpr int n = sizeof...(I);
  constexpr double cs[n] = {coef<M, TR, LD, O, I>()...};
  for (int i = 0; i < n; ++i)
    if (cs[i] != 0.0) return i;
  return 0;
}
template <class M, bool TR, int LD, int R, int O, typename T, int NIN, int NOUT, int... I>
__device__ __forceinline__ void mrhs_row(const T (&in)[R][NIN], T (&out)[R][NOUT],
                                         std::integer_sequence<int, I...> seq) {
  constexpr int FIRST = first_nonzero<M, TR, LD, O>(seq);
  (mrhs_term<M, TR, LD, R, O, I, FIRST>(in, out), ...);
}
template <class M, bool TR, int LD, int R, typename T, int NIN, int NOUT, int... O>
__device__ __forceinline__ void mrhs_all(const T (&in)[R][NIN], T (&out)[R][NOUT],
                                         std::integer_sequence<int, O...>) {
  (mrhs_row<M, TR, LD, R, O>(in, out, std::make_integer_sequence<int, NIN>{}), ...);
}
// Multi-right-hand-side form: out[r][o] = sum_i M(o, i) in[r][i] for R pencils.
// Each coefficient is formed once and used R times back to back (the R
// accumulation chains are independent); the first nonzero term of a row starts
// the sum with a multiply, exact zeros are skipped.
template <class M, int NOUT, int NIN, bool TR, int LD, int R, typename T>
__device__ __forceinline__ void matvec_multi(const T (&in)[R][NIN], T (&out)[R][NOUT]) {
  mrhs_all<M, TR, LD, R>(in, out, std::make_integer_sequence<int, NOUT>{});
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
template <class M, int DIR, int S0, int S1, int S2, int NOUT, bool TR, int LD, int B, int NT,
          typename T>
__device__ __forceinline__ void stage(const T* __restrict__ src, T* __restrict__ dst, int tid) {
  using PI = Pencils<DIR, S0, S1, S2>;
  using PO = Pencils<DIR, DIR == 0 ? NOUT : S0, DIR == 1 ? NOUT : S1, DIR == 2 ? NOUT : S2>;
  constexpr int NIN = PI::L;
  for (int w = tid; w < PI::COUNT * B; w += NT) {
    const int b = w % B, pen = w / B;
    const int bi = PI::base(pen), bo = PO::base(pen);
    T r[NIN], o[NOUT];
#pragma unroll
    for (int i = 0; i < NIN; ++i) r[i] = src[(bi + i * PI::STRIDE) * B + b];
    matvec<M, NOUT, NIN, TR, LD>(r, o);
#pragma unroll
    for (int i = 0; i < NOUT; ++i) dst[(bo + i * PO::STRIDE) * B + b] = o[i];
  }
}

constexpr int kThreads = 256;             // workgroup size of the fused kernels
constexpr size_t kLdsBudget = 64 * 1024;   // LDS per workgroup the kernels stay within

// LDS bytes of the FP64 kernel: three cell buffers, the scaled potential and the map.
constexpr size_t f64_lds_bytes(int np, int nq, int vtile) {
  return (3 * (size_t)nq * nq * nq * vtile + (size_t)nq * nq * nq) * sizeof(double) +
         (size_t)np * np * np * sizeof(int);
}
// Largest vector tile that fits the LDS budget (0 if none).
constexpr int f64_bmax(int np, int nq) {
  int b = 0;
  while (f64_lds_bytes(np, nq, b + 1) <= kLdsBudget && b < 64) ++b;
  return b;
}
// Default tile: enough (vector, pencil) items to occupy the workgroup in the
// pencil stages, within the LDS budget.
constexpr int f64_bdef(int np, int nq) {
  int b = kThreads / (nq * nq);
  if (b < 1) b = 1;
  const int m = f64_bmax(np, nq);
  return b < m ? b : m;
}
// Vector tiles instantiated per (np, nq): 1, 2, 4, 8 and the default, within budget.
constexpr bool f64_tile_built(int np, int nq, int b) {
  return b >= 1 && b <= f64_bmax(np, nq) && (b == 1 || b == 2 || b == 4 || b == 8 || b == f64_bdef(np, nq));
}

constexpr size_t kLdsMax = 160 * 1024;     // LDS per workgroup on gfx950

// LDS bytes of the box-cell kernel: two cell buffers and the scaled potential
// (node numbers stay in the registers of the threads that gather and assemble).
constexpr size_t box_lds_bytes(int np, int nq, int vtile) {
  return (2 * (size_t)nq * nq * nq * vtile + (size_t)nq * nq * nq) * sizeof(double) + 0 * np;
}
// The same for cell arrays of type T (the FP32 vector apply keeps them in float).
template <typename T>
constexpr size_t box_lds_bytes_t(int np, int nq, int vtile) {
  return (2 * (size_t)nq * nq * nq * vtile + (size_t)nq * nq * nq) * sizeof(T) + 0 * np;
}

// Launch shapes of the box-cell kernel: vector tile B, threads NT (0: the
// fewest whole wavefronts that cover the largest phase, nq^2 B / C tasks),
// columns per thread C, and the one-shot grid (one workgroup per item) or the
// persistent grid (resident workgroups, next item prefetched).  B = 8 and 16
// make the [point][vector] LDS accesses of the lanes of one pencil contiguous.
// A shape that does not fit the LDS has B = 0.
struct BoxCfg {
  int B, NT;
  int C = 1;
  bool pers = false;
};
constexpr BoxCfg box_cfg_raw(int idx) {
  switch (idx) {
    case 1: return BoxCfg{8, 512, 1, false};
    case 2: return BoxCfg{8, 256, 2, false};
    case 3: return BoxCfg{8, 512, 1, true};
    case 4: return BoxCfg{8, 256, 2, true};
    case 5: return BoxCfg{8, 0, 1, true};
    case 6: return BoxCfg{8, 0, 1, false};
    case 7: return BoxCfg{4, 256, 1, false};
    case 8: return BoxCfg{4, 0, 1, true};
    case 9: return BoxCfg{4, 0, 1, false};
    // narrow blocks: one (B = 1) or two (B = 2) wavefronts per cell, so the
    // barriers between the stages are those of one or two wavefronts
    case 11: return BoxCfg{1, 0, 1, false};
    case 12: return BoxCfg{2, 0, 1, false};
    default: return BoxCfg{0, 256, 1, false};
  }
}
constexpr BoxCfg box_cfg_fix(int np, int nq, BoxCfg c) {
  if (c.NT == 0) {
    const int tasks = nq * nq * (c.B / c.C);
    c.NT = (tasks + 63) / 64 * 64;
    if (c.NT > 1024) c.NT = 1024;
  }
  if (c.B == 0 || box_lds_bytes(np, nq, c.B) > kLdsMax) c.B = 0;
  (void)np;
  return c;
}
constexpr BoxCfg box_cfg(int np, int nq, int idx) {
  // 0: default (fastest measured per size class): one-shot, B = 8, fewest
  //    whole wavefronts when two 8-column cell buffers fit in 80 KiB of LDS
  //    (three workgroups per CU); else persistent B = 8 if it fits the LDS at
  //    all, else persistent B = 4.  1 .. 9: fixed shapes, for the tuner.
  if (idx == 0) {
    if (box_lds_bytes(np, nq, 8) <= 80 * 1024) return box_cfg_fix(np, nq, box_cfg_raw(6));
    if (box_lds_bytes(np, nq, 8) <= kLdsMax) return box_cfg_fix(np, nq, box_cfg_raw(5));
    return box_cfg_fix(np, nq, box_cfg_raw(8));
  }
  return box_cfg_fix(np, nq, box_cfg_raw(idx));
}
// Shape with one column per thread and the same tile, used when a call cannot
// take 16-byte column pairs (odd nvec or leading dimension, unaligned X or Y).
constexpr int box_cfg_single(int np, int nq, int idx) {
  const BoxCfg c = box_cfg(np, nq, idx);
  if (c.C == 1) return idx;
  if (c.B >= 8 && box_cfg(np, nq, c.pers ? 5 : 6).B > 0) return c.pers ? 5 : 6;
  return c.pers ? 8 : 9;
}
// Workgroups per CU that the LDS allows, and the matching waves per SIMD the
// register allocation must leave room for.
constexpr int box_wg_per_cu(int np, int nq, int B, int NT = 256) {
  const size_t l = box_lds_bytes(np, nq, B);
  int n = (int)(kLdsMax / (l > 0 ? l : 1));
  const int cap = NT <= 128 ? 32 : 8;  // the narrow shapes run many small workgroups
  return n < 1 ? 1 : (n > cap ? cap : n);
}
constexpr int box_waves_per_eu(int np, int nq, int B, int NT) {
  const int w = (box_wg_per_cu(np, nq, B, NT) * (NT / 64) + 3) / 4;
  return w < 1 ? 1 : (w > 8 ? 8 : w);
}

// LDS bytes of the mixed-precision kernel: 64-bit X and Y row offsets, two FP32
// cell buffers, the FP32 scaled potential and one exponent per column.
constexpr size_t mixed_lds_bytes(int np, int nq, int vtile) {
  return 2 * (size_t)np * np * np * sizeof(int64_t) +
         (2 * (size_t)nq * nq * nq * vtile + (size_t)nq * nq * nq) * sizeof(float) +
         (size_t)vtile * sizeof(int);
}
// Launch shapes of the mixed-precision kernel (B columns, NT threads):
// 0: default B = 16, 512 threads (B = 8 if that exceeds 80 KiB of LDS);
// 1: B = 16, 256;  2: B = 8, 256;  3: B = 8, 512.
constexpr BoxCfg mixed_cfg(int np, int nq, int idx) {
  BoxCfg c{0, 512};
  if (idx == 0) {
    if (mixed_lds_bytes(np, nq, 16) <= 80 * 1024) return BoxCfg{16, 512};
    for (int b = 8; b >= 1; b /= 2)
      if (mixed_lds_bytes(np, nq, b) <= kLdsMax) return BoxCfg{b, b >= 8 ? 512 : 256};
    return c;
  }
  if (idx == 1) c = BoxCfg{16, 256};
  if (idx == 2) c = BoxCfg{8, 256};
  if (idx == 3) c = BoxCfg{8, 512};
  if (mixed_lds_bytes(np, nq, c.B) > kLdsMax) c.B = 0;
  return c;
}

// FP32 vector shapes of the mixed-precision apply (shapes 4 .. 6): the box
// kernel's even-odd contractions on FP32 cell arrays (FP64 X and Y, FP64
// assembly), half the LDS per column of the FP64 kernel.  4: B = 16 with two
// columns per thread; 5: B = 8; 6: B = 16, one column per thread; each with
// the fewest whole wavefronts covering the nq^2 B / C pencil tasks.
constexpr int kMixedMfmaCfgs = 4;
constexpr BoxCfg vec32_cfg(int np, int nq, int idx) {
  BoxCfg c{0, 0, 1, false};
  if (idx == 4) c = BoxCfg{16, 0, 2, false};
  if (idx == 5) c = BoxCfg{8, 0, 1, false};
  if (idx == 6) c = BoxCfg{16, 0, 1, false};
  if (c.B == 0) return c;
  c.NT = (nq * nq * c.B / c.C + 63) / 64 * 64;
  if (c.NT > 1024 || box_lds_bytes_t<float>(np, nq, c.B) > kLdsMax) c.B = 0;
  return c;
}
// shape with one column per thread for calls that cannot take column pairs
constexpr int vec32_cfg_single(int idx) { return idx == 4 ? 5 : idx; }
constexpr int vec32_waves_per_eu(int np, int nq, int B, int NT) {
  const size_t l = box_lds_bytes_t<float>(np, nq, B);
  int wg = (int)(kLdsMax / (l > 0 ? l : 1));
  wg = wg < 1 ? 1 : (wg > 8 ? 8 : wg);
  const int w = (wg * (NT / 64) + 3) / 4;
  return w < 1 ? 1 : (w > 8 ? 8 : w);
}

// ---------------------------------------------------------------- batches
// Launch shapes of the persistent batched kernel (kinds q = p + 1, p = 2..8):
// 0: 512 threads; FP64 tile per kind filling the workgroup's pencil tasks
//    (nq^2 B up to 512: B = 16 for nq <= 5, 8 up to 80 KiB of LDS, else 4),
//    mixed the largest of 16 / 8 within 80 KiB;
// 1: 512 threads, FP64 B = 8 / mixed B = 16 for every kind;
// 2: 256 threads, FP64 B = 4 / mixed B = 8.
constexpr int kBatchMinP = 2, kBatchMaxP = 8;
constexpr int batch_threads(int bcfg) { return bcfg == 2 ? 256 : 512; }
// Per-kind launches (shapes 3..5): the kind's own default tile and the fewest
// whole wavefronts covering its pencil tasks (FP64, one column per thread),
// the FP32 vector default, or the BF16 matrix-core default.
constexpr BoxCfg batch_kind_shape(int prec, int np, int nq) {
  if (prec == MF_FP64) {
    BoxCfg c = box_cfg(np, nq, 0);
    c.C = 1;
    c.pers = false;
    c.NT = (nq * nq * c.B + 63) / 64 * 64;
    if (c.NT > 1024) c.NT = 1024;
    return c;
  }
  if (prec == MF_FP32) {  // the FP32 vector shapes, as the single apply's default
    const BoxCfg c = vec32_cfg(np, nq, 6);
    return c.B > 0 ? c : vec32_cfg(np, nq, 5);
  }
  return mixed_cfg(np, nq, 0);
}
constexpr int batch_tile(int prec, int bcfg, int np, int nq) {
  const bool f64 = prec == MF_FP64;
  if (bcfg >= 3) return batch_kind_shape(prec, np, nq).B;
  if (bcfg == 1) return f64 ? 8 : 16;
  if (bcfg == 2) return f64 ? 4 : 8;
  if (f64) {
    if (nq * nq * 16 <= 512 && box_lds_bytes(np, nq, 16) <= 80 * 1024) return 16;
    return box_lds_bytes(np, nq, 8) <= 80 * 1024 ? 8 : 4;
  }
  return mixed_lds_bytes(np, nq, 16) <= 80 * 1024 ? 16 : 8;
}
constexpr size_t batch_lds_bytes(int prec, int bcfg) {
  size_t m = 0;
  for (int p = kBatchMinP; p <= kBatchMaxP; ++p) {
    const int n = p + 1, b = batch_tile(prec, bcfg, n, n);
    const size_t l = prec == MF_FP64 ? box_lds_bytes(n, n, b) : mixed_lds_bytes(n, n, b);
    if (l > m) m = l;
  }
  return m;
}
template <int PREC, int BCFG>
hipError_t launch_batched_kernel(const BatchOp* ops, const uint8_t* item_op, const int64_t* bounds,
                                 const BatchPtrs& ptrs, int grid, hipStream_t s);
template <int PREC, int BCFG>
int batched_occupancy();
// per-kind kernels, p = 2 .. 8: loop = resident grid (shape 3), else one
// item per workgroup (shape 4)
template <int PREC>
hipError_t launch_batched_kind(int p, bool loop, const BatchOp* ops, const uint8_t* item_op,
                               const int64_t* bounds, const BatchPtrs& ptrs, int grid,
                               hipStream_t s);
template <int PREC>
int batched_kind_occupancy(int p);

template <int P>
hipError_t launch_apply_f64_p(const Operator& op, const ApplyLaunch& a, hipStream_t s);
template <int P>
hipError_t launch_apply_mixed_p(const Operator& op, const ApplyLaunch& a, int prec, hipStream_t s);
template <int P>
hipError_t launch_apply_box_p(const Operator& op, const ApplyLaunch& a, hipStream_t s);
template <int P>
hipError_t launch_apply_mfma_p(const Operator& op, const ApplyLaunch& a, hipStream_t s);
template <int P>
hipError_t launch_cheb_p(const Operator& op, const double* Y, double* Out, int64_t ld, int nvec,
                         const ChebArgs& ca, hipStream_t s);

}  // namespace mf
