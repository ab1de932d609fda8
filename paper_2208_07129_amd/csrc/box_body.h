// Body of the FP64 fused apply for axis-aligned (box) cells, as a device
// function over one (cell, column tile) work item, shared by the one-shot
// kernel (apply_box.hip) and the persistent batched kernel (apply_batched.hip).
//
// On a box cell the Jacobian is diagonal, so the 3x3 factor of eq. sjacobian is
// diagonal: G = diag(g0, g1, g2) per cell.  The gradient part of Alg. 2 then
// splits by direction, sum_s Dt_s^T g_s Dt_s T, and the two derivative stages
// of direction s collapse into one symmetric contraction with
// Lf = Dtf^T Dtf (weight-folded).  Per cell e and column:
//   T   = (N x N x N) U_e                          (Alg. 1, eq. tc1-tc3)
//   T  <- det J (V + sigma) o T + sum_s g_s Lf_s T  (eq. helmholtz, eq. mjacobian)
//   V_e = (N x N x N)^T T;  Y += Q_e^T V_e         (Sec. 3.2.3)
// Every 1D contraction runs in even-odd form (eo_matvec).  Only two cell
// buffers live in LDS (the general kernel needs three), and seven stages
// separated by six barriers cover the whole chain (box_mid).
//
// Work split: a tile of B columns is cut into G = B / C groups of C adjacent
// columns; a task is one (pencil, column group), so a thread applies every
// coefficient to C columns (and R pencils when the tasks outnumber the
// threads), and with C = 2 its LDS and global accesses are 16 bytes wide.
// Inside a phase each thread issues all its LDS reads before computing.
// Nodes interior to the cell have exactly one contributor and are written
// with plain stores; nodes on cell faces, edges and corners use FP64 atomics
// (their rows are zeroed beforehand).
#pragma once

#include <type_traits>

#include "mf_internal.h"
#include "sf_common.h"
#include "sf_tables.h"

namespace mf {

// C adjacent columns of one LDS point <-> rows row .. row+C-1 of a register
// block d[RN][N] at entry i.
// T is the arithmetic type of the cell arrays: double (the FP64 apply) or
// float (the FP32 vector apply; X and Y stay FP64 in HBM).
template <typename T>
struct Pair;
template <>
struct Pair<double> {
  using type = double2;
};
template <>
struct Pair<float> {
  using type = float2;
};

template <int C, int RN, int N, typename T>
__device__ __forceinline__ void lds_get(const T* __restrict__ p, T (&d)[RN][N], int row, int i) {
  if constexpr (C == 1) {
    d[row][i] = p[0];
  } else {
    static_assert(C == 2, "C is 1 or 2");
    const auto v = *reinterpret_cast<const typename Pair<T>::type*>(p);
    d[row][i] = v.x;
    d[row + 1][i] = v.y;
  }
}
template <int C, int RN, int N, typename T>
__device__ __forceinline__ void lds_put(T* __restrict__ p, const T (&s)[RN][N], int row, int i) {
  if constexpr (C == 1) {
    p[0] = s[row][i];
  } else {
    typename Pair<T>::type v;
    v.x = s[row][i];
    v.y = s[row + 1][i];
    *reinterpret_cast<typename Pair<T>::type*>(p) = v;
  }
}

// Task rounds of a phase with PENS pencils: T tasks, R per thread.
template <int PENS, int G, int NT>
struct Tasks {
  static constexpr int T = PENS * G;
  static constexpr int R = (T + NT - 1) / NT;
  static constexpr bool EXACT = T % NT == 0;
  // task of round k, clamped to task 0 past the end (its reads stay in
  // bounds; its results are not stored)
  __device__ static inline int clamp(int w) { return (EXACT || w < T) ? w : 0; }
  __device__ static inline bool live(int k, int w) { return EXACT || k < R - 1 || w < T; }
};

// One contraction along DIR: dst (extent NOUT along DIR) = Mat applied to src
// (extents S0, S1, S2), in place allowed when src and dst are one buffer and
// every pencil keeps its positions (each pencil has a single owner).
template <class Mat, bool TR, int LD, int DIR, int S0, int S1, int S2, int NOUT, int B, int C,
          int NT, typename T>
__device__ __forceinline__ void box_stage(const T* src, T* dst, int tid) {
  using PI = Pencils<DIR, S0, S1, S2>;
  using PO = Pencils<DIR, DIR == 0 ? NOUT : S0, DIR == 1 ? NOUT : S1, DIR == 2 ? NOUT : S2>;
  constexpr int NIN = PI::L, G = B / C;
  using TK = Tasks<PI::COUNT, G, NT>;
  constexpr int R = TK::R;
  T in[R * C][NIN], out[R * C][NOUT];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int w = TK::clamp(tid + k * NT);
    const int g = w % G, bi = PI::base(w / G);
#pragma unroll
    for (int i = 0; i < NIN; ++i) lds_get<C>(src + (bi + i * PI::STRIDE) * B + g * C, in, k * C, i);
  }
  eo_matvec<Mat, NOUT, NIN, TR, LD, R * C>(in, out);
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int w = tid + k * NT;
    if (!TK::live(k, w)) continue;
    const int g = w % G, bo = PO::base(w / G);
#pragma unroll
    for (int i = 0; i < NOUT; ++i) lds_put<C>(dst + (bo + i * PO::STRIDE) * B + g * C, out, k * C, i);
  }
}

// Per-thread registers of one work item's extraction: for each of the R1
// tasks (direction-0 pencil (i2, i3), column group) of this thread, the NP
// node numbers of the pencil (-1 for a constrained node) and the gathered X
// values of its C columns.  The same thread owns the same tasks in the last
// phase, so the node numbers also drive the assembly.
//
// With FP32 cell arrays (T = float) every (cell, column) is scaled by a power
// of two 2^-e before the conversion, e the exponent of the column's largest
// gathered magnitude, and the assembly multiplies by 2^e again: the FP32
// stages then see values below 1 whatever the magnitude of X (scaling by a
// power of two is exact).
template <int NP, int B, int C, int NT, typename T = double>
struct BoxGather {
  static constexpr int G = B / C;
  using TK = Tasks<NP * NP, G, NT>;
  static constexpr int T1 = TK::T;
  static constexpr int R1 = TK::R;
  static constexpr bool F32 = std::is_same<T, float>::value;
  int node[R1][NP];
  double x[R1 * C][NP];                 // gathered FP64 values
  T xs[F32 ? R1 * C : 1][NP];           // scaled FP32 values (T = float)
  int ex[F32 ? C : 1];                  // column exponents e (T = float)

  // Node numbers from the structured-grid arithmetic: cell e at (cx, cy, cz),
  // local node (i1, i2, i3) -> grid node (cx p + i1, ...) with the periodic
  // wrap, -1 on the boundary of a zero-Dirichlet mesh.
  __device__ __forceinline__ void load_grid(const GridDesc& gd, int64_t e, int tid) {
    const int ei = (int)e;
    const int cx = ei % gd.n[0], cy = (ei / gd.n[0]) % gd.n[1], cz = ei / (gd.n[0] * gd.n[1]);
#pragma unroll
    for (int k = 0; k < R1; ++k) {
      const int pen = TK::clamp(tid + k * NT) / G;
      const int i2 = pen % NP, i3 = pen / NP;
      int gy = cy * gd.p + i2, gz = cz * gd.p + i3;
      if (gy == gd.N[1]) gy = 0;  // only reachable on a periodic mesh
      if (gz == gd.N[2]) gz = 0;
      const bool yz_bnd =
          gd.dirichlet && (gy == 0 || gy == gd.N[1] - 1 || gz == 0 || gz == gd.N[2] - 1);
      const int rowbase = gd.N[0] * (gy + gd.N[1] * gz);
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        int gx = cx * gd.p + i;
        if (gx == gd.N[0]) gx = 0;
        const bool bnd = yz_bnd || (gd.dirichlet && (gx == 0 || gx == gd.N[0] - 1));
        node[k][i] = bnd ? -1 : rowbase + gx;
      }
    }
  }
  // Invalid lanes (constrained node, columns past nvec, task past the tile)
  // skip the load and keep zero: the loaded registers are not read until the
  // first stage, so a prefetch (the persistent form) does not wait for them.
  // C = 2 needs nvec, ldx even and X 16-byte aligned (checked by the host).
  __device__ __forceinline__ void load_x(const double* __restrict__ X, int64_t ldx, int nvec, int v0,
                                         int tid) {
#pragma unroll
    for (int k = 0; k < R1; ++k) {
      const int w = tid + k * NT;
      const int v = v0 + (w % G) * C;
      const bool wok = w < T1 && v < nvec;
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        const bool ok = wok && node[k][i] >= 0;
        const int64_t at = (int64_t)node[k][i] * ldx + v;
        if constexpr (C == 1) {
          x[k][i] = 0.0;
          if (ok) x[k][i] = X[at];
        } else {
          x[2 * k][i] = 0.0;
          x[2 * k + 1][i] = 0.0;
          if (ok) {
            const double2 xv = *reinterpret_cast<const double2*>(X + at);
            x[2 * k][i] = xv.x;
            x[2 * k + 1][i] = xv.y;
          }
        }
      }
    }
  }
  // T = float: the column exponents (a max-reduction over the lanes of equal
  // column group, then over the wavefronts through `scratch`, NT / 64 * B
  // ints of LDS not otherwise in use before the next barrier) and the scaled
  // FP32 values.  Every thread of the workgroup must call it (one barrier).
  // NT is a multiple of G, so all tasks of a thread share its column group.
  __device__ __forceinline__ void scale(int* __restrict__ scratch, int tid) {
    static_assert(F32 && 64 % G == 0 && NT % G == 0, "G divides 64 and NT");
    constexpr int kNone = -100000;
    int e[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      double m = 0.0;
#pragma unroll
      for (int k = 0; k < R1; ++k)
#pragma unroll
        for (int i = 0; i < NP; ++i) m = fmax(m, fabs(x[k * C + c][i]));
      int em = kNone;
      if (m > 0.0) (void)frexp(m, &em);
#pragma unroll
      for (int off = G; off < 64; off *= 2) em = max(em, __shfl_xor(em, off));
      e[c] = em;
    }
    const int lane = tid & 63, wave = tid >> 6, g = tid % G;
    if (lane < G) {
#pragma unroll
      for (int c = 0; c < C; ++c) scratch[wave * B + g * C + c] = e[c];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < C; ++c) {
      int em = kNone;
#pragma unroll
      for (int w = 0; w < NT / 64; ++w) em = max(em, scratch[w * B + g * C + c]);
      ex[c] = em == kNone ? 0 : em;
#pragma unroll
      for (int k = 0; k < R1; ++k)
#pragma unroll
        for (int i = 0; i < NP; ++i) xs[k * C + c][i] = (T)ldexp(x[k * C + c][i], -ex[c]);
    }
  }
};

// P1: N along direction 0 from the gathered registers (consumed) -> A (NQ,NP,NP).
template <int NP, int NQ, int B, int C, int NT, typename T = double>
__device__ __forceinline__ void box_p1(T* __restrict__ bA, BoxGather<NP, B, C, NT, T>& Gt,
                                       int tid) {
  using GT = BoxGather<NP, B, C, NT, T>;
  constexpr int R1 = GT::R1, G = GT::G;
  T o[R1 * C][NQ];
  if constexpr (GT::F32)
    eo_matvec<MatN<NP, NQ>, NQ, NP, false, NP, R1 * C>(Gt.xs, o);
  else
    eo_matvec<MatN<NP, NQ>, NQ, NP, false, NP, R1 * C>(Gt.x, o);
#pragma unroll
  for (int k = 0; k < R1; ++k) {
    const int w = tid + k * NT;
    if (!GT::TK::live(k, w)) continue;
    const int g = w % G, pen = w / G;
#pragma unroll
    for (int a = 0; a < NQ; ++a) lds_put<C>(bA + (pen * NQ + a) * B + g * C, o, k * C, a);
  }
}

// P2 .. P6 (barrier-separated; starts after the barrier that follows P1).
// The directions of the last forward and the first backward stages are
// chosen so that each pencil owner applies every operator of its direction at
// once, one barrier fewer than a stage per operator:
//   P2  y: N                      A (NQ,NP,NP) -> B (NQ,NQ,NP)
//   P3  z: T = N t; U = vq o T + g2 Lf_2 T   B -> T in A, U in B (in place)
//   P4  x: U += g0 Lf_0 T                   A, B -> B (in place)
//   P5  y: U += g1 Lf_1 T, then N^T         A, B -> B (in place, y extent NP)
//   P6  z: N^T                              B -> B (in place, z extent NP)
// B keeps the (NQ,NQ,NQ) strides throughout, so the result is left in B at
// (q, j, k) -> q + NQ j + NQ^2 k (q < NQ; j, k < NP).  In-place stages are
// safe because every pencil of a stage has a single owner that reads it whole
// before writing it.
struct NoHook {
  __device__ void operator()() const {}
};
// `after_p3` runs once P3's results are behind a barrier (the persistent form
// issues the next item's loads there).
template <int NP, int NQ, int B, int C, int NT, typename T = double, class Hook = NoHook>
__device__ __forceinline__ void box_mid(T* __restrict__ bA, T* __restrict__ bB,
                                        const T* __restrict__ svq, T g0, T g1, T g2, int tid,
                                        Hook after_p3 = Hook()) {
  constexpr int NQ2 = NQ * NQ, G = B / C;
  using Nf = MatN<NP, NQ>;
  using Lf = MatL<NP, NQ>;
  using TK = Tasks<NQ2, G, NT>;
  constexpr int R = TK::R;

  // P2: N along direction 1.
  box_stage<Nf, false, NP, 1, NQ, NP, NP, NQ, B, C, NT, T>(bA, bB, tid);
  __syncthreads();

  // P3: direction-2 pencils (a, b): T = N along 2; U = vq o T + g2 Lf_2 T.
  // (eo_matvec folds its input in place: T is stored and the mass term taken
  // before Lf_2 consumes it.)
  {
    T in[R * C][NP], t[R * C][NQ], m[R * C][NQ], l[R * C][NQ];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int w = TK::clamp(tid + k * NT);
      const int g = w % G, pen = w / G;
#pragma unroll
      for (int i = 0; i < NP; ++i) lds_get<C>(bB + (pen + i * NQ2) * B + g * C, in, k * C, i);
    }
    eo_matvec<Nf, NQ, NP, false, NP, R * C>(in, t);
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int w = TK::clamp(tid + k * NT);
      const int g = w % G, pen = w / G;
      const bool live = TK::live(k, tid + k * NT);
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const T sv = svq[pen + q * NQ2];
#pragma unroll
        for (int c = 0; c < C; ++c) m[k * C + c][q] = sv * t[k * C + c][q];
        if (live) lds_put<C>(bA + (pen + q * NQ2) * B + g * C, t, k * C, q);
      }
    }
    eo_matvec<Lf, NQ, NQ, false, NQ, R * C>(t, l);
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int w = tid + k * NT;
      if (!TK::live(k, w)) continue;
      const int g = w % G, pen = w / G;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
#pragma unroll
        for (int c = 0; c < C; ++c) l[k * C + c][q] = fma(g2, l[k * C + c][q], m[k * C + c][q]);
        lds_put<C>(bB + (pen + q * NQ2) * B + g * C, l, k * C, q);
      }
    }
  }
  __syncthreads();
  after_p3();

  // P4: direction-0 pencils (b, c): U += g0 Lf_0 T.
  {
    T t[R * C][NQ], u[R * C][NQ], o[R * C][NQ];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int w = TK::clamp(tid + k * NT);
      const int g = w % G, pen = w / G;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        lds_get<C>(bA + (pen * NQ + q) * B + g * C, t, k * C, q);
        lds_get<C>(bB + (pen * NQ + q) * B + g * C, u, k * C, q);
      }
    }
    eo_matvec<Lf, NQ, NQ, false, NQ, R * C>(t, o);
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int w = tid + k * NT;
      if (!TK::live(k, w)) continue;
      const int g = w % G, pen = w / G;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
#pragma unroll
        for (int c = 0; c < C; ++c) o[k * C + c][q] = fma(g0, o[k * C + c][q], u[k * C + c][q]);
        lds_put<C>(bB + (pen * NQ + q) * B + g * C, o, k * C, q);
      }
    }
  }
  __syncthreads();

  // P5: direction-1 pencils (a, c): u = U + g1 Lf_1 T, then N^T along 1.
  {
    T t[R * C][NQ], u[R * C][NQ], o[R * C][NQ], v[R * C][NP];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int w = TK::clamp(tid + k * NT);
      const int g = w % G, pen = w / G;
      const int base = (pen / NQ) * NQ2 + (pen % NQ);
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        lds_get<C>(bA + (base + q * NQ) * B + g * C, t, k * C, q);
        lds_get<C>(bB + (base + q * NQ) * B + g * C, u, k * C, q);
      }
    }
    eo_matvec<Lf, NQ, NQ, false, NQ, R * C>(t, o);
#pragma unroll
    for (int r = 0; r < R * C; ++r)
#pragma unroll
      for (int q = 0; q < NQ; ++q) u[r][q] = fma(g1, o[r][q], u[r][q]);
    eo_matvec<Nf, NP, NQ, true, NP, R * C>(u, v);
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int w = tid + k * NT;
      if (!TK::live(k, w)) continue;
      const int g = w % G, pen = w / G;
      const int base = (pen / NQ) * NQ2 + (pen % NQ);
#pragma unroll
      for (int j = 0; j < NP; ++j) lds_put<C>(bB + (base + j * NQ) * B + g * C, v, k * C, j);
    }
  }
  __syncthreads();

  // P6: direction-2 pencils (a, j), a < NQ, j < NP: N^T along 2, in place.
  {
    using TK6 = Tasks<NQ * NP, G, NT>;
    constexpr int R6 = TK6::R;
    T u[R6 * C][NQ], v[R6 * C][NP];
#pragma unroll
    for (int k = 0; k < R6; ++k) {
      const int w = TK6::clamp(tid + k * NT);
      const int g = w % G, pen = w / G;  // pen = a + NQ j
#pragma unroll
      for (int c = 0; c < NQ; ++c) lds_get<C>(bB + (pen + c * NQ2) * B + g * C, u, k * C, c);
    }
    eo_matvec<Nf, NP, NQ, true, NP, R6 * C>(u, v);
#pragma unroll
    for (int k = 0; k < R6; ++k) {
      const int w = tid + k * NT;
      if (!TK6::live(k, w)) continue;
      const int g = w % G, pen = w / G;
#pragma unroll
      for (int i = 0; i < NP; ++i) lds_put<C>(bB + (pen + i * NQ2) * B + g * C, v, k * C, i);
    }
  }
  __syncthreads();
}

// P7: N^T along direction 0 and the assembly of this thread's pencils.
template <int NP, int NQ, int B, int C, int NT, bool ACCUM, typename T = double>
__device__ __forceinline__ void box_p8(const T* __restrict__ bB,
                                       const BoxGather<NP, B, C, NT, T>& Gt, double* __restrict__ Y,
                                       int64_t ldy, int nvec, int v0, int tid) {
  using GT = BoxGather<NP, B, C, NT, T>;
  constexpr int R1 = GT::R1, G = GT::G;
  T t[R1 * C][NQ], o[R1 * C][NP];
#pragma unroll
  for (int k = 0; k < R1; ++k) {
    const int w = GT::TK::clamp(tid + k * NT);
    const int g = w % G, pen = w / G;
    const int base = ((pen % NP) + NQ * (pen / NP)) * NQ;  // (j, k) in the NQ-strided layout
#pragma unroll
    for (int q = 0; q < NQ; ++q) lds_get<C>(bB + (base + q) * B + g * C, t, k * C, q);
  }
  eo_matvec<MatN<NP, NQ>, NP, NQ, true, NP, R1 * C>(t, o);
#pragma unroll
  for (int k = 0; k < R1; ++k) {
    const int w = tid + k * NT;
    const int g = w % G, pen = w / G, v = v0 + g * C;
    if (w >= GT::T1 || v >= nvec) continue;
    const int i2 = pen % NP, i3 = pen / NP;
    const bool inner_pen = i2 > 0 && i2 < NP - 1 && i3 > 0 && i3 < NP - 1;
    double sc[C];  // undoes the column scaling of FP32 cell arrays
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if constexpr (GT::F32) sc[c] = ldexp(1.0, Gt.ex[c]);
      else sc[c] = 1.0;
    }
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const int node = Gt.node[k][i];
      if (node < 0) continue;
      double* dst = Y + (int64_t)node * ldy + v;
      if (i > 0 && i < NP - 1 && inner_pen) {
        if constexpr (C == 1) {
          if (ACCUM) *dst += (double)o[k][i] * sc[0];
          else *dst = (double)o[k][i] * sc[0];
        } else {
          double2* d2 = reinterpret_cast<double2*>(dst);
          double2 val = make_double2((double)o[2 * k][i] * sc[0], (double)o[2 * k + 1][i] * sc[1]);
          if (ACCUM) {
            const double2 old = *d2;
            val.x += old.x;
            val.y += old.y;
          }
          *d2 = val;
        }
      } else {
#pragma unroll
        for (int c = 0; c < C; ++c) unsafeAtomicAdd(dst + c, (double)o[k * C + c][i] * sc[c]);
      }
    }
  }
}

// Persistent form of the item loop: the workgroup owns items it0, it0 + W,
// ... < end (cell = order[item / ntiles], columns (item % ntiles) B ..).  The
// X values (and scaled potential) of item i+1 are loaded into registers while
// item i runs its contractions, so the extraction latency hides behind
// arithmetic instead of idling the workgroup; node numbers are recomputed from
// the grid for the assembly rather than held through the contractions.
template <int NP, int NQ, int B, int C, int NT, bool ACCUM, typename T = double>
__device__ __forceinline__ void box_items(T* __restrict__ lds, const GridDesc& grid,
                                          const int32_t* __restrict__ order,
                                          const double* __restrict__ geo,
                                          const double* __restrict__ vq,
                                          const double* __restrict__ X, double* __restrict__ Y,
                                          int64_t ldx, int64_t ldy, int nvec, int ntiles,
                                          int64_t it, int64_t end, int64_t W) {
  static_assert(std::is_same<T, double>::value, "the persistent form is built for FP64 only");
  constexpr int NQ3 = NQ * NQ * NQ;
  constexpr int RV = (NQ3 + NT - 1) / NT;
  T* bA = lds;
  T* bB = bA + NQ3 * B;
  T* svq = bB + NQ3 * B;
  const int tid = threadIdx.x;
  if (it >= end) return;
  auto load_vq = [&](int64_t e, T (&r)[RV]) {
#pragma unroll
    for (int k = 0; k < RV; ++k) {
      const int i = tid + k * NT;
      r[k] = (T)vq[e * NQ3 + (i < NQ3 ? i : 0)];
    }
  };
  BoxGather<NP, B, C, NT, T> cur;
  T vqc[RV];
  {
    const int64_t e = order[it / ntiles];
    cur.load_grid(grid, e, tid);
    cur.load_x(X, ldx, nvec, (int)(it % ntiles) * B, tid);
    load_vq(e, vqc);
  }
  for (;;) {
    const int64_t e = order[it / ntiles];
    const int v0 = (int)(it % ntiles) * B;
    const T g0 = (T)geo[e * 6 + 0], g1 = (T)geo[e * 6 + 3], g2 = (T)geo[e * 6 + 5];
#pragma unroll
    for (int k = 0; k < RV; ++k)
      if (RV * NT == NQ3 || tid + k * NT < NQ3) svq[tid + k * NT] = vqc[k];
    box_p1<NP, NQ, B, C, NT, T>(bA, cur, tid);
    const int64_t nx = it + W;
    __syncthreads();
    // prefetch the next item into the registers P1 freed, once P3 is done: the
    // loads then overlap P4 .. P7, and their registers stay free through the
    // heavier stages before
    box_mid<NP, NQ, B, C, NT, T>(bA, bB, svq, g0, g1, g2, tid, [&]() {
      if (nx < end) {
        const int64_t en = order[nx / ntiles];
        cur.load_grid(grid, en, tid);
        cur.load_x(X, ldx, nvec, (int)(nx % ntiles) * B, tid);
        load_vq(en, vqc);
      }
    });
    {
      BoxGather<NP, B, C, NT, T> here;  // node numbers only (x unused)
      here.load_grid(grid, e, tid);
      box_p8<NP, NQ, B, C, NT, ACCUM, T>(bB, here, Y, ldy, nvec, v0, tid);
    }
    if (nx >= end) break;
    it = nx;
    // no barrier here: the next P1 writes A and svq, whose last readers (P5,
    // P3) are behind barriers; B is rewritten only after the barrier that
    // follows the next P1, when every thread has finished this P7.
  }
}

// One (cell e, columns v0 .. v0+B-1) work item.  `lds` holds
// box_lds_bytes_t<T>(NP, NQ, B) bytes; the caller synchronises the workgroup
// before reusing it for another item.
template <int NP, int NQ, int B, int C, int NT, bool ACCUM, typename T = double>
__device__ __forceinline__ void box_cell_tile(T* __restrict__ lds, const GridDesc& grid,
                                              const double* __restrict__ geo,
                                              const double* __restrict__ vq,
                                              const double* __restrict__ X, double* __restrict__ Y,
                                              int64_t ldx, int64_t ldy, int nvec, int64_t e,
                                              int v0) {
  constexpr int NQ3 = NQ * NQ * NQ;
  T* bA = lds;
  T* bB = bA + NQ3 * B;
  T* svq = bB + NQ3 * B;
  const int tid = threadIdx.x;
  BoxGather<NP, B, C, NT, T> Gt;
  Gt.load_grid(grid, e, tid);
  for (int i = tid; i < NQ3; i += NT) svq[i] = (T)vq[e * NQ3 + i];
  const T g0 = (T)geo[e * 6 + 0], g1 = (T)geo[e * 6 + 3], g2 = (T)geo[e * 6 + 5];
  Gt.load_x(X, ldx, nvec, v0, tid);
  if constexpr (std::is_same<T, float>::value)
    Gt.scale(reinterpret_cast<int*>(bB), tid);  // B is first written in P2
  box_p1<NP, NQ, B, C, NT, T>(bA, Gt, tid);
  __syncthreads();
  box_mid<NP, NQ, B, C, NT, T>(bA, bB, svq, g0, g1, g2, tid);
  box_p8<NP, NQ, B, C, NT, ACCUM, T>(bB, Gt, Y, ldy, nvec, v0, tid);
}

// ------------------------------------------------ Chebyshev filter step
// One step of the Chebyshev filter of subspace iteration (Alg. ChFSi) on the
// standard form of the generalised eigenproblem (eq. shep), fused into one
// pass:  Out := a D A (D Y) + b Y + c Xp,  D = M^{-1/2} (diagonal; 0 on
// constrained rows), A the operator.  The gather scales each row by D and
// loads Xp for the thread's cell-interior rows (its latency hides behind the
// contractions); the assembly writes
// a D (.) + b Y + c Xp on those rows (one contributor) and atomically
// adds a D (.) on face rows, which an initialisation kernel set to b Y + c Xp
// beforehand.  Out may be Xp (every element is read before it is written, by
// the same thread); Xp may be NULL (c ignored).
template <int NP, int NQ, int B, int NT>
__device__ __forceinline__ void box_cell_tile_cheb(double* __restrict__ lds, const GridDesc& grid,
                                                   const double* __restrict__ geo,
                                                   const double* __restrict__ vq,
                                                   const double* __restrict__ Y,
                                                   double* Out, int64_t ld, int nvec,
                                                   int64_t e, int v0, const ChebArgs& ca) {
  constexpr int C = 1, NQ3 = NQ * NQ * NQ;
  using GT = BoxGather<NP, B, C, NT>;
  constexpr int R1 = GT::R1, G = GT::G;
  double* bA = lds;
  double* bB = bA + NQ3 * B;
  double* svq = bB + NQ3 * B;
  const int tid = threadIdx.x;
  GT Gt;
  Gt.load_grid(grid, e, tid);
  for (int i = tid; i < NQ3; i += NT) svq[i] = vq[e * NQ3 + i];
  const double g0 = geo[e * 6 + 0], g1 = geo[e * 6 + 3], g2 = geo[e * 6 + 5];
  Gt.load_x(Y, ld, nvec, v0, tid);
#pragma unroll
  for (int k = 0; k < R1; ++k)
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const int node = Gt.node[k][i];
      Gt.x[k][i] *= node >= 0 ? ca.D[node] : 0.0;
    }
  box_p1<NP, NQ, B, C, NT>(bA, Gt, tid);
  // Xp of this thread's cell-interior rows, issued after P1 and first used in
  // the assembly, so that its latency hides behind the contractions
  double xp[R1][NP];
#pragma unroll
  for (int k = 0; k < R1; ++k) {
    const int w = tid + k * NT;
    const int pen = GT::TK::clamp(w) / G, v = v0 + w % G;
    const int i2 = pen % NP, i3 = pen / NP;
    const bool inner_pen = w < GT::T1 && v < nvec && i2 > 0 && i2 < NP - 1 && i3 > 0 &&
                           i3 < NP - 1;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const int node = Gt.node[k][i];
      const bool inner = inner_pen && i > 0 && i < NP - 1 && node >= 0;
      xp[k][i] = inner && ca.Xp ? ca.Xp[(int64_t)node * ld + v] : 0.0;
    }
  }
  __syncthreads();
  box_mid<NP, NQ, B, C, NT>(bA, bB, svq, g0, g1, g2, tid);
  // P7: N^T along direction 0, then the fused assembly.  D and Y of the
  // thread's rows are loaded again (cache hits: this workgroup gathered them)
  // before the stage's LDS reads, so their latency overlaps the stage instead
  // of delaying the stores (holding them in registers through the whole chain
  // would exceed the register budget of three workgroups per CU).
  double dn[R1][NP], yv[R1][NP];
#pragma unroll
  for (int k = 0; k < R1; ++k) {
    const int w = tid + k * NT;
    const int pen = GT::TK::clamp(w) / G, v = v0 + w % G;
    const int i2 = pen % NP, i3 = pen / NP;
    const bool inner_pen = w < GT::T1 && v < nvec && i2 > 0 && i2 < NP - 1 && i3 > 0 &&
                           i3 < NP - 1;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const int node = Gt.node[k][i];
      const bool inner = inner_pen && i > 0 && i < NP - 1 && node >= 0;
      dn[k][i] = node >= 0 ? ca.D[node] : 0.0;
      yv[k][i] = inner ? Y[(int64_t)node * ld + v] : 0.0;
    }
  }
  double t[R1][NQ], o[R1][NP];
#pragma unroll
  for (int k = 0; k < R1; ++k) {
    const int w = GT::TK::clamp(tid + k * NT);
    const int g = w % G, pen = w / G;
    const int base = ((pen % NP) + NQ * (pen / NP)) * NQ;
#pragma unroll
    for (int q = 0; q < NQ; ++q) lds_get<C>(bB + (base + q) * B + g, t, k, q);
  }
  eo_matvec<MatN<NP, NQ>, NP, NQ, true, NP, R1>(t, o);
#pragma unroll
  for (int k = 0; k < R1; ++k) {
    const int w = tid + k * NT;
    const int g = w % G, pen = w / G, v = v0 + g;
    if (w >= GT::T1 || v >= nvec) continue;
    const int i2 = pen % NP, i3 = pen / NP;
    const bool inner_pen = i2 > 0 && i2 < NP - 1 && i3 > 0 && i3 < NP - 1;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const int node = Gt.node[k][i];
      if (node < 0) continue;
      const int64_t at = (int64_t)node * ld + v;
      const double val = ca.a * dn[k][i] * o[k][i];
      if (i > 0 && i < NP - 1 && inner_pen)
        Out[at] = fma(ca.c, xp[k][i], fma(ca.b, yv[k][i], val));
      else
        unsafeAtomicAdd(Out + at, val);
    }
  }
}

}  // namespace mf
