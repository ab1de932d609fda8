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
// Only two cell buffers live in LDS (the general kernel needs three).  Inside
// a phase each thread owns R pencils and issues all their LDS reads before
// computing.  Nodes interior to the cell have exactly one contributor and are
// written with plain stores; nodes on cell faces, edges and corners use FP64
// atomics (their rows are zeroed beforehand).
#pragma once

#include "mf_internal.h"
#include "sf_common.h"
#include "sf_tables.h"

namespace mf {

// One phase: every (vector, pencil) task w in [0, TASKS), R = ceil(TASKS/NT)
// rounds per thread.  load(w, in) fills a round's inputs; comp(in, out) maps
// all R rounds at once (multi-right-hand-side contractions); store(w, out)
// writes a round.  All LDS reads of a phase are issued before any compute.
template <int TASKS, int NT>
struct Rounds {
  static constexpr int R = (TASKS + NT - 1) / NT;
  static constexpr bool EXACT = TASKS % NT == 0;
};
template <int TASKS, int NT, int NIN, int NOUT, class Load, class Comp, class Store>
__device__ __forceinline__ void phase(int tid, Load load, Comp comp, Store store) {
  constexpr int R = Rounds<TASKS, NT>::R;
  constexpr bool EXACT = Rounds<TASKS, NT>::EXACT;
  double in[R][NIN];
  double out[R][NOUT];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int w = tid + k * NT;
    if (EXACT || k < R - 1 || w < TASKS) {
      load(w, in[k]);
    } else {
#pragma unroll
      for (int i = 0; i < NIN; ++i) in[k][i] = 0.0;
    }
  }
  comp(in, out);
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int w = tid + k * NT;
    if (EXACT || k < R - 1 || w < TASKS) store(w, out[k]);
  }
}

// One (cell e, columns v0 .. v0+B-1) work item.  `lds` holds
// box_lds_bytes(NP, NQ, B) bytes; the caller synchronises the workgroup
// before reusing it for another item.
template <int NP, int NQ, int B, int NT, bool ACCUM>
__device__ __forceinline__ void box_cell_tile(double* __restrict__ lds,
                                              const int32_t* __restrict__ cmap,
                                              const double* __restrict__ geo,
                                              const double* __restrict__ vq,
                                              const double* __restrict__ X, double* __restrict__ Y,
                                              int64_t ldx, int64_t ldy, int nvec, int64_t e,
                                              int v0) {
  constexpr int NP2 = NP * NP, NP3 = NP * NP * NP, NQ2 = NQ * NQ, NQ3 = NQ * NQ * NQ;
  using Nf = MatN<NP, NQ>;
  using Lf = MatL<NP, NQ>;
  double* bA = lds;
  double* bB = bA + NQ3 * B;
  double* svq = bB + NQ3 * B;
  // per cell node: row offsets node*ldx and node*ldy, -1 for a constrained node
  int64_t* sxo = reinterpret_cast<int64_t*>(svq + NQ3);
  int64_t* syo = sxo + NP3;
  const int tid = threadIdx.x;

  for (int i = tid; i < NP3; i += NT) {
    const int node = cmap[e * NP3 + i];
    sxo[i] = node >= 0 ? (int64_t)node * ldx : -1;
    syo[i] = node >= 0 ? (int64_t)node * ldy : -1;
  }
  for (int i = tid; i < NQ3; i += NT) svq[i] = vq[e * NQ3 + i];
  const double g0 = geo[e * 6 + 0], g1 = geo[e * 6 + 3], g2 = geo[e * 6 + 5];
  __syncthreads();

  // P1: extraction fused with N along direction 0: (NP,NP,NP) -> A (NQ,NP,NP).
  phase<NP2 * B, NT, NP, NQ>(
      tid,
      [&](int w, double (&r)[NP]) {
        // branch-free: invalid lanes (constrained node, column past nvec) read
        // X[0] and select zero
        const int b = w % B, pen = w / B, v = v0 + b;
        const bool vok = v < nvec;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
          const int64_t off = sxo[pen * NP + i];
          const bool ok = vok && off >= 0;
          const double x = X[ok ? off + v : 0];
          r[i] = ok ? x : 0.0;
        }
      },
      [&](auto& r, auto& o) { matvec_multi<Nf, NQ, NP, false, NP>(r, o); },
      [&](int w, double (&o)[NQ]) {
        const int b = w % B, pen = w / B;
#pragma unroll
        for (int a = 0; a < NQ; ++a) bA[(pen * NQ + a) * B + b] = o[a];
      });
  __syncthreads();

  // P2, P3: N along directions 1 and 2 -> T in A (NQ,NQ,NQ).
  {
    using PI = Pencils<1, NQ, NP, NP>;
    using PO = Pencils<1, NQ, NQ, NP>;
    phase<PI::COUNT * B, NT, NP, NQ>(
        tid,
        [&](int w, double (&r)[NP]) {
          const int b = w % B, base = PI::base(w / B);
#pragma unroll
          for (int i = 0; i < NP; ++i) r[i] = bA[(base + i * PI::STRIDE) * B + b];
        },
        [&](auto& r, auto& o) { matvec_multi<Nf, NQ, NP, false, NP>(r, o); },
        [&](int w, double (&o)[NQ]) {
          const int b = w % B, base = PO::base(w / B);
#pragma unroll
          for (int a = 0; a < NQ; ++a) bB[(base + a * PO::STRIDE) * B + b] = o[a];
        });
  }
  __syncthreads();
  {
    using PI = Pencils<2, NQ, NQ, NP>;
    phase<PI::COUNT * B, NT, NP, NQ>(
        tid,
        [&](int w, double (&r)[NP]) {
          const int b = w % B, pen = w / B;
#pragma unroll
          for (int i = 0; i < NP; ++i) r[i] = bB[(pen + i * NQ2) * B + b];
        },
        [&](auto& r, auto& o) { matvec_multi<Nf, NQ, NP, false, NP>(r, o); },
        [&](int w, double (&o)[NQ]) {
          const int b = w % B, pen = w / B;
#pragma unroll
          for (int a = 0; a < NQ; ++a) bA[(pen + a * NQ2) * B + b] = o[a];
        });
  }
  __syncthreads();

  // P4: B = g0 Lf_0 T (direction-0 pencils).
  phase<NQ2 * B, NT, NQ, NQ>(
      tid,
      [&](int w, double (&t)[NQ]) {
        const int b = w % B, pen = w / B;
#pragma unroll
        for (int k = 0; k < NQ; ++k) t[k] = bA[(pen * NQ + k) * B + b];
      },
      [&](auto& t, auto& o) {
        matvec_multi<Lf, NQ, NQ, false, NQ>(t, o);
        for (auto& ok : o)
#pragma unroll
          for (int k = 0; k < NQ; ++k) ok[k] *= g0;
      },
      [&](int w, double (&o)[NQ]) {
        const int b = w % B, pen = w / B;
#pragma unroll
        for (int k = 0; k < NQ; ++k) bB[(pen * NQ + k) * B + b] = o[k];
      });
  __syncthreads();

  // P5: B += g1 Lf_1 T (direction-1 pencils).
  phase<NQ2 * B, NT, 2 * NQ, NQ>(
      tid,
      [&](int w, double (&t)[2 * NQ]) {
        const int b = w % B, pen = w / B;
        const int base = (pen / NQ) * NQ2 + (pen % NQ);
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
          t[k] = bA[(base + k * NQ) * B + b];
          t[NQ + k] = bB[(base + k * NQ) * B + b];
        }
      },
      [&](auto& t, auto& o) {
        constexpr int R = sizeof(t) / sizeof(t[0]);
        double u[R][NQ];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int k = 0; k < NQ; ++k) u[r][k] = t[r][k];
        matvec_multi<Lf, NQ, NQ, false, NQ>(u, o);
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int k = 0; k < NQ; ++k) o[r][k] = fma(g1, o[r][k], t[r][NQ + k]);
      },
      [&](int w, double (&o)[NQ]) {
        const int b = w % B, pen = w / B;
        const int base = (pen / NQ) * NQ2 + (pen % NQ);
#pragma unroll
        for (int k = 0; k < NQ; ++k) bB[(base + k * NQ) * B + b] = o[k];
      });
  __syncthreads();

  // P6: direction-2 pencils: u = vq o T + g2 Lf_2 T + B, then N^T along 2;
  // written into A in place as (NQ,NQ,NP) (each pencil has a single owner).
  phase<NQ2 * B, NT, 3 * NQ, NP>(
      tid,
      [&](int w, double (&t)[3 * NQ]) {
        const int b = w % B, pen = w / B;
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
          t[k] = bA[(pen + k * NQ2) * B + b];
          t[NQ + k] = bB[(pen + k * NQ2) * B + b];
          t[2 * NQ + k] = svq[pen + k * NQ2];
        }
      },
      [&](auto& t, auto& o) {
        constexpr int R = sizeof(t) / sizeof(t[0]);
        double u[R][NQ], l[R][NQ];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int k = 0; k < NQ; ++k) u[r][k] = t[r][k];
        matvec_multi<Lf, NQ, NQ, false, NQ>(u, l);
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int k = 0; k < NQ; ++k)
            u[r][k] = fma(t[r][2 * NQ + k], t[r][k], fma(g2, l[r][k], t[r][NQ + k]));
        matvec_multi<Nf, NP, NQ, true, NP>(u, o);
      },
      [&](int w, double (&o)[NP]) {
        const int b = w % B, pen = w / B;
#pragma unroll
        for (int i = 0; i < NP; ++i) bA[(pen + i * NQ2) * B + b] = o[i];
      });
  __syncthreads();

  // P7: N^T along direction 1: A (NQ,NQ,NP) -> B (NQ,NP,NP).
  {
    using PI = Pencils<1, NQ, NQ, NP>;
    using PO = Pencils<1, NQ, NP, NP>;
    phase<PI::COUNT * B, NT, NQ, NP>(
        tid,
        [&](int w, double (&t)[NQ]) {
          const int b = w % B, base = PI::base(w / B);
#pragma unroll
          for (int k = 0; k < NQ; ++k) t[k] = bA[(base + k * PI::STRIDE) * B + b];
        },
        [&](auto& t, auto& o) { matvec_multi<Nf, NP, NQ, true, NP>(t, o); },
        [&](int w, double (&o)[NP]) {
          const int b = w % B, base = PO::base(w / B);
#pragma unroll
          for (int i = 0; i < NP; ++i) bB[(base + i * PO::STRIDE) * B + b] = o[i];
        });
  }
  __syncthreads();

  // P8: N^T along direction 0 fused with the assembly.
  phase<NP2 * B, NT, NQ, NP>(
      tid,
      [&](int w, double (&t)[NQ]) {
        const int b = w % B, pen = w / B;
#pragma unroll
        for (int k = 0; k < NQ; ++k) t[k] = bB[(pen * NQ + k) * B + b];
      },
      [&](auto& t, auto& o) { matvec_multi<Nf, NP, NQ, true, NP>(t, o); },
      [&](int w, double (&o)[NP]) {
        const int b = w % B, pen = w / B, v = v0 + b;
        if (v >= nvec) return;
        const int i2 = pen % NP, i3 = pen / NP;
        const bool inner_pen = i2 > 0 && i2 < NP - 1 && i3 > 0 && i3 < NP - 1;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
          const int64_t off = syo[pen * NP + i];
          if (off < 0) continue;
          double* dst = Y + off + v;
          if (i > 0 && i < NP - 1 && inner_pen) {
            if (ACCUM) *dst += o[i];
            else *dst = o[i];
          } else {
            unsafeAtomicAdd(dst, o[i]);
          }
        }
      });
}

}  // namespace mf
