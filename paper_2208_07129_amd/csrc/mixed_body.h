// Body of the mixed-precision fused apply for axis-aligned cells, as a device
// function over one (cell, column tile) work item, shared by the one-shot
// kernel (apply_mixed.hip) and the persistent batched kernel: the contractions run on
// the matrix cores in FP32 (v_mfma_f32_4x4x1f32) or with BF16 operands
// (v_mfma_f32_4x4x4bf16_1k), accumulating in FP32; X is read and Y is
// assembled in FP64.
//
// Same algebra and phase order as the FP64 box-cell kernel (Alg. 2 with a
// diagonal 3x3 factor, eq. helmholtz); see apply_box.hip.  Differences:
//  - Cell arrays in LDS are FP32 (half the bytes), so B = 16 columns fit.
//  - One pencil per lane on the matrix cores: the 4x4 block MFMAs form 16
//    independent 4x4 products per wavefront; with the lane's own pencil as the
//    B operand (column l%4 of block l/4) and rows 4g..4g+3 of the 1D matrix as
//    the A operand (row l%4 supplied by lane l), result register i of lane l is
//    output 4g+i of that lane's pencil.  The A operands are per-lane constants
//    held in registers for the whole kernel.
//  - Per-column scaling: for every (cell, column) the gathered FP64 values are
//    multiplied by 2^-e, e the exponent of their largest magnitude, before the
//    conversion, and the cell result by 2^e before the FP64 assembly; powers
//    of two make both steps exact, and the FP32/BF16 range then holds any
//    column whose per-cell spread fits it.
#pragma once

#include "mf_internal.h"
#include "sf_common.h"
#include "sf_tables.h"

namespace mf {
namespace mixed {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));

// Per-lane A operands of an NOUT x NIN matrix: a[r4][g][k] = M(4g + r4, k),
// zero for padded rows.  M(o, i) = src[o*LD + i], or src[i*LD + o] if TR.
template <int NOUT, int NIN>
struct ATable {
  static constexpr int G = (NOUT + 3) / 4;
  float a[4][G][NIN];
};
template <int NP, int NQ, int WHICH>  // 0: N (NQ x NP), 1: N^T (NP x NQ), 2: L (NQ x NQ)
struct ACoef {
  static constexpr int NOUT = WHICH == 1 ? NP : NQ;
  static constexpr int NIN = WHICH == 0 ? NP : NQ;
  static constexpr ATable<NOUT, NIN> make() {
    ATable<NOUT, NIN> t{};
    const auto& T = Tab<NP, NQ>::v;
    for (int r4 = 0; r4 < 4; ++r4)
      for (int g = 0; g < ATable<NOUT, NIN>::G; ++g)
        for (int k = 0; k < NIN; ++k) {
          const int o = 4 * g + r4;
          double v = 0.0;
          if (o < NOUT) {
            if (WHICH == 0) v = T.Nf[o * NP + k];
            if (WHICH == 1) v = T.Nf[k * NP + o];
            if (WHICH == 2) v = T.Lf[o * NQ + k];
          }
          t.a[r4][g][k] = (float)v;
        }
    return t;
  }
  static constexpr ATable<NOUT, NIN> value = make();
};

__device__ __forceinline__ short to_bf16(float f) {
  // round to nearest even (inputs are finite)
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

// Per-lane coefficient registers of one matrix, in the operand form of PREC.
template <int NOUT, int NIN, int PREC>
struct ARegs;
template <int NOUT, int NIN>
struct ARegs<NOUT, NIN, MF_FP32> {
  static constexpr int G = (NOUT + 3) / 4;
  float a[G][NIN];
  __device__ __forceinline__ void load(const ATable<NOUT, NIN>& t, int r4) {
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int k = 0; k < NIN; ++k) a[g][k] = t.a[r4][g][k];
  }
};
template <int NOUT, int NIN>
struct ARegs<NOUT, NIN, MF_BF16> {
  static constexpr int G = (NOUT + 3) / 4;
  static constexpr int KC = (NIN + 3) / 4;
  v4s a[G][KC];
  __device__ __forceinline__ void load(const ATable<NOUT, NIN>& t, int r4) {
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int c = 0; c < KC; ++c) {
        v4s v;
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = (4 * c + j < NIN) ? to_bf16(t.a[r4][g][4 * c + j]) : (short)0;
        a[g][c] = v;
      }
  }
};

// out[r][o] = sum_k M(o, k) in[r][k] for the R pencils of this lane, on the
// matrix cores.
template <int NOUT, int NIN, int R>
__device__ __forceinline__ void mfma_mv(const ARegs<NOUT, NIN, MF_FP32>& A,
                                        const float (&in)[R][NIN], float (&out)[R][NOUT]) {
  constexpr int G = (NOUT + 3) / 4;
  v4f acc[R][G];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int g = 0; g < G; ++g) acc[r][g] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k < NIN; ++k)
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int g = 0; g < G; ++g)
        acc[r][g] = __builtin_amdgcn_mfma_f32_4x4x1f32(A.a[g][k], in[r][k], acc[r][g], 0, 0, 0);
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int o = 0; o < NOUT; ++o) out[r][o] = acc[r][o / 4][o % 4];
}
template <int NOUT, int NIN, int R>
__device__ __forceinline__ void mfma_mv(const ARegs<NOUT, NIN, MF_BF16>& A,
                                        const float (&in)[R][NIN], float (&out)[R][NOUT]) {
  constexpr int G = (NOUT + 3) / 4, KC = (NIN + 3) / 4;
  v4s b[R][KC];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int c = 0; c < KC; ++c) {
      v4s v;
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j] = (4 * c + j < NIN) ? to_bf16(in[r][4 * c + j]) : (short)0;
      b[r][c] = v;
    }
  v4f acc[R][G];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int g = 0; g < G; ++g) acc[r][g] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int c = 0; c < KC; ++c)
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int g = 0; g < G; ++g)
        acc[r][g] = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(A.a[g][c], b[r][c], acc[r][g], 0, 0, 0);
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int o = 0; o < NOUT; ++o) out[r][o] = acc[r][o / 4][o % 4];
}

}  // namespace mixed

// One (cell e, columns v0 .. v0+B-1) work item in mixed precision.  `lds_d`
// holds mixed_lds_bytes(NP, NQ, B) bytes; the caller synchronises the
// workgroup before reusing it for another item.
template <int NP, int NQ, int B, int NT, bool ACCUM, int PREC>
__device__ __forceinline__ void mixed_cell_tile(double* __restrict__ lds_d,
                                                const int32_t* __restrict__ cmap,
                                                const double* __restrict__ geo,
                                                const double* __restrict__ vq,
                                                const double* __restrict__ X,
                                                double* __restrict__ Y, int64_t ldx, int64_t ldy,
                                                int nvec, int64_t e, int v0) {
  using namespace mixed;
  constexpr int NP2 = NP * NP, NP3 = NP * NP * NP, NQ2 = NQ * NQ, NQ3 = NQ * NQ * NQ;
  int64_t* sxo = reinterpret_cast<int64_t*>(lds_d);
  int64_t* syo = sxo + NP3;
  float* bA = reinterpret_cast<float*>(syo + NP3);
  float* bB = bA + NQ3 * B;
  float* svq = bB + NQ3 * B;
  int* sexp = reinterpret_cast<int*>(svq + NQ3);
  const int tid = threadIdx.x;
  const int r4 = tid & 3;

  ARegs<NQ, NP, PREC> aN;
  ARegs<NP, NQ, PREC> aNT;
  ARegs<NQ, NQ, PREC> aL;
  aN.load(ACoef<NP, NQ, 0>::value, r4);
  aNT.load(ACoef<NP, NQ, 1>::value, r4);
  aL.load(ACoef<NP, NQ, 2>::value, r4);

  for (int i = tid; i < NP3; i += NT) {
    const int node = cmap[e * NP3 + i];
    sxo[i] = node >= 0 ? (int64_t)node * ldx : -1;
    syo[i] = node >= 0 ? (int64_t)node * ldy : -1;
  }
  for (int i = tid; i < NQ3; i += NT) svq[i] = (float)vq[e * NQ3 + i];
  for (int i = tid; i < B; i += NT) sexp[i] = -1100;
  const float g0 = (float)geo[e * 6 + 0], g1 = (float)geo[e * 6 + 3], g2 = (float)geo[e * 6 + 5];
  __syncthreads();

  // P1a: gather in FP64 and find the exponent of each column's largest entry.
  constexpr int T1 = NP2 * B, R1 = (T1 + NT - 1) / NT;
  double xg[R1][NP];
#pragma unroll
  for (int k = 0; k < R1; ++k) {
    const int w = tid + k * NT;
    const int wc = w < T1 ? w : 0;  // clamped: addresses stay inside the tile
    const int b = wc % B, pen = wc / B, v = v0 + b;
    const bool wok = w < T1 && v < nvec;
    double m = 0.0;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const int64_t off = wok ? sxo[pen * NP + i] : -1;
      const bool ok = off >= 0;
      const double x = X[ok ? off + v : 0];
      xg[k][i] = ok ? x : 0.0;
      m = fmax(m, fabs(xg[k][i]));
    }
    if (wok && m > 0.0) atomicMax(&sexp[b], ilogb(m));
  }
  __syncthreads();
  // P1b: scale by 2^-(e+1) (exact), convert, N along direction 0 -> A (NQ,NP,NP).
  {
    float xs[R1][NP], o[R1][NQ];
#pragma unroll
    for (int k = 0; k < R1; ++k) {
      const int b = (tid + k * NT) % B;
      const int ex = sexp[b];
      const double s = ex > -1100 ? ldexp(1.0, -(ex + 1)) : 1.0;
#pragma unroll
      for (int i = 0; i < NP; ++i) xs[k][i] = (float)(xg[k][i] * s);
    }
    mfma_mv(aN, xs, o);
#pragma unroll
    for (int k = 0; k < R1; ++k) {
      const int w = tid + k * NT;
      if (w < T1) {
        const int b = w % B, pen = w / B;
#pragma unroll
        for (int a = 0; a < NQ; ++a) bA[(pen * NQ + a) * B + b] = o[k][a];
      }
    }
  }
  __syncthreads();

  // Generic contraction phase on FP32 LDS data.
  auto run = [&](auto tasks_tag, auto nin_tag, auto nout_tag, auto& A, auto load, auto post,
                 auto store) {
    constexpr int TASKS = decltype(tasks_tag)::value;
    constexpr int NIN = decltype(nin_tag)::value;
    constexpr int NOUT = decltype(nout_tag)::value;
    constexpr int R = (TASKS + NT - 1) / NT;
    float in[R][NIN], out[R][NOUT];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int w = tid + k * NT;
      if (w < TASKS) {
        load(w, in[k]);
      } else {
#pragma unroll
        for (int i = 0; i < NIN; ++i) in[k][i] = 0.f;
      }
    }
    mfma_mv(A, in, out);
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int w = tid + k * NT;
      if (w < TASKS) {
        post(w, out[k]);
        store(w, out[k]);
      }
    }
  };
  using IC = std::integral_constant<int, 0>;
  auto nothing = [](int, auto&) {};

  // P2: N along direction 1: A (NQ,NP,NP) -> B (NQ,NQ,NP).
  {
    using PI = Pencils<1, NQ, NP, NP>;
    using PO = Pencils<1, NQ, NQ, NP>;
    run(std::integral_constant<int, PI::COUNT * B>{}, std::integral_constant<int, NP>{},
        std::integral_constant<int, NQ>{}, aN,
        [&](int w, float (&r)[NP]) {
          const int b = w % B, base = PI::base(w / B);
#pragma unroll
          for (int i = 0; i < NP; ++i) r[i] = bA[(base + i * PI::STRIDE) * B + b];
        },
        nothing,
        [&](int w, float (&o)[NQ]) {
          const int b = w % B, base = PO::base(w / B);
#pragma unroll
          for (int a = 0; a < NQ; ++a) bB[(base + a * PO::STRIDE) * B + b] = o[a];
        });
  }
  __syncthreads();
  // P3: N along direction 2: B (NQ,NQ,NP) -> T in A (NQ,NQ,NQ).
  run(std::integral_constant<int, NQ2 * B>{}, std::integral_constant<int, NP>{},
      std::integral_constant<int, NQ>{}, aN,
      [&](int w, float (&r)[NP]) {
        const int b = w % B, pen = w / B;
#pragma unroll
        for (int i = 0; i < NP; ++i) r[i] = bB[(pen + i * NQ2) * B + b];
      },
      nothing,
      [&](int w, float (&o)[NQ]) {
        const int b = w % B, pen = w / B;
#pragma unroll
        for (int a = 0; a < NQ; ++a) bA[(pen + a * NQ2) * B + b] = o[a];
      });
  __syncthreads();
  // P4: B = g0 L_0 T.
  run(std::integral_constant<int, NQ2 * B>{}, std::integral_constant<int, NQ>{},
      std::integral_constant<int, NQ>{}, aL,
      [&](int w, float (&t)[NQ]) {
        const int b = w % B, pen = w / B;
#pragma unroll
        for (int k = 0; k < NQ; ++k) t[k] = bA[(pen * NQ + k) * B + b];
      },
      [&](int, float (&o)[NQ]) {
#pragma unroll
        for (int k = 0; k < NQ; ++k) o[k] *= g0;
      },
      [&](int w, float (&o)[NQ]) {
        const int b = w % B, pen = w / B;
#pragma unroll
        for (int k = 0; k < NQ; ++k) bB[(pen * NQ + k) * B + b] = o[k];
      });
  __syncthreads();
  // P5: B += g1 L_1 T.
  run(std::integral_constant<int, NQ2 * B>{}, std::integral_constant<int, NQ>{},
      std::integral_constant<int, NQ>{}, aL,
      [&](int w, float (&t)[NQ]) {
        const int b = w % B, pen = w / B;
        const int base = (pen / NQ) * NQ2 + (pen % NQ);
#pragma unroll
        for (int k = 0; k < NQ; ++k) t[k] = bA[(base + k * NQ) * B + b];
      },
      [&](int w, float (&o)[NQ]) {
        const int b = w % B, pen = w / B;
        const int base = (pen / NQ) * NQ2 + (pen % NQ);
#pragma unroll
        for (int k = 0; k < NQ; ++k) o[k] = fmaf(g1, o[k], bB[(base + k * NQ) * B + b]);
      },
      [&](int w, float (&o)[NQ]) {
        const int b = w % B, pen = w / B;
        const int base = (pen / NQ) * NQ2 + (pen % NQ);
#pragma unroll
        for (int k = 0; k < NQ; ++k) bB[(base + k * NQ) * B + b] = o[k];
      });
  __syncthreads();
  // P6: direction-2 pencils: u = vq o T + g2 L_2 T + B, then N^T along 2 into A
  // (in place, (NQ,NQ,NP)).
  {
    constexpr int TASKS = NQ2 * B, R = (TASKS + NT - 1) / NT;
    float t[R][NQ], l[R][NQ], o[R][NP];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int w = tid + k * NT;
      const int wc = w < TASKS ? w : 0;  // clamped: addresses stay inside the tile
      const int b = wc % B, pen = wc / B;
#pragma unroll
      for (int q = 0; q < NQ; ++q) t[k][q] = bA[(pen + q * NQ2) * B + b];
    }
    mfma_mv(aL, t, l);
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int w = tid + k * NT;
      const int wc = w < TASKS ? w : 0;
      const int b = wc % B, pen = wc / B;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const float bb = bB[(pen + q * NQ2) * B + b];
        const float vv = svq[pen + q * NQ2];
        t[k][q] = fmaf(vv, t[k][q], fmaf(g2, l[k][q], bb));
      }
    }
    mfma_mv(aNT, t, o);
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int w = tid + k * NT;
      if (w < TASKS) {
        const int b = w % B, pen = w / B;
#pragma unroll
        for (int i = 0; i < NP; ++i) bA[(pen + i * NQ2) * B + b] = o[k][i];
      }
    }
  }
  __syncthreads();
  // P7: N^T along direction 1: A (NQ,NQ,NP) -> B (NQ,NP,NP).
  {
    using PI = Pencils<1, NQ, NQ, NP>;
    using PO = Pencils<1, NQ, NP, NP>;
    run(std::integral_constant<int, PI::COUNT * B>{}, std::integral_constant<int, NQ>{},
        std::integral_constant<int, NP>{}, aNT,
        [&](int w, float (&t)[NQ]) {
          const int b = w % B, base = PI::base(w / B);
#pragma unroll
          for (int k = 0; k < NQ; ++k) t[k] = bA[(base + k * PI::STRIDE) * B + b];
        },
        nothing,
        [&](int w, float (&o)[NP]) {
          const int b = w % B, base = PO::base(w / B);
#pragma unroll
          for (int i = 0; i < NP; ++i) bB[(base + i * PO::STRIDE) * B + b] = o[i];
        });
  }
  __syncthreads();
  // P8: N^T along direction 0, unscale by 2^(e+1), FP64 assembly.
  run(std::integral_constant<int, NP2 * B>{}, std::integral_constant<int, NQ>{},
      std::integral_constant<int, NP>{}, aNT,
      [&](int w, float (&t)[NQ]) {
        const int b = w % B, pen = w / B;
#pragma unroll
        for (int k = 0; k < NQ; ++k) t[k] = bB[(pen * NQ + k) * B + b];
      },
      nothing,
      [&](int w, float (&o)[NP]) {
        const int b = w % B, pen = w / B, v = v0 + b;
        if (v >= nvec) return;
        const int ex = sexp[b];
        const double s = ex > -1100 ? ldexp(1.0, ex + 1) : 1.0;
        const int i2 = pen % NP, i3 = pen / NP;
        const bool inner_pen = i2 > 0 && i2 < NP - 1 && i3 > 0 && i3 < NP - 1;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
          const int64_t off = syo[pen * NP + i];
          if (off < 0) continue;
          double* dst = Y + off + v;
          const double val = (double)o[i] * s;
          if (i > 0 && i < NP - 1 && inner_pen) {
            if (ACCUM) *dst += val;
            else *dst = val;
          } else {
            unsafeAtomicAdd(dst, val);
          }
        }
      });
  (void)IC::value;
}

}  // namespace mf
