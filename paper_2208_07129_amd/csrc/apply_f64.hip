// FP64 fused matrix-free apply: extraction, the twelve 1D contraction stages of
// the sum-factorised cell operator, the quadrature-point scaling and the
// assembly, in one launch over (cell, vector tile) work items.
//
// Semantics per cell e and column beta (Alg. 2 with the factorisation of
// eq. helmholtz, weight-folded matrices of Sec. 3.2.4):
//   T   = (N x N x N) U_e                   three N stages (Alg. 1, eq. tc1-tc3)
//   T_s = Dt_s T, s = 0,1,2                 collocation derivatives (eq. DU)
//   S_s = sum_d G_sd T_d                    3x3 scaling (eq. sjacobian)
//   T   = (det J (V+sigma)) o T + sum_s Dt_s^T S_s     (eq. mjacobian)
//   V_e = (N x N x N)^T T                   three N^T stages
//   Y  += Q_e^T V_e                         assembly (Sec. 3.2.3), FP64 atomics
//
// Compiled once per polynomial degree (MF_P) so the instantiations build in
// parallel; q runs over p+1 .. p+3.
#include "mf_internal.h"
#include "sf_common.h"
#include "sf_tables.h"

#ifndef MF_P
#error "compile with -DMF_P=<degree>"
#endif

namespace mf {
namespace {

template <int NP, int NQ, int B>
__global__ void __launch_bounds__(kThreads)
apply_f64_kernel(const int32_t* __restrict__ cmap, const double* __restrict__ geo,
                 const double* __restrict__ vq, const double* __restrict__ X, double* __restrict__ Y,
                 int64_t ldx, int64_t ldy, int nvec, int ntiles, int64_t nitems, int64_t chunk) {
  constexpr int NT = kThreads;
  constexpr int NP3 = NP * NP * NP, NQ2 = NQ * NQ, NQ3 = NQ * NQ * NQ;
  using Nf = MatN<NP, NQ>;  // folded N1D, NQ x NP
  using Df = MatD<NP, NQ>;  // folded Dt, NQ x NQ
  extern __shared__ double lds[];
  const int64_t item = xcd_item(blockIdx.x, chunk);
  if (item >= nitems) return;
  const int64_t e = item / ntiles;
  const int v0 = (int)(item % ntiles) * B;

  double* bA = lds;
  double* bB = bA + NQ3 * B;
  double* bC = bB + NQ3 * B;
  double* svq = bC + NQ3 * B;
  int* smap = reinterpret_cast<int*>(svq + NQ3);
  const int tid = threadIdx.x;

  for (int i = tid; i < NP3; i += NT) smap[i] = cmap[e * NP3 + i];
  for (int i = tid; i < NQ3; i += NT) svq[i] = vq[e * NQ3 + i];
  const double g00 = geo[e * 6 + 0], g01 = geo[e * 6 + 1], g02 = geo[e * 6 + 2];
  const double g11 = geo[e * 6 + 3], g12 = geo[e * 6 + 4], g22 = geo[e * 6 + 5];
  __syncthreads();

  // Extraction fused with the first N stage (direction 0): (NP,NP,NP) -> A (NQ,NP,NP).
  for (int w = tid; w < NP * NP * B; w += NT) {
    const int b = w % B, pen = w / B, v = v0 + b;
    double r[NP], o[NQ];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const int node = smap[pen * NP + i];
      r[i] = (node >= 0 && v < nvec) ? X[(int64_t)node * ldx + v] : 0.0;
    }
    matvec<Nf, NQ, NP, false, NP>(r, o);
#pragma unroll
    for (int a = 0; a < NQ; ++a) bA[(pen * NQ + a) * B + b] = o[a];
  }
  __syncthreads();
  stage<Nf, 1, NQ, NP, NP, NQ, false, NP, B, NT>(bA, bB, tid);   // -> (NQ,NQ,NP)
  __syncthreads();
  stage<Nf, 2, NQ, NQ, NP, NQ, false, NP, B, NT>(bB, bA, tid);   // -> T (NQ,NQ,NQ)
  __syncthreads();
  // Derivatives along directions 0 and 1 (no barrier needed between them).
  stage<Df, 0, NQ, NQ, NQ, NQ, false, NQ, B, NT>(bA, bB, tid);   // T0 -> B
  stage<Df, 1, NQ, NQ, NQ, NQ, false, NQ, B, NT>(bA, bC, tid);   // T1 -> C
  __syncthreads();
  // Direction-2 pencils: derivative along 2, 3x3 scaling, mass term, and the
  // transposed derivative along 2.  Each pencil is owned by one thread, so the
  // in-place updates of A, B, C are race-free.
  for (int w = tid; w < NQ2 * B; w += NT) {
    const int b = w % B, pen = w / B;
    double t[NQ], t0[NQ], t1[NQ], t2[NQ], s2[NQ], o[NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
      t[k] = bA[(pen + k * NQ2) * B + b];
      t0[k] = bB[(pen + k * NQ2) * B + b];
      t1[k] = bC[(pen + k * NQ2) * B + b];
    }
    matvec<Df, NQ, NQ, false, NQ>(t, t2);
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
      const double s0 = g00 * t0[k] + g01 * t1[k] + g02 * t2[k];
      const double s1 = g01 * t0[k] + g11 * t1[k] + g12 * t2[k];
      s2[k] = g02 * t0[k] + g12 * t1[k] + g22 * t2[k];
      bB[(pen + k * NQ2) * B + b] = s0;
      bC[(pen + k * NQ2) * B + b] = s1;
      t[k] *= svq[pen + k * NQ2];
    }
    matvec<Df, NQ, NQ, true, NQ>(s2, o);
#pragma unroll
    for (int k = 0; k < NQ; ++k) bA[(pen + k * NQ2) * B + b] = t[k] + o[k];
  }
  __syncthreads();
  // A += Dt_1^T S1 (direction-1 pencils).
  for (int w = tid; w < NQ2 * B; w += NT) {
    const int b = w % B, pen = w / B;
    const int base = (pen / NQ) * NQ2 + (pen % NQ);
    double s[NQ], o[NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) s[k] = bC[(base + k * NQ) * B + b];
    matvec<Df, NQ, NQ, true, NQ>(s, o);
#pragma unroll
    for (int k = 0; k < NQ; ++k) bA[(base + k * NQ) * B + b] += o[k];
  }
  __syncthreads();
  // Direction-0 pencils: A + Dt_0^T S0, then the first N^T stage -> C (NP,NQ,NQ).
  for (int w = tid; w < NQ2 * B; w += NT) {
    const int b = w % B, pen = w / B;
    double s[NQ], t[NQ], o[NP];
#pragma unroll
    for (int k = 0; k < NQ; ++k) s[k] = bB[(pen * NQ + k) * B + b];
    matvec<Df, NQ, NQ, true, NQ>(s, t);
#pragma unroll
    for (int k = 0; k < NQ; ++k) t[k] += bA[(pen * NQ + k) * B + b];
    matvec<Nf, NP, NQ, true, NP>(t, o);
#pragma unroll
    for (int i = 0; i < NP; ++i) bC[(pen * NP + i) * B + b] = o[i];
  }
  __syncthreads();
  stage<Nf, 1, NP, NQ, NQ, NP, true, NP, B, NT>(bC, bA, tid);    // -> (NP,NP,NQ)
  __syncthreads();
  // Last N^T stage (direction 2) fused with the assembly.
  for (int w = tid; w < NP * NP * B; w += NT) {
    const int b = w % B, pen = w / B, v = v0 + b;
    double t[NQ], o[NP];
#pragma unroll
    for (int k = 0; k < NQ; ++k) t[k] = bA[(pen + k * NP * NP) * B + b];
    matvec<Nf, NP, NQ, true, NP>(t, o);
    if (v < nvec) {
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        const int node = smap[pen + i * NP * NP];
        if (node >= 0) unsafeAtomicAdd(Y + (int64_t)node * ldy + v, o[i]);
      }
    }
  }
}

template <int NP, int NQ, int B>
hipError_t launch_pqb(const ApplyLaunch& a, hipStream_t s) {
  const int ntiles = (a.nvec + B - 1) / B;
  const int64_t nitems = a.ncells * ntiles;
  const int64_t chunk = (nitems + kXcds - 1) / kXcds;
  constexpr size_t lds = f64_lds_bytes(NP, NQ, B);
  static_assert(lds <= kLdsBudget, "LDS budget");
  hipLaunchKernelGGL((apply_f64_kernel<NP, NQ, B>), dim3((unsigned)(chunk * kXcds)), dim3(kThreads),
                     lds, s, a.map, a.geo, a.vq, a.X, a.Y, a.ldx, a.ldy, a.nvec, ntiles, nitems,
                     chunk);
  return hipGetLastError();
}

template <int NP, int NQ, int B>
hipError_t try_tile(const ApplyLaunch& a, hipStream_t s, bool& done) {
  if constexpr (f64_tile_built(NP, NQ, B)) {
    if (a.vtile == B) {
      done = true;
      return launch_pqb<NP, NQ, B>(a, s);
    }
  }
  return hipSuccess;
}

template <int NP, int NQ>
hipError_t launch_pq(const ApplyLaunch& a, hipStream_t s) {
  bool done = false;
  hipError_t err = hipSuccess;
  if (!done) err = try_tile<NP, NQ, 1>(a, s, done);
  if (!done) err = try_tile<NP, NQ, 2>(a, s, done);
  if (!done) err = try_tile<NP, NQ, 4>(a, s, done);
  if (!done) err = try_tile<NP, NQ, 8>(a, s, done);
  if constexpr (f64_bdef(NP, NQ) >= 1)
    if (!done) err = try_tile<NP, NQ, f64_bdef(NP, NQ)>(a, s, done);
  return done ? err : hipErrorInvalidValue;
}

}  // namespace

template <>
hipError_t launch_apply_f64_p<MF_P>(const Operator& op, const ApplyLaunch& a, hipStream_t s) {
  switch (op.q - MF_P) {
    case 1: return launch_pq<MF_P + 1, MF_P + 1>(a, s);
    case 2: return launch_pq<MF_P + 1, MF_P + 2>(a, s);
    case 3:
      if constexpr (f64_bmax(MF_P + 1, MF_P + 3) >= 1) return launch_pq<MF_P + 1, MF_P + 3>(a, s);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mf
