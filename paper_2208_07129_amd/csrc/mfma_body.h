// FP64 matrix-core body of the fused apply on axis-aligned (box) cells with
// N = p + 1 = q <= 8 points per direction.
//
// The stages are those of the vector body (box_body.h): N along x, y, z, then
// at the quadrature points U = det J (V + sigma) o T + sum_s g_s Lf_s T with
// Lf = Dtf^T Dtf (the two derivative stages of a direction collapsed, the 3x3
// factor being diagonal on a box cell), then N^T along y, z, x (Alg. 1 and
// Alg. 2 with eq. tc1-tc3).  Every 1D contraction runs on the matrix cores in
// even-odd form:
//
//   v_mfma_f64_4x4x4_4b computes four independent 4x4x4 products per
//   wavefront; A[b][i][k] sits in lane i + 4b + 16k, B[b][k][j] in lane
//   j + 4b + 16k and the result D[b][i][j] in lane j + 4b + 16i.
//
// So lane l holds "row" k = l >> 4 of column n = l & 15 in both the B operand
// and the result, and a result can be the next product's operand.  A column
// is one (pencil, matrix column) pair of the cell tile; a lane row holds a
// mirrored pair of the pencil's points (x_r, x_{N-1-r}) (the middle point
// twice for odd N), so the centrosymmetric 1D matrices split into a 4x4 even
// block acting on x_r + x_{N-1-r} and a 4x4 odd block acting on
// x_r - x_{N-1-r}: one contraction of 16 columns is two matrix-core products
// and four adds, folding stays inside the lane, and the result lands where the
// next contraction along the same direction reads it (P3 chains N and Lf, P5
// chains Lf and N^T without LDS).
//
// Cell tiles live in LDS as [point][column] (x fastest, 8 columns innermost):
// two buffers of 8 N^3 doubles and the N^3 scaled potential.  A stage's N^2
// pencils (u, w) (u the faster of the two directions across the stage) go to
// the wavefronts in groups of two pencils x 8 columns: wavefront (pair j, half
// h) owns the pencils (2j, w) and (2j+1, w) of the lines w = h, h+2, ...; for
// odd N one more wavefront owns (N-1, w) and (N-1, w+1) for w = 0, 2, ....
// Group k of a wavefront then sits 2k lines from group 0, a compile-time LDS
// distance, and every pencil has one owning lane set, so stages work in place.
//
// LDS banks: a half-wavefront read (two lane rows of two pencils, four 64-byte
// runs) is free of bank conflicts when the runs fall on the four quarters of
// the 64 banks, a 16-lane write when its two runs differ by an odd multiple of
// 64 bytes.  The lane rows hold the pairs in the order 0, 2, 1, 3, so the two
// rows of a half-wavefront are two points apart (2, 2N or 2N^2 points: 2 mod
// 4 for odd N), and the two pencils of a group one line or one u apart (odd
// point distance for odd N).
#pragma once

#include "mf_internal.h"
#include "sf_common.h"
#include "sf_tables.h"

namespace mf {

// Pair held by lane row k (rows beyond the used pairs take a used one; the
// first lane row of a pair is its owner).
template <int N>
constexpr int mfma_pair_of_row(int k) {
  constexpr int perm[4] = {0, 2, 1, 3};
  const int H = (N + 1) / 2;  // pairs, the middle point counted as one
  int p = perm[k];
  if (p >= H) p = H - 1;
  return p;
}
template <int N>
constexpr bool mfma_row_owner(int k) {
  for (int j = 0; j < k; ++j)
    if (mfma_pair_of_row<N>(j) == mfma_pair_of_row<N>(k)) return false;
  return true;
}

// 4x4 even and odd blocks of a centrosymmetric N x N matrix (EoMat of
// sf_common.h) in lane-row order.  The even input of the middle row is 2 x_mid
// (both reads of that row hit the same point), so the middle column carries
// half the coefficient; its odd input is 0.  A lane row that repeats a pair
// contributes nothing as an input (zero column) and reproduces the owner's
// output (the owner's row), so it stores exactly what its twin stores.
struct EoBlock4 {
  double e[4][4];
  double o[4][4];
};
template <class M, int N, bool TR>
constexpr EoBlock4 eo_block4() {
  using E = EoMat<M, N, N, TR, N>;
  static_assert(E::HO + E::MO <= 4, "at most 8 points per direction");
  EoBlock4 b{};
  for (int ko = 0; ko < 4; ++ko) {
    const int o = mfma_pair_of_row<N>(ko);
    for (int ki = 0; ki < 4; ++ki) {
      if (!mfma_row_owner<N>(ki)) continue;
      const int i = mfma_pair_of_row<N>(ki);
      const double c = E::e(o, i);
      b.e[ko][ki] = (E::MI && i == E::HI) ? 0.5 * c : c;
      if (o < E::HO && i < E::HI) b.o[ko][ki] = E::d(o, i);
    }
  }
  return b;
}
// The three matrices of the chain: N (interpolation), Lf (collapsed
// derivative), N^T.
template <int N>
struct MfmaCoef {
  EoBlock4 m[3];
};
template <int N>
constexpr MfmaCoef<N> mfma_coef() {
  return MfmaCoef<N>{{eo_block4<MatN<N, N>, N, false>(), eo_block4<MatL<N, N>, N, false>(),
                      eo_block4<MatN<N, N>, N, true>()}};
}
template <int N>
__constant__ MfmaCoef<N> kMfmaCoef = mfma_coef<N>();

// One even-odd contraction of the lane's mirrored pair (lo = x_r, hi =
// x_{N-1-r}; both the middle point on the middle row) with the lane's A values.
__device__ __forceinline__ void eo_mfma(double lo, double hi, double ae, double ao, double& ylo,
                                        double& yhi) {
  const double ev = __builtin_amdgcn_mfma_f64_4x4x4f64(ae, lo + hi, 0.0, 0, 0, 0);
  const double od = __builtin_amdgcn_mfma_f64_4x4x4f64(ao, lo - hi, 0.0, 0, 0, 0);
  ylo = ev + od;
  yhi = ev - od;
}

template <int N>
struct MfmaShape {
  static constexpr int UP = N / 2;             // u pairs (2j, 2j+1)
  static constexpr int SINGLE = N % 2;         // one wavefront for u = N-1 (odd N)
  static constexpr int W = 2 * UP + SINGLE;    // wavefronts
  static constexpr int NT = 64 * W;
  static constexpr int G = (N + 1) / 2;        // groups per wavefront (lines 2 apart)
};

// LDS of a work item: the scaled potential (N^3, padded to even), then the two
// cell buffers of 8 N^3 doubles.
template <int N>
constexpr int mfma_svq_len() {
  return (N * N * N + 1) / 2 * 2;
}
template <int N>
constexpr size_t mfma_lds_bytes() {
  return ((size_t)mfma_svq_len<N>() + 2 * (size_t)N * N * N * 8) * sizeof(double);
}
// Wavefronts per SIMD that the LDS allows (workgroups per CU times W / 4).
template <int N>
constexpr int mfma_waves_per_eu() {
  const int wg = (int)(kLdsMax / mfma_lds_bytes<N>());
  const int w = (wg * MfmaShape<N>::W + 3) / 4;
  return w < 1 ? 1 : (w > 8 ? 8 : w);
}

// Per-lane state.  Group k of the lane is the pencil (u, line(k)); lo / hi are
// the LDS offsets (doubles) of the lane's two points in group 0 for the three
// directions; group k adds 2 k kStep[DIR] (compile time), except the last
// group, whose own offsets lo_l / hi_l hold the stand-in line of the odd
// wavefront's second pencil.
template <int N>
struct MfmaLane {
  using S = MfmaShape<N>;
  static constexpr int B = 8;
  static constexpr int kStep[3] = {N * N * B, N * N * B, N * B};  // one line
  int col, u, pr, w0, dl;
  bool owner_row, pair, stand_last, last_ok;
  int lo[3], hi[3], lo_l[3], hi_l[3];
  __device__ MfmaLane(int tid) {
    const int l = tid & 63, wave = tid >> 6;
    const int k = l >> 4, pi = (l & 15) >> 3;
    col = l & 7;
    if (wave < 2 * S::UP) {  // pencils (2j + pi, h + 2 g)
      u = 2 * (wave >> 1) + pi;
      w0 = wave & 1;
      dl = 0;
    } else {                 // pencils (N-1, 2 g + pi)
      u = N - 1;
      w0 = 0;
      dl = pi;
    }
    constexpr int prs[4] = {mfma_pair_of_row<N>(0), mfma_pair_of_row<N>(1),
                            mfma_pair_of_row<N>(2), mfma_pair_of_row<N>(3)};
    constexpr bool own[4] = {mfma_row_owner<N>(0), mfma_row_owner<N>(1), mfma_row_owner<N>(2),
                             mfma_row_owner<N>(3)};
    pr = k == 0 ? prs[0] : k == 1 ? prs[1] : k == 2 ? prs[2] : prs[3];
    owner_row = k == 0 ? own[0] : k == 1 ? own[1] : k == 2 ? own[2] : own[3];
    pair = pr < N / 2;
    const int rh = N - 1 - pr;  // = pr on the middle row
    last_ok = w0 + 2 * (S::G - 1) < N;          // wave-uniform
    const int wl = w0 + 2 * (S::G - 1) + dl;    // line of the last group
    stand_last = wl >= N;                       // odd wavefront's missing second pencil
    const int wlast = stand_last ? wl - 1 : wl;
    const int w = w0 + dl;
    lo[0] = (N * u + pr + N * N * w) * B + col;  // x: pencil (y, z) = (u, w)
    hi[0] = (N * u + rh + N * N * w) * B + col;
    lo[1] = (u + N * pr + N * N * w) * B + col;  // y: pencil (x, z) = (u, w)
    hi[1] = (u + N * rh + N * N * w) * B + col;
    lo[2] = (u + N * w + N * N * pr) * B + col;  // z: pencil (x, y) = (u, w)
    hi[2] = (u + N * w + N * N * rh) * B + col;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      lo_l[d] = lo[d] + (wlast - w) * kStep[d];
      hi_l[d] = hi[d] + (wlast - w) * kStep[d];
    }
  }
  // group k exists for this wavefront (wave-uniform)
  __device__ __forceinline__ bool has(int k) const { return k < S::G - 1 || last_ok; }
  // line of group k of this lane
  __device__ __forceinline__ int line(int k) const {
    const int w = w0 + 2 * k + dl;
    return w < N ? w : w - 1;
  }
  // this lane's result of group k is stored (not a stand-in, not a repeated row)
  __device__ __forceinline__ bool stores(int k) const {
    return has(k) && owner_row && !(k == S::G - 1 && stand_last);
  }
  template <int DIR>
  __device__ __forceinline__ int off_lo(int k) const {
    return k == S::G - 1 ? lo_l[DIR] : lo[DIR] + 2 * k * kStep[DIR];
  }
  template <int DIR>
  __device__ __forceinline__ int off_hi(int k) const {
    return k == S::G - 1 ? hi_l[DIR] : hi[DIR] + 2 * k * kStep[DIR];
  }
};

// Read / write the lane's pair of every group of a stage along DIR.
template <int N, int DIR>
__device__ __forceinline__ void mfma_read(const double* __restrict__ buf, const MfmaLane<N>& L,
                                          double (&lo)[MfmaShape<N>::G],
                                          double (&hi)[MfmaShape<N>::G]) {
#pragma unroll
  for (int k = 0; k < MfmaShape<N>::G; ++k) {
    lo[k] = 0.0;
    hi[k] = 0.0;
    if (L.has(k)) {
      lo[k] = buf[L.template off_lo<DIR>(k)];
      hi[k] = buf[L.template off_hi<DIR>(k)];
    }
  }
}
template <int N, int DIR>
__device__ __forceinline__ void mfma_write(double* __restrict__ buf, const MfmaLane<N>& L,
                                           const double (&lo)[MfmaShape<N>::G],
                                           const double (&hi)[MfmaShape<N>::G]) {
#pragma unroll
  for (int k = 0; k < MfmaShape<N>::G; ++k) {
    if (L.has(k)) {
      buf[L.template off_lo<DIR>(k)] = lo[k];
      buf[L.template off_hi<DIR>(k)] = hi[k];
    }
  }
}

// One (cell e, columns v0 .. v0+7) work item of Y (+)= A X on the matrix
// cores.  `lds` holds mfma_lds_bytes<N>() bytes.
template <int N, bool ACCUM>
__device__ __forceinline__ void mfma_cell_tile(double* __restrict__ lds, const GridDesc& grid,
                                               const double* __restrict__ geo,
                                               const double* __restrict__ vq,
                                               const double* __restrict__ X, double* __restrict__ Y,
                                               int64_t ldx, int64_t ldy, int nvec, int e, int v0) {
  using S = MfmaShape<N>;
  constexpr int G = S::G, N3 = N * N * N, B = 8;
  double* svq = lds;
  double* bA = svq + mfma_svq_len<N>();
  double* bB = bA + N3 * B;
  const int tid = threadIdx.x;
  const MfmaLane<N> L(tid);
  // A operands: lane l holds block entry [l & 3][l >> 4] of each matrix
  const int ai = tid & 3, ak = (tid & 63) >> 4;
  const double nE = kMfmaCoef<N>.m[0].e[ai][ak], nO = kMfmaCoef<N>.m[0].o[ai][ak];
  const double lE = kMfmaCoef<N>.m[1].e[ai][ak], lO = kMfmaCoef<N>.m[1].o[ai][ak];
  const double tE = kMfmaCoef<N>.m[2].e[ai][ak], tO = kMfmaCoef<N>.m[2].o[ai][ak];

  // gather (Q, with C on X): x-pencil (y, z) = (u, line(k)); node numbers from
  // the structured grid (periodic wrap, -1 on the boundary of a zero-Dirichlet
  // mesh); stand-in lanes load their twins' values, columns past nvec zeros
  const int cx = e % grid.n[0], cy = (e / grid.n[0]) % grid.n[1], cz = e / (grid.n[0] * grid.n[1]);
  const int v = v0 + L.col;
  int gy = cy * grid.p + L.u;
  if (gy == grid.N[1]) gy = 0;
  int gxl = cx * grid.p + L.pr, gxh = cx * grid.p + N - 1 - L.pr;
  if (gxl == grid.N[0]) gxl = 0;
  if (gxh == grid.N[0]) gxh = 0;
  const bool dir = grid.dirichlet;
  const bool yb = dir && (gy == 0 || gy == grid.N[1] - 1);
  const bool xy_lo = yb || (dir && (gxl == 0 || gxl == grid.N[0] - 1));
  const bool xy_hi = yb || (dir && (gxh == 0 || gxh == grid.N[0] - 1));
  int nlo[G], nhi[G];
  double lo[G], hi[G];
#pragma unroll
  for (int k = 0; k < G; ++k) {
    int gz = cz * grid.p + L.line(k);
    if (gz == grid.N[2]) gz = 0;
    const bool zb = dir && (gz == 0 || gz == grid.N[2] - 1);
    const int base = grid.N[0] * (gy + grid.N[1] * gz);
    const bool skip = zb || v >= nvec || !L.has(k);
    nlo[k] = (xy_lo || skip) ? -1 : base + gxl;
    nhi[k] = (xy_hi || skip) ? -1 : base + gxh;
  }
#pragma unroll
  for (int k = 0; k < G; ++k) {
    lo[k] = nlo[k] >= 0 ? X[(int64_t)nlo[k] * ldx + v] : 0.0;
    hi[k] = nhi[k] >= 0 ? X[(int64_t)nhi[k] * ldx + v] : 0.0;
  }
  for (int i = tid; i < N3; i += S::NT) svq[i] = vq[(int64_t)e * N3 + i];
  const double g0 = geo[(int64_t)e * 6 + 0], g1 = geo[(int64_t)e * 6 + 3],
               g2 = geo[(int64_t)e * 6 + 5];

  // P1: N along x (from the gathered registers) -> A
  {
    double ylo[G], yhi[G];
#pragma unroll
    for (int k = 0; k < G; ++k) eo_mfma(lo[k], hi[k], nE, nO, ylo[k], yhi[k]);
    mfma_write<N, 0>(bA, L, ylo, yhi);
  }
  __syncthreads();
  // P2: N along y, A -> B
  {
    double ylo[G], yhi[G];
    mfma_read<N, 1>(bA, L, lo, hi);
#pragma unroll
    for (int k = 0; k < G; ++k) eo_mfma(lo[k], hi[k], nE, nO, ylo[k], yhi[k]);
    mfma_write<N, 1>(bB, L, ylo, yhi);
  }
  __syncthreads();
  // P3: z: T = N t -> A; U = vq o T + g2 Lf T -> B
  {
    double tlo[G], thi[G], llo[G], lhi[G];
    mfma_read<N, 2>(bB, L, lo, hi);
#pragma unroll
    for (int k = 0; k < G; ++k) {
      eo_mfma(lo[k], hi[k], nE, nO, tlo[k], thi[k]);
      eo_mfma(tlo[k], thi[k], lE, lO, llo[k], lhi[k]);
    }
    mfma_write<N, 2>(bA, L, tlo, thi);
#pragma unroll
    for (int k = 0; k < G; ++k) {
      if (L.has(k)) {
        // the potential at the lane's two points (LDS offset / 8 = point index)
        llo[k] = fma(g2, llo[k], svq[L.template off_lo<2>(k) / B] * tlo[k]);
        lhi[k] = fma(g2, lhi[k], svq[L.template off_hi<2>(k) / B] * thi[k]);
      }
    }
    mfma_write<N, 2>(bB, L, llo, lhi);
  }
  __syncthreads();
  // P4: x: U += g0 Lf T
  {
    double ulo[G], uhi[G], llo[G], lhi[G];
    mfma_read<N, 0>(bA, L, lo, hi);
    mfma_read<N, 0>(bB, L, ulo, uhi);
#pragma unroll
    for (int k = 0; k < G; ++k) {
      eo_mfma(lo[k], hi[k], lE, lO, llo[k], lhi[k]);
      ulo[k] = fma(g0, llo[k], ulo[k]);
      uhi[k] = fma(g0, lhi[k], uhi[k]);
    }
    mfma_write<N, 0>(bB, L, ulo, uhi);
  }
  __syncthreads();
  // P5: y: U += g1 Lf T, then N^T
  {
    double ulo[G], uhi[G], llo[G], lhi[G];
    mfma_read<N, 1>(bA, L, lo, hi);
    mfma_read<N, 1>(bB, L, ulo, uhi);
#pragma unroll
    for (int k = 0; k < G; ++k) {
      eo_mfma(lo[k], hi[k], lE, lO, llo[k], lhi[k]);
      ulo[k] = fma(g1, llo[k], ulo[k]);
      uhi[k] = fma(g1, lhi[k], uhi[k]);
      eo_mfma(ulo[k], uhi[k], tE, tO, llo[k], lhi[k]);
    }
    mfma_write<N, 1>(bB, L, llo, lhi);
  }
  __syncthreads();
  // P6: z: N^T, in place in B
  {
    double ylo[G], yhi[G];
    mfma_read<N, 2>(bB, L, lo, hi);
#pragma unroll
    for (int k = 0; k < G; ++k) eo_mfma(lo[k], hi[k], tE, tO, ylo[k], yhi[k]);
    mfma_write<N, 2>(bB, L, ylo, yhi);
  }
  __syncthreads();
  // P7: x: N^T, then the assembly (Q^T and the sum over cells): nodes interior
  // to the cell have one contributor (plain stores), the others FP64 atomics
  // (their rows were zeroed beforehand); stand-in lanes store nothing
  {
    double ylo[G], yhi[G];
    mfma_read<N, 0>(bB, L, lo, hi);
#pragma unroll
    for (int k = 0; k < G; ++k) eo_mfma(lo[k], hi[k], tE, tO, ylo[k], yhi[k]);
    const bool inner_u = L.u > 0 && L.u < N - 1 && L.pr > 0;
#pragma unroll
    for (int k = 0; k < G; ++k) {
      if (!L.stores(k)) continue;
      const int w = L.line(k);
      const bool inner = inner_u && w > 0 && w < N - 1;
      if (nlo[k] >= 0) {
        double* dst = Y + (int64_t)nlo[k] * ldy + v;
        if (inner) {
          if (ACCUM) *dst += ylo[k];
          else *dst = ylo[k];
        } else {
          unsafeAtomicAdd(dst, ylo[k]);
        }
      }
      if (L.pair && nhi[k] >= 0) {
        double* dst = Y + (int64_t)nhi[k] * ldy + v;
        if (inner) {
          if (ACCUM) *dst += yhi[k];
          else *dst = yhi[k];
        } else {
          unsafeAtomicAdd(dst, yhi[k]);
        }
      }
    }
  }
}

}  // namespace mf
