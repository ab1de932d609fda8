// Kernels of the block-CG building blocks: the operator diagonal (Jacobi),
// column dot products, Y := aX + bY, the Jacobi scaling and the small SPD
// solve of the k x k block step.  The Gram blocks' partial products and the
// block updates are matrix-core kernels of their own (blas64.hip).
#include <cmath>

#include "mf_internal.h"
#include "sf_common.h"

namespace mf {
namespace {

// One workgroup per cell.  `tab` = [wN2 (nq x np) | a (np) | b (np) | c (np)]
// with wN2(q, i) = w_q N(q, i)^2, a(i) = sum_q w_q D(q, i)^2,
// b(i) = sum_q w_q N(q, i)^2, c(i) = sum_q w_q D(q, i) N(q, i).  For the
// affine cell the element-matrix diagonal is
//   sum_{s,t} G_st prod_d T_{st,d}(i_d) + sum_Q det J (V + sigma)_Q prod_d wN2(q_d, i_d)
// with T = a in the direction s = t, c in the directions s != t, b elsewhere.
__global__ void diag_kernel(GridDesc g, const double* __restrict__ geo,
                            const double* __restrict__ vq, const double* __restrict__ tab, int np,
                            int nq, double* __restrict__ diag) {
  extern __shared__ double sh[];
  const int nq3 = nq * nq * nq, np3 = np * np * np;
  const int tabn = nq * np + 3 * np;
  const int64_t e = blockIdx.x;
  double* svq = sh;
  double* st = sh + nq3;
  for (int i = threadIdx.x; i < nq3; i += blockDim.x) svq[i] = vq[e * nq3 + i];
  for (int i = threadIdx.x; i < tabn; i += blockDim.x) st[i] = tab[i];
  __syncthreads();
  const double* wN2 = st;
  const double* ta = st + nq * np;
  const double* tb = ta + np;
  const double* tc = tb + np;
  const double* G = geo + e * 6;  // (00, 01, 02, 11, 12, 22)
  const int ce = (int)e;
  const int cx = ce % g.n[0], cy = (ce / g.n[0]) % g.n[1], cz = ce / (g.n[0] * g.n[1]);
  for (int i = threadIdx.x; i < np3; i += blockDim.x) {
    const int i1 = i % np, i2 = (i / np) % np, i3 = i / (np * np);
    const int node = grid_node(g, cx, cy, cz, i1, i2, i3);
    if (node < 0) continue;
    const double a1 = ta[i1], a2 = ta[i2], a3 = ta[i3];
    const double b1 = tb[i1], b2 = tb[i2], b3 = tb[i3];
    const double c1 = tc[i1], c2 = tc[i2], c3 = tc[i3];
    double d = G[0] * a1 * b2 * b3 + G[3] * b1 * a2 * b3 + G[5] * b1 * b2 * a3 +
               2.0 * (G[1] * c1 * c2 * b3 + G[2] * c1 * b2 * c3 + G[4] * b1 * c2 * c3);
    double m = 0.0;
    for (int q3 = 0; q3 < nq; ++q3) {
      double m2 = 0.0;
      for (int q2 = 0; q2 < nq; ++q2) {
        double m1 = 0.0;
        const double* v = svq + nq * (q2 + nq * q3);
        for (int q1 = 0; q1 < nq; ++q1) m1 = fma(v[q1], wN2[q1 * np + i1], m1);
        m2 = fma(m1, wN2[q2 * np + i2], m2);
      }
      m = fma(m2, wN2[q3 * np + i3], m);
    }
    unsafeAtomicAdd(diag + node, d + m);
  }
}

// Constrained (zero-Dirichlet boundary) rows of the diagonal := 1.
__global__ void diag_constrained_kernel(GridDesc g, double* __restrict__ diag) {
  const int64_t total = (int64_t)g.N[0] * g.N[1] * g.N[2];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int gx = (int)(i % g.N[0]), gy = (int)((i / g.N[0]) % g.N[1]),
              gz = (int)(i / ((int64_t)g.N[0] * g.N[1]));
    if (gx == 0 || gx == g.N[0] - 1 || gy == 0 || gy == g.N[1] - 1 || gz == 0 || gz == g.N[2] - 1)
      diag[i] = 1.0;
  }
}

__global__ void fill_kernel(double* __restrict__ v, int64_t n, double x) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    v[i] = x;
}

// Column dot products out[j] = sum_i A[i, j] B[i, j]: rows in chunks of
// kDotRows per workgroup; RPB = max(1, 256 / k) rows in flight per pass,
// lanes over columns (coalesced), partial sums combined in LDS, one FP64
// atomic per column per workgroup.
constexpr int kDotRows = 2048;
__global__ void __launch_bounds__(256)
col_dots_kernel(int64_t n, int k, const double* __restrict__ A, int64_t lda,
                const double* __restrict__ B, int64_t ldb, double* __restrict__ out) {
  __shared__ double part[256];
  const int t = threadIdx.x;
  const int rpb = k < 256 ? 256 / k : 1;
  const int64_t r0 = (int64_t)blockIdx.x * kDotRows;
  const int64_t r1 = r0 + kDotRows < n ? r0 + kDotRows : n;
  for (int j0 = 0; j0 < k; j0 += 256) {
    const int j = j0 + (rpb > 1 ? t % k : t);
    const int rr = rpb > 1 ? t / k : 0;
    double acc = 0.0;
    if (j < k && rr < rpb)
      for (int64_t r = r0 + rr; r < r1; r += rpb) acc = fma(A[r * lda + j], B[r * ldb + j], acc);
    part[t] = acc;
    __syncthreads();
    if (rpb > 1) {
      if (t < k) {
        double s = 0.0;
        for (int m = 0; m < rpb; ++m) s += part[t + m * k];
        unsafeAtomicAdd(out + t, s);
      }
    } else if (j < k) {
      unsafeAtomicAdd(out + j, acc);
    }
    __syncthreads();
  }
}

// Gram block C = alpha A^T B + beta C in two stages: partial products of row
// chunks (blas64.hip) into work[b], then their sum into C here, in chunk order.
// The work array holds up to 512 chunks of at least 2048 rows.
constexpr int kGramRows = 2048, kGramMaxBlocks = 512;

// C[i / cols][i % cols] := alpha sum_b work[b len + i] + beta C[..] for the
// len = rows cols elements (beta = 0: C not read).  A workgroup takes 64
// consecutive elements; its eight wavefronts sum the chunks b = w, w + 8, ...
// (coalesced 512-byte rows of the partials), then wavefront 0 adds the eight
// sums in wavefront order: a fixed order, so the result does not depend on
// timing.  One thread per element summing all chunks left most CUs idle at
// k = 128 (64 workgroups).
constexpr int kRedThreads = 512, kRedElems = 64, kRedGroups = kRedThreads / kRedElems;
__global__ void __launch_bounds__(kRedThreads)
chunk_sum_kernel(int rows, int cols, int nb, const double* __restrict__ work, double alpha,
                 double beta, double* __restrict__ C, int ldc) {
  __shared__ double part[kRedThreads];
  const int64_t len = (int64_t)rows * cols;
  const int e = blockIdx.x * kRedElems + (threadIdx.x & (kRedElems - 1));
  const int g = threadIdx.x / kRedElems;
  double s = 0.0;
  if (e < len) {
    const double* w = work + e;
#pragma unroll 8
    for (int b = g; b < nb; b += kRedGroups) s += w[(int64_t)b * len];
  }
  part[threadIdx.x] = s;
  __syncthreads();
  if (g == 0 && e < len) {
    for (int h = 1; h < kRedGroups; ++h) s += part[h * kRedElems + threadIdx.x];
    double* c = C + (int64_t)(e / cols) * ldc + e % cols;
    *c = beta == 0.0 ? alpha * s : fma(beta, *c, alpha * s);
  }
}

// Y := a X + b Y (b = 0: Y is not read).
__global__ void axpby_kernel(int64_t n, int k, double a, const double* X, int64_t ldx, double b,
                             double* Y, int64_t ldy) {
  const int64_t total = n * k;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / k;
    const int j = (int)(i % k);
    const double x = a * X[r * ldx + j];
    Y[r * ldy + j] = b == 0.0 ? x : fma(b, Y[r * ldy + j], x);
  }
}

__global__ void jacobi_kernel(int64_t n, int k, const double* __restrict__ diag,
                              const double* R, int64_t ldr, double* Z, int64_t ldz) {
  const int64_t total = n * k;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / k;
    const int j = (int)(i % k);
    Z[r * ldz + j] = R[r * ldr + j] / diag[r];
  }
}

// X := G^{-1} S (G k x k SPD, S k x m).  One workgroup per panel of 64
// right-hand-side columns; each forms the lower Cholesky factor of G in LDS
// itself (packed storage, row r at r(r+1)/2) by the blocked right-looking
// method with blocks of kSpdBlock columns: one wavefront factors the diagonal
// block (its lanes in step, no workgroup barrier), one thread per row below
// solves that row's block of the panel, then all threads apply the rank-8
// update to the trailing triangle, the panel rows staged contiguously in LDS
// so a row's eight factors are two 32-byte reads (three barriers per block,
// against three per column for the unblocked method).  Then it runs the two
// triangular solves on its panel: 16 adjacent lanes own a column, split each
// row's dot product and combine it with lane shuffles, so a column needs no
// barrier (its lanes are in one wavefront).  The factorisation is repeated per
// panel rather than shared through global memory: it costs less than a second
// launch.
constexpr int kSpdMaxK = 128, kSpdThreads = 1024, kSpdPanel = 64, kSpdBlock = 8;
constexpr int kSpdLanes = kSpdThreads / kSpdPanel;  // lanes per right-hand side
// The panel is held column by column (a column's k values contiguous, so the 16
// lanes of one dot product read neighbouring words) with a column stride of
// 144 doubles (= 128 mod 256 bytes): two columns read by one half-wavefront
// fall on different halves of the banks.
constexpr int kSpdPS = kSpdMaxK + 16;
__device__ inline int tri(int r, int c) { return r * (r + 1) / 2 + c; }
__global__ void __launch_bounds__(kSpdThreads)
spd_solve_kernel(int k, int m, const double* __restrict__ G, const double* __restrict__ S,
                 double* __restrict__ X, int* __restrict__ status) {
  extern __shared__ double sh[];
  const int ntri = (k * (k + 1) / 2 + 1) / 2 * 2;    // 16-byte aligned sizes
  double* L = sh;                                   // k(k+1)/2
  double* Lc = L + ntri;                            // k x kSpdBlock: the current panel rows
  double* Dinv = Lc + kSpdMaxK * kSpdBlock;         // k: 1 / L(r, r)
  double* P = Dinv + kSpdMaxK;                      // kSpdPanel columns of kSpdPS
  __shared__ int bad;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, nwaves = kSpdThreads / 64;
  for (int r = wave; r < k; r += nwaves)
    for (int c = lane; c <= r; c += 64) L[tri(r, c)] = G[(int64_t)r * k + c];
  if (t == 0) bad = 0;
  __syncthreads();
  for (int cb = 0; cb < k; cb += kSpdBlock) {
    const int nb = k - cb < kSpdBlock ? k - cb : kSpdBlock;
    if (wave == 0) {  // the diagonal block, unblocked, lanes 0 .. nb-1 own its rows
      for (int j = 0; j < nb; ++j) {
        const double d = L[tri(cb + j, cb + j)];
        if (!(d > 0.0) || !isfinite(d)) {
          if (lane == 0) bad = cb + j + 1;
          break;  // uniform across the wavefront
        }
        const double sd = sqrt(d), id = 1.0 / sd;
        __builtin_amdgcn_wave_barrier();
        if (lane == j) {
          L[tri(cb + j, cb + j)] = sd;
          Dinv[cb + j] = id;
        }
        if (lane > j && lane < nb) L[tri(cb + lane, cb + j)] *= id;
        __builtin_amdgcn_wave_barrier();
        if (lane > j && lane < nb) {
          const double lj = L[tri(cb + lane, cb + j)];
          for (int i = j + 1; i <= lane; ++i)
            L[tri(cb + lane, cb + i)] -= lj * L[tri(cb + i, cb + j)];
        }
        __builtin_amdgcn_wave_barrier();
      }
    }
    __syncthreads();
    if (bad) break;
    // rows below the block: L(r, block) := L(r, block) D^{-T}, staged in Lc
    for (int r = cb + nb + t; r < k; r += kSpdThreads) {
      double v[kSpdBlock];
#pragma unroll
      for (int j = 0; j < kSpdBlock; ++j) {
        if (j >= nb) break;
        double a = L[tri(r, cb + j)];
        for (int i = 0; i < j; ++i) a -= v[i] * L[tri(cb + j, cb + i)];
        v[j] = a * Dinv[cb + j];
        L[tri(r, cb + j)] = v[j];
        Lc[r * kSpdBlock + j] = v[j];
      }
    }
    __syncthreads();
    // trailing update: L(r, s) -= sum_j L(r, cb + j) L(s, cb + j), s <= r, both past the block
    for (int r = cb + nb + wave; r < k; r += nwaves) {
      double lr[kSpdBlock];
#pragma unroll
      for (int j = 0; j < kSpdBlock; ++j) lr[j] = j < nb ? Lc[r * kSpdBlock + j] : 0.0;
      double* row = L + tri(r, 0);
      for (int s2 = cb + nb + lane; s2 <= r; s2 += 64) {
        double acc = row[s2];
#pragma unroll
        for (int j = 0; j < kSpdBlock; ++j) acc -= lr[j] * Lc[s2 * kSpdBlock + j];
        row[s2] = acc;
      }
    }
    __syncthreads();
  }
  if (t == 0 && blockIdx.x == 0) *status = bad;
  if (bad) return;
  const int q = t % kSpdLanes, jc = t / kSpdLanes;  // lane within the column, panel column
  const int j0 = blockIdx.x * kSpdPanel;
  const int w = m - j0 < kSpdPanel ? m - j0 : kSpdPanel;
  for (int r = wave; r < k; r += nwaves)
    P[lane * kSpdPS + r] = lane < w ? S[(int64_t)r * m + j0 + lane] : 0.0;
  __syncthreads();
  // L y = s (rows in order)
  for (int r = 0; r < k; ++r) {
    double acc = 0.0;
    const double* lrow = L + tri(r, 0);
    for (int c = q; c < r; c += kSpdLanes) acc = fma(lrow[c], P[jc * kSpdPS + c], acc);
#pragma unroll
    for (int off = 1; off < kSpdLanes; off *= 2) acc += __shfl_xor(acc, off);
    if (q == 0) P[jc * kSpdPS + r] = (P[jc * kSpdPS + r] - acc) * Dinv[r];
    __builtin_amdgcn_wave_barrier();
  }
  // L^T x = y (rows in reverse)
  for (int r = k - 1; r >= 0; --r) {
    double acc = 0.0;
    for (int c = r + 1 + q; c < k; c += kSpdLanes)
      acc = fma(L[tri(c, r)], P[jc * kSpdPS + c], acc);
#pragma unroll
    for (int off = 1; off < kSpdLanes; off *= 2) acc += __shfl_xor(acc, off);
    if (q == 0) P[jc * kSpdPS + r] = (P[jc * kSpdPS + r] - acc) * Dinv[r];
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  for (int r = wave; r < k; r += nwaves)
    if (lane < w) X[(int64_t)r * m + j0 + lane] = P[lane * kSpdPS + r];
}

// Symmetric eigen-decomposition of a k x k block (k <= kEigMaxK) by the
// cyclic Jacobi method, one workgroup: the block and the accumulated rotations
// in LDS; each round applies k/2 disjoint plane rotations (round-robin pairing,
// so every pair of indices meets once per sweep): the rotation angles of the
// round's pairs, then the row updates, then the column updates of the block
// and of the rotations, a barrier after each.  Sweeps until the off-diagonal
// Frobenius norm is below 1e-14 of the block's (at most kEigMaxSweeps).  The
// eigenvalues are sorted ascending by rank; with vpow != 0 the eigenvector
// columns are scaled by w_j^vpow (every w_j must then be positive).
constexpr int kEigMaxK = 64, kEigThreads = 256, kEigMaxSweeps = 40, kEigLd = kEigMaxK + 1;
__global__ void __launch_bounds__(kEigThreads)
sym_eig_kernel(int k, const double* __restrict__ A, int64_t lda, double* __restrict__ w,
               double* __restrict__ V, int64_t ldv, double vpow, int* __restrict__ status) {
  extern __shared__ double sh[];
  double* a = sh;                           // kk x kEigLd
  double* v = a + kEigMaxK * kEigLd;        // kk x kEigLd
  __shared__ double cs_c[kEigMaxK / 2], cs_s[kEigMaxK / 2], red[kEigThreads];
  __shared__ int pp[kEigMaxK / 2], pq[kEigMaxK / 2];
  __shared__ int done;
  const int t = threadIdx.x;
  const int kk = k + (k & 1);               // an odd k gets a decoupled padding index
  for (int i = t; i < kk * kk; i += kEigThreads) {
    const int r = i / kk, c = i % kk;
    a[r * kEigLd + c] = (r < k && c < k) ? A[(int64_t)r * lda + c] : 0.0;
    v[r * kEigLd + c] = r == c ? 1.0 : 0.0;
  }
  __syncthreads();
  double nrm = 0.0;
  for (int i = t; i < k * k; i += kEigThreads) {
    const double x = a[(i / k) * kEigLd + i % k];
    nrm += x * x;
  }
  red[t] = nrm;
  __syncthreads();
  for (int st = kEigThreads / 2; st > 0; st >>= 1) {
    if (t < st) red[t] += red[t + st];
    __syncthreads();
  }
  const double thresh = 1e-28 * red[0];
  __syncthreads();
  const int m = kk - 1, np2 = kk / 2;
  int sweeps = 0;
  if (t == 0) done = (kk < 2) ? 1 : 0;
  __syncthreads();
  while (!done && sweeps < kEigMaxSweeps) {
    for (int r = 0; r < m; ++r) {
      if (t < np2) {
        // circle method: position 0 holds index 0, position i the index 1 + (i - 1 + r) mod m
        const int i0 = t, i1 = kk - 1 - t;
        const int x0 = i0 == 0 ? 0 : 1 + (i0 - 1 + r) % m;
        const int x1 = 1 + (i1 - 1 + r) % m;
        const int p = x0 < x1 ? x0 : x1, q = x0 < x1 ? x1 : x0;
        double c = 1.0, s = 0.0;
        const double apq = a[p * kEigLd + q];
        if (q < k && fabs(apq) > 1e-300) {
          const double th = (a[q * kEigLd + q] - a[p * kEigLd + p]) / (2.0 * apq);
          const double at = fabs(th);
          const double tn = (th >= 0.0 ? 1.0 : -1.0) / (at + (at < 1e150 ? sqrt(th * th + 1.0) : at));
          c = 1.0 / sqrt(tn * tn + 1.0);
          s = tn * c;
        }
        pp[t] = p;
        pq[t] = q;
        cs_c[t] = c;
        cs_s[t] = s;
      }
      __syncthreads();
      for (int i = t; i < np2 * kk; i += kEigThreads) {  // rows p, q of every pair
        const int pr = i / kk, j = i % kk;
        const int p = pp[pr], q = pq[pr];
        const double c = cs_c[pr], s = cs_s[pr];
        const double ap = a[p * kEigLd + j], aq = a[q * kEigLd + j];
        a[p * kEigLd + j] = c * ap - s * aq;
        a[q * kEigLd + j] = s * ap + c * aq;
      }
      __syncthreads();
      for (int i = t; i < np2 * kk; i += kEigThreads) {  // columns p, q: block and rotations
        const int pr = i / kk, j = i % kk;
        const int p = pp[pr], q = pq[pr];
        const double c = cs_c[pr], s = cs_s[pr];
        const double ap = a[j * kEigLd + p], aq = a[j * kEigLd + q];
        a[j * kEigLd + p] = c * ap - s * aq;
        a[j * kEigLd + q] = s * ap + c * aq;
        const double vp = v[j * kEigLd + p], vq = v[j * kEigLd + q];
        v[j * kEigLd + p] = c * vp - s * vq;
        v[j * kEigLd + q] = s * vp + c * vq;
      }
      __syncthreads();
    }
    ++sweeps;
    double off = 0.0;
    for (int i = t; i < k * k; i += kEigThreads) {
      const int r = i / k, c = i % k;
      if (r != c) {
        const double x = a[r * kEigLd + c];
        off += x * x;
      }
    }
    red[t] = off;
    __syncthreads();
    for (int st = kEigThreads / 2; st > 0; st >>= 1) {
      if (t < st) red[t] += red[t + st];
      __syncthreads();
    }
    if (t == 0) done = red[0] <= thresh;
    __syncthreads();
  }
  // sort by rank (ties by index) and write w and the scaled eigenvectors
  int bad = 0;
  for (int j = t; j < k; j += kEigThreads) {
    const double lj = a[j * kEigLd + j];
    int rank = 0;
    for (int i = 0; i < k; ++i) {
      const double li = a[i * kEigLd + i];
      rank += (li < lj) || (li == lj && i < j);
    }
    w[rank] = lj;
    double f = 1.0;
    if (vpow != 0.0) {
      if (lj > 0.0) f = pow(lj, vpow);
      else bad = 1;
    }
    for (int i = 0; i < k; ++i) V[(int64_t)i * ldv + rank] = v[i * kEigLd + j] * f;
  }
  red[t] = bad;
  __syncthreads();
  if (t == 0) {
    int anybad = 0;
    for (int i = 0; i < kEigThreads; ++i) anybad |= red[i] != 0.0;
    *status = anybad ? 2 : (done ? 0 : 1);
  }
}

unsigned grid_for(int64_t total, int threads) {
  int64_t b = (total + threads - 1) / threads;
  if (b > 65536) b = 65536;
  return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

hipError_t launch_diagonal(const Operator& op, const double* d_tab, double* diag, hipStream_t s) {
  const int64_t nd = op.ndofs;
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(nd, 256)), dim3(256), 0, s, diag, nd, 0.0);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  const size_t lds = ((size_t)op.nq * op.nq * op.nq + (size_t)op.nq * op.np + 3 * op.np) * sizeof(double);
  hipLaunchKernelGGL(diag_kernel, dim3((unsigned)op.ncells), dim3(256), lds, s, op.grid, op.d_geo,
                     op.d_vq, d_tab, op.np, op.nq, diag);
  err = hipGetLastError();
  if (err != hipSuccess || !op.grid.dirichlet) return err;
  hipLaunchKernelGGL(diag_constrained_kernel, dim3(grid_for(nd, 256)), dim3(256), 0, s, op.grid,
                     diag);
  return hipGetLastError();
}

hipError_t launch_col_dots(int64_t n, int k, const double* A, int64_t lda, const double* B,
                           int64_t ldb, double* out, hipStream_t s) {
  hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(256), 0, s, out, (int64_t)k, 0.0);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess || n == 0) return err;
  const int64_t blocks = (n + kDotRows - 1) / kDotRows;
  hipLaunchKernelGGL(col_dots_kernel, dim3((unsigned)blocks), dim3(256), 0, s, n, k, A, lda, B, ldb,
                     out);
  return hipGetLastError();
}

hipError_t launch_gram_reduce(int k, int nb, const double* work, double alpha, double beta,
                              double* C, int ldc, hipStream_t s) {
  return launch_chunk_sum(k, k, nb, work, alpha, beta, C, ldc, s);
}

hipError_t launch_chunk_sum(int rows, int cols, int nb, const double* work, double alpha,
                            double beta, double* C, int ldc, hipStream_t s) {
  const int64_t len = (int64_t)rows * cols;
  hipLaunchKernelGGL(chunk_sum_kernel, dim3((unsigned)((len + kRedElems - 1) / kRedElems)),
                     dim3(kRedThreads), 0, s, rows, cols, nb, work, alpha, beta, C, ldc);
  return hipGetLastError();
}

int64_t gram_blocks(int64_t n) {
  int64_t nb = (n + kGramRows - 1) / kGramRows;
  if (nb > kGramMaxBlocks) nb = kGramMaxBlocks;
  return nb < 1 ? 1 : nb;
}

hipError_t launch_axpby(int64_t n, int k, double a, const double* X, int64_t ldx, double b,
                        double* Y, int64_t ldy, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(axpby_kernel, dim3(grid_for(n * k, 256)), dim3(256), 0, s, n, k, a, X, ldx, b,
                     Y, ldy);
  return hipGetLastError();
}

hipError_t launch_jacobi(int64_t n, int k, const double* diag, const double* R, int64_t ldr,
                         double* Z, int64_t ldz, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(jacobi_kernel, dim3(grid_for(n * k, 256)), dim3(256), 0, s, n, k, diag, R,
                     ldr, Z, ldz);
  return hipGetLastError();
}

int spd_max_k() { return kSpdMaxK; }
int eig_max_k() { return kEigMaxK; }

hipError_t launch_sym_eig(int k, const double* A, int64_t lda, double* w, double* V, int64_t ldv,
                          double vpow, int* status, hipStream_t s) {
  const size_t lds = 2 * (size_t)kEigMaxK * kEigLd * sizeof(double);
  hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void*>(sym_eig_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(sym_eig_kernel, dim3(1), dim3(kEigThreads), lds, s, k, A, lda, w, V, ldv, vpow,
                     status);
  return hipGetLastError();
}

hipError_t launch_spd_solve(int k, int m, const double* G, const double* S, double* X, int* status,
                            hipStream_t s) {
  const size_t lds = ((size_t)(k * (k + 1) / 2 + 1) / 2 * 2 + (size_t)kSpdMaxK * kSpdBlock +
                      (size_t)kSpdMaxK + (size_t)kSpdPS * kSpdPanel) * sizeof(double);
  if (lds > 64 * 1024) {
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void*>(spd_solve_kernel),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
  }
  const unsigned panels = (unsigned)((m + kSpdPanel - 1) / kSpdPanel);
  hipLaunchKernelGGL(spd_solve_kernel, dim3(panels), dim3(kSpdThreads), lds, s, k, m, G, S, X,
                     status);
  return hipGetLastError();
}

}  // namespace mf
