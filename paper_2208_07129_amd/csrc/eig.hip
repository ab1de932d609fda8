// Symmetric eigen-decomposition of k x k blocks with 64 < k <= 2048 (the
// orthogonalisation and Rayleigh-Ritz steps of Alg. ChFSi at block sizes of
// hundreds to a thousand vectors) by the two-sided block Jacobi method.
//
// The indices are cut into blocks of 32 (k padded to a multiple of 64 with
// decoupled zero rows and columns).  One sweep pairs every two blocks once
// (round-robin pairing of the nb blocks, nb - 1 rounds).  In a round, each of
// the nb/2 disjoint block pairs gets one cyclic Jacobi sweep over its 64
// indices (one workgroup, the 64 x 64 sub-block in LDS), whose accumulated
// rotation J_i (64 x 64, orthogonal) is then applied to the whole matrix,
// A := J^T A J with J = diag(J_i) in the pairs' index sets, and to the
// accumulated eigenvectors, V := V J: one workgroup per 64 x 64 piece of A
// (two small products each) or of V.  Every pair of indices is rotated at
// least once per sweep, so this is a cyclic Jacobi ordering and converges
// quadratically.  After each sweep the off-diagonal Frobenius norm is
// measured; once it is at most 1e-14 of the block's, a device flag stops the
// remaining launches (they return at once), so the host never waits.
#include <algorithm>

#include "mf_internal.h"

namespace mf {
namespace {

constexpr int kBj = 32, kBjPair = 2 * kBj, kBjThreads = 256, kBjLd = kBjPair + 1;
constexpr int kBjMaxK = 2048, kBjMaxSweeps = 40, kBjNormThreads = 1024;

struct BjState {  // at the start of the work array
  double nrm2;    // squared Frobenius norm of the block
  double off2;    // squared off-diagonal norm after the last sweep
  double done;    // 1 once off2 <= 1e-28 nrm2
  double sweeps;  // sweeps taken
};
constexpr int64_t kBjHead = 8;  // doubles reserved for BjState (keeps the arrays 64-byte aligned)

__host__ __device__ inline int bj_padded(int k) { return (k + kBjPair - 1) / kBjPair * kBjPair; }

// Pair t of round r of the round-robin pairing of n items (n even): position
// 0 holds item 0, position i > 0 item 1 + (i - 1 + r) mod (n - 1), and
// positions t and n - 1 - t meet.
__device__ inline void round_robin(int n, int r, int t, int& p, int& q) {
  const int m = n - 1, i1 = n - 1 - t;
  const int x0 = t == 0 ? 0 : 1 + (t - 1 + r) % m;
  const int x1 = 1 + (i1 - 1 + r) % m;
  p = x0 < x1 ? x0 : x1;
  q = x0 < x1 ? x1 : x0;
}

// Global index of position i (< 64) of the block pair (P, Q).
__device__ inline int pair_index(int P, int Q, int i) {
  return i < kBj ? P * kBj + i : Q * kBj + (i - kBj);
}

__global__ void bj_init_kernel(int k, int K, const double* __restrict__ A, int64_t lda,
                               double* __restrict__ Aw, double* __restrict__ Vw) {
  const int64_t total = (int64_t)K * K;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx / K), j = (int)(idx - (int64_t)i * K);
    Aw[idx] = (i < k && j < k) ? A[(int64_t)i * lda + j] : 0.0;
    Vw[idx] = i == j ? 1.0 : 0.0;
  }
}

// first = true: the block's norm and whether it is diagonal already;
// otherwise (after a sweep, unless done): one more sweep counted, and done
// when the off-diagonal norm is small enough.  One workgroup, fixed summation
// order.
__global__ void __launch_bounds__(kBjNormThreads)
bj_norm_kernel(int K, const double* __restrict__ Aw, BjState* st, int first) {
  if (!first && st->done != 0.0) return;
  __shared__ double ra[kBjNormThreads], ro[kBjNormThreads];
  const int t = threadIdx.x;
  double all = 0.0, off = 0.0;
  for (int i = 0; i < K; ++i)
    for (int j = t; j < K; j += kBjNormThreads) {
      const double x = Aw[(int64_t)i * K + j];
      all = fma(x, x, all);
      if (i != j) off = fma(x, x, off);
    }
  ra[t] = all;
  ro[t] = off;
  __syncthreads();
  for (int s = kBjNormThreads / 2; s > 0; s >>= 1) {
    if (t < s) {
      ra[t] += ra[t + s];
      ro[t] += ro[t + s];
    }
    __syncthreads();
  }
  if (t == 0) {
    if (first) {
      st->nrm2 = ra[0];
      st->sweeps = 0.0;
    } else {
      st->sweeps += 1.0;
    }
    st->off2 = ro[0];
    st->done = ro[0] <= 1e-28 * st->nrm2 ? 1.0 : 0.0;
  }
}

// One cyclic Jacobi sweep over the 64 indices of block pair blockIdx.x of
// round r; writes the accumulated rotation to J + 64^2 blockIdx.x (row-major,
// column j = the new basis vector j in the pair's old coordinates).
__global__ void __launch_bounds__(kBjThreads)
bj_pair_kernel(int K, int r, const double* __restrict__ Aw, double* __restrict__ J,
               const BjState* __restrict__ st) {
  if (st->done != 0.0) return;
  extern __shared__ double sh[];
  double* a = sh;                       // 64 x kBjLd
  double* v = sh + kBjPair * kBjLd;     // 64 x kBjLd
  __shared__ double cs_c[kBjPair / 2], cs_s[kBjPair / 2];
  __shared__ int pp[kBjPair / 2], pq[kBjPair / 2];
  const int t = threadIdx.x, nb = K / kBj;
  int P, Q;
  round_robin(nb, r, blockIdx.x, P, Q);
  for (int i = t; i < kBjPair * kBjPair; i += kBjThreads) {
    const int row = i / kBjPair, col = i % kBjPair;
    a[row * kBjLd + col] = Aw[(int64_t)pair_index(P, Q, row) * K + pair_index(P, Q, col)];
    v[row * kBjLd + col] = row == col ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int rr = 0; rr < kBjPair - 1; ++rr) {
    if (t < kBjPair / 2) {
      int p, q;
      round_robin(kBjPair, rr, t, p, q);
      double c = 1.0, s = 0.0;
      const double apq = a[p * kBjLd + q];
      if (fabs(apq) > 1e-300) {
        const double th = (a[q * kBjLd + q] - a[p * kBjLd + p]) / (2.0 * apq);
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
    for (int i = t; i < kBjPair / 2 * kBjPair; i += kBjThreads) {  // rows p, q
      const int pr = i / kBjPair, j = i % kBjPair;
      const int p = pp[pr], q = pq[pr];
      const double c = cs_c[pr], s = cs_s[pr];
      const double ap = a[p * kBjLd + j], aq = a[q * kBjLd + j];
      a[p * kBjLd + j] = c * ap - s * aq;
      a[q * kBjLd + j] = s * ap + c * aq;
    }
    __syncthreads();
    for (int i = t; i < kBjPair / 2 * kBjPair; i += kBjThreads) {  // columns p, q
      const int pr = i / kBjPair, j = i % kBjPair;
      const int p = pp[pr], q = pq[pr];
      const double c = cs_c[pr], s = cs_s[pr];
      const double ap = a[j * kBjLd + p], aq = a[j * kBjLd + q];
      a[j * kBjLd + p] = c * ap - s * aq;
      a[j * kBjLd + q] = s * ap + c * aq;
      const double vp = v[j * kBjLd + p], vq = v[j * kBjLd + q];
      v[j * kBjLd + p] = c * vp - s * vq;
      v[j * kBjLd + q] = s * vp + c * vq;
    }
    __syncthreads();
  }
  double* out = J + (int64_t)blockIdx.x * kBjPair * kBjPair;
  for (int i = t; i < kBjPair * kBjPair; i += kBjThreads)
    out[i] = v[(i / kBjPair) * kBjLd + i % kBjPair];
}

// The round's rotation applied to the matrix and to the eigenvectors.
// Workgroups [0, np^2): the piece of A in the rows of pair i and the columns
// of pair j, replaced by J_i^T piece J_j.  Workgroups [np^2, np^2 + np K/64):
// rows 64 rb .. 64 rb + 63 of V in the columns of pair j, replaced by
// piece J_j.  The pieces are disjoint, so the update is in place.
__global__ void __launch_bounds__(kBjThreads)
bj_update_kernel(int K, int r, double* __restrict__ Aw, double* __restrict__ Vw,
                 const double* __restrict__ J, const BjState* __restrict__ st) {
  if (st->done != 0.0) return;
  extern __shared__ double sh[];
  double* B = sh;                       // the piece (then J_i^T piece)
  double* Ji = sh + kBjPair * kBjLd;
  double* Jj = sh + 2 * kBjPair * kBjLd;
  const int t = threadIdx.x, nb = K / kBj, np = nb / 2;
  int wg = blockIdx.x;
  const bool on_a = wg < np * np;
  int i = 0, j, rb = 0;
  if (on_a) {
    i = wg / np;
    j = wg % np;
  } else {
    wg -= np * np;
    rb = wg / np;
    j = wg % np;
  }
  int Pj, Qj, Pi = 0, Qi = 0;
  round_robin(nb, r, j, Pj, Qj);
  if (on_a) round_robin(nb, r, i, Pi, Qi);
  const double* jj = J + (int64_t)j * kBjPair * kBjPair;
  const double* ji = J + (int64_t)i * kBjPair * kBjPair;
  double* base = on_a ? Aw : Vw;
  for (int e = t; e < kBjPair * kBjPair; e += kBjThreads) {
    const int row = e / kBjPair, col = e % kBjPair;
    const int grow = on_a ? pair_index(Pi, Qi, row) : rb * kBjPair + row;
    B[row * kBjLd + col] = base[(int64_t)grow * K + pair_index(Pj, Qj, col)];
    Jj[row * kBjLd + col] = jj[e];
    if (on_a) Ji[row * kBjLd + col] = ji[e];
  }
  __syncthreads();
  // thread (ty, tx): rows ty + 16 u, columns tx + 16 w of the 64 x 64 result
  const int ty = t / 16, tx = t % 16;
  double acc[4][4];
  if (on_a) {  // B := J_i^T B
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int w = 0; w < 4; ++w) acc[u][w] = 0.0;
    for (int b = 0; b < kBjPair; ++b) {
      double x[4], y[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) x[u] = Ji[b * kBjLd + ty + 16 * u];
#pragma unroll
      for (int w = 0; w < 4; ++w) y[w] = B[b * kBjLd + tx + 16 * w];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int w = 0; w < 4; ++w) acc[u][w] = fma(x[u], y[w], acc[u][w]);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int w = 0; w < 4; ++w) B[(ty + 16 * u) * kBjLd + tx + 16 * w] = acc[u][w];
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int w = 0; w < 4; ++w) acc[u][w] = 0.0;
  for (int b = 0; b < kBjPair; ++b) {  // B J_j
    double x[4], y[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) x[u] = B[(ty + 16 * u) * kBjLd + b];
#pragma unroll
    for (int w = 0; w < 4; ++w) y[w] = Jj[b * kBjLd + tx + 16 * w];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int w = 0; w < 4; ++w) acc[u][w] = fma(x[u], y[w], acc[u][w]);
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int row = ty + 16 * u;
    const int grow = on_a ? pair_index(Pi, Qi, row) : rb * kBjPair + row;
#pragma unroll
    for (int w = 0; w < 4; ++w)
      base[(int64_t)grow * K + pair_index(Pj, Qj, tx + 16 * w)] = acc[u][w];
  }
}

// Eigenvalues ascending by rank (ties by index), eigenvector columns moved to
// their rank and scaled by w^vpow.
__global__ void bj_output_kernel(int k, int K, const double* __restrict__ Aw,
                                 const double* __restrict__ Vw, double* __restrict__ w,
                                 double* __restrict__ V, int64_t ldv, double vpow) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  const double lj = Aw[(int64_t)j * K + j];
  int rank = 0;
  for (int i = 0; i < k; ++i) {
    const double li = Aw[(int64_t)i * K + i];
    rank += (li < lj) || (li == lj && i < j);
  }
  w[rank] = lj;
  const double f = (vpow != 0.0 && lj > 0.0) ? pow(lj, vpow) : 1.0;
  for (int i = 0; i < k; ++i) V[(int64_t)i * ldv + rank] = Vw[(int64_t)i * K + j] * f;
}

// status: 2 if vpow != 0 and some eigenvalue <= 0, else 0 converged / 1 not.
__global__ void bj_status_kernel(int k, int K, const double* __restrict__ Aw, double vpow,
                                 const BjState* __restrict__ st, int* __restrict__ status) {
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  if (vpow != 0.0)
    for (int j = threadIdx.x; j < k; j += blockDim.x)
      if (!(Aw[(int64_t)j * K + j] > 0.0)) atomicOr(&bad, 1);
  __syncthreads();
  if (threadIdx.x == 0) *status = bad ? 2 : (st->done != 0.0 ? 0 : 1);
}

}  // namespace

int eig_blocked_max_k() { return kBjMaxK; }

int64_t sym_eig_blocked_work(int k) {
  const int64_t K = bj_padded(k), np = K / kBjPair;
  return kBjHead + 2 * K * K + np * kBjPair * kBjPair;
}

hipError_t launch_sym_eig_blocked(int k, const double* A, int64_t lda, double* w, double* V,
                                  int64_t ldv, double vpow, int* status, double* work,
                                  hipStream_t s) {
  const int K = bj_padded(k), nb = K / kBj, np = nb / 2;
  BjState* st = reinterpret_cast<BjState*>(work);
  double* Aw = work + kBjHead;
  double* Vw = Aw + (int64_t)K * K;
  double* J = Vw + (int64_t)K * K;
  const size_t lds_pair = 2 * (size_t)kBjPair * kBjLd * sizeof(double);
  const size_t lds_upd = 3 * (size_t)kBjPair * kBjLd * sizeof(double);
  KernelFacts f;  // raise the dynamic LDS limits on this device
  hipError_t err = kernel_facts(reinterpret_cast<const void*>(bj_pair_kernel), kBjThreads, lds_pair, f);
  if (err == hipSuccess)
    err = kernel_facts(reinterpret_cast<const void*>(bj_update_kernel), kBjThreads, lds_upd, f);
  if (err != hipSuccess) return err;
  const int64_t total = (int64_t)K * K;
  const unsigned init_blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(bj_init_kernel, dim3(init_blocks), dim3(256), 0, s, k, K, A, lda, Aw, Vw);
  hipLaunchKernelGGL(bj_norm_kernel, dim3(1), dim3(kBjNormThreads), 0, s, K, Aw, st, 1);
  const unsigned upd_blocks = (unsigned)(np * np + (K / kBjPair) * np);
  for (int sweep = 0; sweep < kBjMaxSweeps; ++sweep) {
    for (int r = 0; r < nb - 1; ++r) {
      hipLaunchKernelGGL(bj_pair_kernel, dim3(np), dim3(kBjThreads), lds_pair, s, K, r, Aw, J, st);
      hipLaunchKernelGGL(bj_update_kernel, dim3(upd_blocks), dim3(kBjThreads), lds_upd, s, K, r, Aw,
                         Vw, J, st);
    }
    hipLaunchKernelGGL(bj_norm_kernel, dim3(1), dim3(kBjNormThreads), 0, s, K, Aw, st, 0);
  }
  hipLaunchKernelGGL(bj_output_kernel, dim3((k + 127) / 128), dim3(128), 0, s, k, K, Aw, Vw, w, V,
                     ldv, vpow);
  hipLaunchKernelGGL(bj_status_kernel, dim3(1), dim3(256), 0, s, k, K, Aw, vpow, st, status);
  return hipGetLastError();
}

}  // namespace mf
