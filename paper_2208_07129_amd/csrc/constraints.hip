// Hanging-node constraints as locally dense products (Sec. 3.2.2): each set I
// holds the slave rows S_I, the master rows M_I (one coarse face) and the
// dense weights W_I.  C:   X_S := W_I X_M.   C^T:  Y_M += W_I^T Y_S, Y_S := 0.
//
// One workgroup per (set, 64-column tile, chunk of the set's slaves): lane =
// column, so every row access is one contiguous 512-byte segment of a
// dof-major multivector, and the weights are wave-uniform (one W_I row or
// column per wave step).  A set has up to (2p+1)^2 slaves, so the slave chunks
// give the launch several workgroups per set (a few hundred sets alone would
// leave most of the 256 CUs idle).  The work is bound by the bytes of the
// slave and master rows; W_I and re-read master rows come from the caches.
#include "mf_internal.h"

namespace mf {
namespace {

constexpr int kCT = 64;                       // columns per tile, one per lane
constexpr int kDistThreads = 256;             // 4 waves
constexpr int kCondThreads = 512;             // 8 waves
constexpr int kCondWaves = kCondThreads / kCT;
constexpr int kMaxMPerWave = 16;              // masters per wave in C^T
constexpr int kDistSlaves = 32;               // slaves per workgroup in C
constexpr int kCondSlaves = 32;               // slaves per workgroup in C^T
static_assert(kCondWaves * kMaxMPerWave >= (kMaxP + 1) * (kMaxP + 1), "masters of one face");

// C for slaves [chunk * kDistSlaves, ...) of set `set`, columns of tile `tile`.
__device__ __forceinline__ void distribute_item(const ConstraintSet* __restrict__ sets,
                                                const int32_t* __restrict__ idx,
                                                const double* __restrict__ W,
                                                double* __restrict__ X, int64_t ld, int nvec,
                                                double* __restrict__ xm, int64_t set, int tile,
                                                int chunk) {
  const ConstraintSet cs = sets[set];
  const int sb = chunk * kDistSlaves;
  if (sb >= cs.ns) return;  // uniform over the workgroup
  const int se = min(cs.ns, sb + kDistSlaves);
  const int tid = threadIdx.x, lane = tid % kCT;
  const int wave = __builtin_amdgcn_readfirstlane(tid / kCT);
  const int col = tile * kCT + lane;
  const bool ok = col < nvec;
  for (int m = wave; m < cs.nm; m += kDistThreads / kCT) {
    const int g = idx[cs.m0 + m];
    xm[m * kCT + lane] = (ok && g >= 0) ? X[(int64_t)g * ld + col] : 0.0;
  }
  __syncthreads();
  // W_I rows are wave-uniform: scalar loads, the LDS serves the master values
  for (int s = sb + wave; s < se; s += kDistThreads / kCT) {
    const double* w = W + cs.w0 + (int64_t)s * cs.nm;
    double acc = 0.0;
    for (int m = 0; m < cs.nm; ++m) acc = fma(w[m], xm[m * kCT + lane], acc);
    if (ok) X[(int64_t)idx[cs.s0 + s] * ld + col] = acc;
  }
}

__global__ void __launch_bounds__(kDistThreads)
distribute_kernel(const ConstraintSet* __restrict__ sets, const int32_t* __restrict__ idx,
                  const double* __restrict__ W, double* __restrict__ X, int64_t ld, int nvec) {
  extern __shared__ double xm[];  // nm x kCT master values
  distribute_item(sets, idx, W, X, ld, nvec, xm, blockIdx.x, blockIdx.y, blockIdx.z);
}

__global__ void __launch_bounds__(kCondThreads)
condense_kernel(const ConstraintSet* __restrict__ sets, const int32_t* __restrict__ idx,
                const double* __restrict__ W, double* __restrict__ Y, int64_t ld, int nvec) {
  __shared__ double ys[kCondSlaves * kCT];                      // staged slave values
  __shared__ double wl[kCondSlaves * (kMaxP + 1) * (kMaxP + 1)];  // the chunk's W_I rows
  const ConstraintSet cs = sets[blockIdx.x];
  const int sb = blockIdx.z * kCondSlaves;
  if (sb >= cs.ns) return;  // uniform over the workgroup
  const int cnt = min(kCondSlaves, cs.ns - sb);
  const int tid = threadIdx.x, lane = tid % kCT;
  const int wave = __builtin_amdgcn_readfirstlane(tid / kCT);
  const int col = blockIdx.y * kCT + lane;
  const bool ok = col < nvec;
  // each slave row belongs to exactly one set and one chunk: read it, then clear it
  for (int s = wave; s < cnt; s += kCondWaves) {
    double v = 0.0;
    if (ok) {
      const int64_t at = (int64_t)idx[cs.s0 + sb + s] * ld + col;
      v = Y[at];
      Y[at] = 0.0;
    }
    ys[s * kCT + lane] = v;
  }
  const double* wsrc = W + cs.w0 + (int64_t)sb * cs.nm;
  for (int i = tid; i < cnt * cs.nm; i += kCondThreads) wl[i] = wsrc[i];
  __syncthreads();
  double acc[kMaxMPerWave];
#pragma unroll
  for (int j = 0; j < kMaxMPerWave; ++j) acc[j] = 0.0;
  for (int s = 0; s < cnt; ++s) {
    const double v = ys[s * kCT + lane];
    const double* w = wl + s * cs.nm;
#pragma unroll
    for (int j = 0; j < kMaxMPerWave; ++j) {
      const int m = wave + kCondWaves * j;
      if (m < cs.nm) acc[j] = fma(w[m], v, acc[j]);
    }
  }
  if (!ok) return;
#pragma unroll
  for (int j = 0; j < kMaxMPerWave; ++j) {
    const int m = wave + kCondWaves * j;
    if (m < cs.nm) {
      const int g = idx[cs.m0 + m];
      // masters on a coarse edge belong to two sets, and every chunk adds its part
      if (g >= 0) unsafeAtomicAdd(Y + (int64_t)g * ld + col, acc[j]);
    }
  }
}

// kZeroRows rows per workgroup (a quarter per wavefront), one column per lane.
// The wavefront's row numbers are loaded together before any store, so their
// latency is paid once rather than once per row.
constexpr int kZeroRows = 32;
__device__ __forceinline__ void zero_rows_item(double* __restrict__ Y,
                                               const int32_t* __restrict__ rows, int64_t n,
                                               int ncols, int64_t ld, int64_t block) {
  constexpr int kPer = kZeroRows / 4;
  const int wave = threadIdx.x / kCT, lane = threadIdx.x % kCT;
  const int64_t i0 = block * kZeroRows + wave * kPer;
  int32_t r[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) r[k] = i0 + k < n ? rows[i0 + k] : -1;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    if (r[k] < 0) continue;
    double* row = Y + (int64_t)r[k] * ld;
    for (int c = lane; c < ncols; c += kCT) row[c] = 0.0;
  }
}

__global__ void __launch_bounds__(256)
zero_listed_kernel(double* __restrict__ Y, const int32_t* __restrict__ rows, int64_t n, int ncols,
                   int64_t ld) {
  zero_rows_item(Y, rows, n, ncols, ld, blockIdx.x);
}

}  // namespace

hipError_t launch_zero_listed_rows(double* Y, const int32_t* rows, int64_t n, int ncols, int64_t ld,
                                   hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_listed_kernel, dim3((unsigned)((n + kZeroRows - 1) / kZeroRows)),
                     dim3(256), 0, s, Y, rows, n, ncols, ld);
  return hipGetLastError();
}

hipError_t launch_constraints_distribute(const Operator& op, double* X, int nvec, int64_t ld,
                                         hipStream_t s) {
  if (op.nsets <= 0) return hipSuccess;
  if (op.max_masters > (kMaxP + 1) * (kMaxP + 1)) return hipErrorInvalidValue;
  const dim3 grid((unsigned)op.nsets, (unsigned)((nvec + kCT - 1) / kCT),
                  (unsigned)((op.max_slaves + kDistSlaves - 1) / kDistSlaves));
  const size_t lds = (size_t)op.max_masters * kCT * sizeof(double);
  hipLaunchKernelGGL(distribute_kernel, grid, dim3(kDistThreads), lds, s, op.d_sets, op.d_cidx,
                     op.d_cw, X, ld, nvec);
  return hipGetLastError();
}

hipError_t launch_constraints_condense(const Operator& op, double* Y, int nvec, int64_t ld,
                                       hipStream_t s) {
  if (op.nsets <= 0) return hipSuccess;
  if (op.max_masters > kCondWaves * kMaxMPerWave) return hipErrorInvalidValue;
  const dim3 grid((unsigned)op.nsets, (unsigned)((nvec + kCT - 1) / kCT),
                  (unsigned)((op.max_slaves + kCondSlaves - 1) / kCondSlaves));
  hipLaunchKernelGGL(condense_kernel, grid, dim3(kCondThreads), 0, s, op.d_sets, op.d_cidx,
                     op.d_cw, Y, ld, nvec);
  return hipGetLastError();
}

}  // namespace mf
