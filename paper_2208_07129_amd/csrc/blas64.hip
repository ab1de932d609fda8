// FP64 tall-skinny products of block CG on the matrix cores
// (v_mfma_f64_16x16x4f64): Gram blocks C = alpha A^T B + beta C of n x k
// multivectors (n >> k) and block updates Y = beta Y + alpha P M.
//
// Lane layout of v_mfma_f64_16x16x4f64 (one wavefront, D = A B + C with A
// 16 x 4, B 4 x 16): A[i][c] in lane i + 16 c, B[c][j] in lane j + 16 c, and
// D[i][j] in lane j + 16 (i mod 4), accumulator register i / 4.
#include <mutex>

#include "mf_internal.h"

namespace mf {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kGramThreads = 256;  // four wavefronts, each a 64 x 64 block of C
constexpr int kGramBlock = 128;    // C columns / rows per workgroup
constexpr int kGramAhead = 3;      // 4-row steps loaded ahead

__device__ __forceinline__ v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Partial Gram blocks: workgroup (b, t) sums the rows [b R, min(n, (b+1) R)) of
// A^T B into work[b][i k + j] for the 128 x 128 block t of C (i, j < k).
// Wave w covers rows 64 (w / 2) .. and columns 64 (w % 2) .. of the block as
// 4 x 4 tiles of 16 x 16.  TWO: two Gram blocks with the same left operand,
// A^T B into work and A^T B2 into work2, by eight wavefronts (the last four on
// B2): each row of A is fetched from HBM once for both, the second wavefront
// that reads it finding it in the caches.
template <bool TWO>
__global__ void __launch_bounds__(TWO ? 2 * kGramThreads : kGramThreads)
gram_partial_kernel(int64_t n, int k, const double* __restrict__ A, int64_t lda,
                    const double* __restrict__ B1, int64_t ldb1, const double* __restrict__ B2,
                    int64_t ldb2, int64_t rows, double* __restrict__ work1,
                    double* __restrict__ work2) {
  const int lane = threadIdx.x & 63, wave = (threadIdx.x >> 6) & 3;
  const bool second = TWO && threadIdx.x >= kGramThreads;
  const double* __restrict__ B = second ? B2 : B1;
  const int64_t ldb = second ? ldb2 : ldb1;
  double* __restrict__ work = second ? work2 : work1;
  const int nbj = (k + kGramBlock - 1) / kGramBlock;
  const int bi = blockIdx.y / nbj, bj = blockIdx.y % nbj;
  const int i0 = bi * kGramBlock + (wave >> 1) * 64, j0 = bj * kGramBlock + (wave & 1) * 64;
  const int64_t r0 = (int64_t)blockIdx.x * rows;
  int64_t r1 = r0 + rows;
  if (r1 > n) r1 = n;
  const int c = lane >> 4, m = lane & 15;
  v4d acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
  bool ia[4], jb[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    ia[t] = i0 + 16 * t + m < k;
    jb[t] = j0 + 16 * t + m < k;
  }
  const double* pa = A + i0 + m;
  const double* pb = B + j0 + m;
  // operands of the 4-row step at rb (this lane's row rb + c), loaded one step
  // ahead of the products
  auto load = [&](int64_t rb, double (&a)[4], double (&b)[4]) {
    const int64_t r = rb + c;
    const bool rok = r < r1;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      a[t] = (rok && ia[t]) ? pa[r * lda + 16 * t] : 0.0;
      b[t] = (rok && jb[t]) ? pb[r * ldb + 16 * t] : 0.0;
    }
  };
  // a ring of kGramAhead steps in flight, so that HBM latency hides behind the
  // products of the steps before
  double a[kGramAhead][4], b[kGramAhead][4];
#pragma unroll
  for (int d = 0; d < kGramAhead; ++d) load(r0 + 4 * d, a[d], b[d]);
  for (int64_t rb = r0; rb < r1; rb += 4 * kGramAhead) {
#pragma unroll
    for (int d = 0; d < kGramAhead; ++d) {
#pragma unroll
      for (int ta = 0; ta < 4; ++ta)
#pragma unroll
        for (int tb = 0; tb < 4; ++tb) acc[ta][tb] = mfma16(a[d][ta], b[d][tb], acc[ta][tb]);
      load(rb + 4 * (d + kGramAhead), a[d], b[d]);
    }
  }
  double* out = work + (int64_t)blockIdx.x * k * k;
#pragma unroll
  for (int ta = 0; ta < 4; ++ta)
#pragma unroll
    for (int tb = 0; tb < 4; ++tb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = i0 + 16 * ta + 4 * q + c, j = j0 + 16 * tb + m;
        if (i < k && j < k) out[(int64_t)i * k + j] = acc[ta][tb][q];
      }
}

// Y := beta Y + alpha P M for n x kp P (ldp), kp x k M (ldm), n x k Y (ldy),
// M small enough for LDS.  M is staged once per workgroup in LDS, rows padded
// to a multiple of 16 doubles that is 16 mod 32 (two rows of a
// half-wavefront's fragment then fall on different halves of the 64 banks).
// Each of the 8 wavefronts takes strips of 16 rows of Y and all k columns (up
// to 8 tiles of 16): the strip's P values (up to 128 columns at a time, 32
// per lane) and its old Y values are loaded into registers before the
// products, so their latency hides behind the strip's matrix-core products;
// the B operand comes from LDS.
__host__ __device__ constexpr int update_ld(int k) {
  const int kp16 = (k + 15) / 16 * 16;
  return kp16 % 32 == 16 ? kp16 : kp16 + 16;
}
constexpr int kUpdThreads = 512, kUpdTiles = 8, kUpdLds = 20480, kUpdChunk = 128;
constexpr int kUpdRowsPerWg = 1024;
// KT column tiles of 16 (k <= 16 KT).  Loads never branch: row and column
// indices are clamped into the operands and the values outside them replaced
// by zero, so the whole strip is one basic block the compiler can schedule.
// M rows kp .. kp4 - 1 (kp4 = kp rounded up to 4) are zero in LDS.  EXACT:
// k = 16 KT, so the output columns are fixed offsets from one row pointer.
// NORMS: also the squared norms of the new Y's columns over the workgroup's
// rows, into npart[blockIdx.x k + j] (each lane sums its rows, then the four
// lanes of a column, then the eight wavefronts in order).
template <int KT, bool EXACT, bool NORMS>
__global__ void __launch_bounds__(kUpdThreads)
update_kernel(int64_t n, int k, int kp, double alpha, const double* __restrict__ P, int64_t ldp,
              const double* __restrict__ M, int ldm, double beta, double* __restrict__ Y,
              int64_t ldy, double* __restrict__ npart) {
  extern __shared__ double mlds[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int ldl = update_ld(16 * KT);
  const int kp4 = (kp + 3) & ~3;
  for (int i = threadIdx.x; i < kp4 * ldl; i += kUpdThreads) {
    const int r = i / ldl, c = i - r * ldl;
    mlds[i] = (c < k && r < kp) ? M[(int64_t)r * ldm + c] : 0.0;
  }
  __syncthreads();
  const int c = lane >> 4, m = lane & 15;
  int col[KT];  // this lane's output column in tile t, clamped into Y
  bool cok[KT];
#pragma unroll
  for (int t = 0; t < KT; ++t) {
    cok[t] = EXACT || 16 * t + m < k;
    col[t] = EXACT ? 16 * t + m : (cok[t] ? 16 * t + m : k - 1);
  }
  const bool use_y = beta != 0.0;
  double sq[KT];
#pragma unroll
  for (int t = 0; t < KT; ++t) sq[t] = 0.0;
  const int64_t wg0 = (int64_t)blockIdx.x * kUpdRowsPerWg;
  for (int64_t r0 = wg0 + 16 * wave; r0 < wg0 + kUpdRowsPerWg && r0 < n;
       r0 += 16 * (kUpdThreads / 64)) {
    const bool rok = r0 + m < n;
    const double* pp = P + (rok ? r0 + m : n - 1) * ldp;
    // old Y of the strip (lane holds rows r0 + 4 q + c, columns 16 t + m)
    double* yrow[4];
    bool yok[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t r = r0 + 4 * q + c;
      yok[q] = r < n;
      yrow[q] = Y + (yok[q] ? r : n - 1) * ldy + (EXACT ? m : 0);
    }
    double yo[KT][4];
    if (use_y) {
#pragma unroll
      for (int t = 0; t < KT; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) yo[t][q] = yrow[q][EXACT ? 16 * t : col[t]];
    }
    v4d acc[KT];
#pragma unroll
    for (int t = 0; t < KT; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
    for (int cb = 0; cb < kp; cb += kUpdChunk) {
      const int steps = kp - cb >= kUpdChunk ? kUpdChunk / 4 : (kp - cb + 3) / 4;
      if (steps == kUpdChunk / 4) {
        double pa[kUpdChunk / 4];
#pragma unroll
        for (int s4 = 0; s4 < kUpdChunk / 4; ++s4) pa[s4] = pp[cb + 4 * s4 + c];
#pragma unroll
        for (int s4 = 0; s4 < kUpdChunk / 4; ++s4) {
          const double* pm = mlds + (cb + 4 * s4 + c) * ldl + m;
#pragma unroll
          for (int t = 0; t < KT; ++t) acc[t] = mfma16(rok ? pa[s4] : 0.0, pm[16 * t], acc[t]);
        }
      } else {  // the last, partial chunk of P's columns
        for (int s4 = 0; s4 < steps; ++s4) {
          const int cc = cb + 4 * s4 + c;
          const double a = pp[cc < kp ? cc : kp - 1];
          const double* pm = mlds + cc * ldl + m;
#pragma unroll
          for (int t = 0; t < KT; ++t) acc[t] = mfma16((rok && cc < kp) ? a : 0.0, pm[16 * t], acc[t]);
        }
      }
    }
    if (EXACT && r0 + 16 <= n) {  // whole strip: no guards on the stores
#pragma unroll
      for (int t = 0; t < KT; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double y = use_y ? fma(beta, yo[t][q], alpha * acc[t][q]) : alpha * acc[t][q];
          yrow[q][16 * t] = y;
          if (NORMS) sq[t] = fma(y, y, sq[t]);
        }
    } else {
#pragma unroll
      for (int t = 0; t < KT; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (yok[q] && cok[t]) {
            const double y = use_y ? fma(beta, yo[t][q], alpha * acc[t][q]) : alpha * acc[t][q];
            yrow[q][EXACT ? 16 * t : col[t]] = y;
            if (NORMS) sq[t] = fma(y, y, sq[t]);
          }
    }
  }
  if constexpr (NORMS) {
    __shared__ double wsum[kUpdThreads / 64][16 * KT];
#pragma unroll
    for (int t = 0; t < KT; ++t) {
      double v = sq[t];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      if (lane < 16) wsum[wave][16 * t + lane] = v;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < k; j += kUpdThreads) {
      double v = wsum[0][j];
#pragma unroll
      for (int w = 1; w < kUpdThreads / 64; ++w) v += wsum[w][j];
      npart[(int64_t)blockIdx.x * k + j] = v;
    }
  }
}

// The same for larger blocks: 64 rows per workgroup, 128 columns per
// grid.y, M read from global memory.
constexpr int kUpdWideThreads = 256;
__global__ void __launch_bounds__(kUpdWideThreads)
update_wide_kernel(int64_t n, int k, int kp, double alpha, const double* __restrict__ P,
                   int64_t ldp, const double* __restrict__ M, int ldm, double beta,
                   double* __restrict__ Y, int64_t ldy) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
  const int j0 = blockIdx.y * 16 * kUpdTiles;
  if (r0 >= n) return;
  const int c = lane >> 4, m = lane & 15;
  v4d acc[kUpdTiles];
#pragma unroll
  for (int t = 0; t < kUpdTiles; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
  const int64_t ra = r0 + m;
  const bool rok = ra < n;
  bool jok[kUpdTiles];
#pragma unroll
  for (int t = 0; t < kUpdTiles; ++t) jok[t] = j0 + 16 * t + m < k;
  const double* pp = P + ra * ldp;
  for (int c0 = 0; c0 < kp; c0 += 4) {
    const int cc = c0 + c;
    const double a = (rok && cc < kp) ? pp[cc] : 0.0;
    const double* pm = M + (int64_t)cc * ldm + j0 + m;
#pragma unroll
    for (int t = 0; t < kUpdTiles; ++t) {
      const double b = (cc < kp && jok[t]) ? pm[16 * t] : 0.0;
      acc[t] = mfma16(a, b, acc[t]);
    }
  }
#pragma unroll
  for (int t = 0; t < kUpdTiles; ++t) {
    if (!jok[t]) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t r = r0 + 4 * q + c;
      if (r >= n) continue;
      double* y = Y + r * ldy + j0 + 16 * t + m;
      *y = beta == 0.0 ? alpha * acc[t][q] : fma(beta, *y, alpha * acc[t][q]);
    }
  }
}

}  // namespace

int64_t gram_chunks(int64_t n) { return gram_blocks(n); }

int64_t update_workgroups(int64_t n) { return (n + kUpdRowsPerWg - 1) / kUpdRowsPerWg; }

int64_t gram_partial_rows(int64_t n, int64_t nb) {
  int64_t rows = (n + nb - 1) / nb;
  return rows < 1 ? 1 : rows;
}

hipError_t launch_gram_partial(int64_t n, int k, const double* A, int64_t lda, const double* B,
                               int64_t ldb, int64_t nb, double* work, hipStream_t s) {
  const int nbk = (k + kGramBlock - 1) / kGramBlock;
  const int64_t rows = gram_partial_rows(n, nb);
  hipLaunchKernelGGL(gram_partial_kernel<false>, dim3((unsigned)nb, (unsigned)(nbk * nbk)),
                     dim3(kGramThreads), 0, s, n, k, A, lda, B, ldb, B, ldb, rows, work, work);
  return hipGetLastError();
}

int64_t gram2_chunks(int64_t n) { return (gram_chunks(n) + 1) / 2; }

hipError_t launch_gram2_partial(int64_t n, int k, const double* A, int64_t lda, const double* B1,
                                int64_t ldb1, const double* B2, int64_t ldb2, int64_t nb,
                                double* work1, double* work2, hipStream_t s) {
  const int nbk = (k + kGramBlock - 1) / kGramBlock;
  const int64_t rows = gram_partial_rows(n, nb);
  hipLaunchKernelGGL(gram_partial_kernel<true>, dim3((unsigned)nb, (unsigned)(nbk * nbk)),
                     dim3(2 * kGramThreads), 0, s, n, k, A, lda, B1, ldb1, B2, ldb2, rows, work1,
                     work2);
  return hipGetLastError();
}

template <int KT>
hipError_t launch_update_kt(int64_t n, int k, int kp, double alpha, const double* P, int64_t ldp,
                            const double* M, int ldm, double beta, double* Y, int64_t ldy,
                            double* npart, hipStream_t s) {
  const size_t lds = (size_t)((kp + 3) & ~3) * update_ld(16 * KT) * sizeof(double);
  auto kern = k == 16 * KT ? (npart ? update_kernel<KT, true, true> : update_kernel<KT, true, false>)
                           : (npart ? update_kernel<KT, false, true> : update_kernel<KT, false, false>);
  KernelFacts f;  // raises the dynamic LDS limit on this device
  hipError_t err = kernel_facts(reinterpret_cast<const void*>(kern), kUpdThreads, lds, f);
  if (err != hipSuccess) return err;
  const int64_t wgs = (n + kUpdRowsPerWg - 1) / kUpdRowsPerWg;
  hipLaunchKernelGGL(kern, dim3((unsigned)wgs), dim3(kUpdThreads), lds, s, n, k, kp, alpha, P, ldp,
                     M, ldm, beta, Y, ldy, npart);
  return hipGetLastError();
}

bool update_in_lds(int k, int kp) {
  return k <= 16 * kUpdTiles && (int64_t)((kp + 3) & ~3) * update_ld(k) <= kUpdLds;
}

hipError_t launch_block_update(int64_t n, int k, int kp, double alpha, const double* P,
                               int64_t ldp, const double* M, int ldm, double beta, double* Y,
                               int64_t ldy, hipStream_t s, double* npart) {
  if (update_in_lds(k, kp)) {
    switch ((k + 15) / 16) {
      case 1: return launch_update_kt<1>(n, k, kp, alpha, P, ldp, M, ldm, beta, Y, ldy, npart, s);
      case 2: return launch_update_kt<2>(n, k, kp, alpha, P, ldp, M, ldm, beta, Y, ldy, npart, s);
      case 3: return launch_update_kt<3>(n, k, kp, alpha, P, ldp, M, ldm, beta, Y, ldy, npart, s);
      case 4: return launch_update_kt<4>(n, k, kp, alpha, P, ldp, M, ldm, beta, Y, ldy, npart, s);
      case 5: return launch_update_kt<5>(n, k, kp, alpha, P, ldp, M, ldm, beta, Y, ldy, npart, s);
      case 6: return launch_update_kt<6>(n, k, kp, alpha, P, ldp, M, ldm, beta, Y, ldy, npart, s);
      case 7: return launch_update_kt<7>(n, k, kp, alpha, P, ldp, M, ldm, beta, Y, ldy, npart, s);
      default: return launch_update_kt<8>(n, k, kp, alpha, P, ldp, M, ldm, beta, Y, ldy, npart, s);
    }
  }
  if (npart) return hipErrorInvalidValue;  // column norms only on the LDS path
  const int64_t wgs = (n + 63) / 64;
  const int nj = (k + 16 * kUpdTiles - 1) / (16 * kUpdTiles);
  hipLaunchKernelGGL(update_wide_kernel, dim3((unsigned)wgs, (unsigned)nj), dim3(kUpdWideThreads),
                     0, s, n, k, kp, alpha, P, ldp, M, ldm, beta, Y, ldy);
  return hipGetLastError();
}

// ------------------------------------------------ allocation-free Gram block
// The partial products of mf_block_gram_noalloc live in a file-scope device
// array: kScratchChunks chunks of up to kScratchMaxK^2 doubles (64 MiB), held
// by every GPU the library runs on until the process ends.  Every element a
// call reads was written by the same call's partial-product kernel first, so
// nothing needs clearing; calls that overlap in time on one GPU race.
constexpr int kScratchMaxK = 128;
constexpr int64_t kScratchChunks = 512;
static __device__ __align__(256) double scratch[kScratchChunks * kScratchMaxK * kScratchMaxK];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};

// The device address of `scratch` on the current device (the array's name is
// a host-side stand-in that must not reach a kernel).
int scratch_address(double** out) {
  int dev = 0;
  hipError_t err = hipGetDevice(&dev);
  if (err != hipSuccess) return hip_fail(err, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(MF_ERR_UNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (err != hipSuccess) return hip_fail(err, "hipGetSymbolAddress(scratch)");
    g_scratch[dev] = static_cast<double*>(p);
  }
  *out = g_scratch[dev];
  return MF_OK;
}

}  // namespace mf

using namespace mf;

extern "C" int mf_block_gram_noalloc(int64_t n, int k, const double* A, int64_t lda,
                                     const double* B, int64_t ldb, double alpha, double beta,
                                     double* C, int ldc, void* stream) {
  if (!C || (n > 0 && (!A || !B))) return fail(MF_ERR_ARG, "A, B and C must be non-NULL");
  if (n < 0 || k < 1 || lda < k || ldb < k || ldc < k)
    return fail(MF_ERR_ARG, "need n >= 0, k >= 1, lda, ldb, ldc >= k");
  if (k > kScratchMaxK)
    return fail(MF_ERR_UNSUPPORTED,
                "mf_block_gram_noalloc takes k <= 128 (its scratch holds 512 partial blocks of "
                "128 x 128); use mf_block_gram with a work array");
  const int64_t nb = gram_chunks(n);  // <= 512 = kScratchChunks
  const char* c0 = reinterpret_cast<const char*>(C);
  const size_t cs = ((size_t)(k - 1) * ldc + k) * sizeof(double);
  auto overlaps = [&](const double* X, int64_t ld) {
    if (n == 0) return false;
    const char* x0 = reinterpret_cast<const char*>(X);
    const size_t xs = ((size_t)(n - 1) * ld + k) * sizeof(double);
    return c0 < x0 + xs && x0 < c0 + cs;
  };
  if (overlaps(A, lda) || overlaps(B, ldb)) return fail(MF_ERR_ARG, "C overlaps A or B");
  double* work = nullptr;
  if (int st = scratch_address(&work)) return st;
  hipStream_t hs = static_cast<hipStream_t>(stream);
  hipError_t err = launch_gram_partial(n, k, A, lda, B, ldb, nb, work, hs);
  if (err == hipSuccess) err = launch_gram_reduce(k, (int)nb, work, alpha, beta, C, ldc, hs);
  if (err != hipSuccess) return hip_fail(err, "Gram kernel launch");
  return MF_OK;
}
