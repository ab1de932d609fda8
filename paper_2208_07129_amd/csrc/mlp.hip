// Kernels of the learned cell-local preconditioner: a small MLP applied to
// every (cell, column) of a residual block, trained on the GPU.
//
// Batch layout is feature-major: an activation block is [features][rows],
// row = e * k + j for cell e and column j, so a layer is C = W^T X with the
// long batch dimension as the GEMM's N and the weights as the row-major A
// operand.  The cell-blocked variant stores each cell's features x columns
// block contiguously (element (i, e k + j) at e * ld + i * k + j): the cell
// gather and the node assembly then stream whole cells instead of 256-byte
// pieces a batch row apart.  The GEMM runs on the gfx950 matrix cores
// (v_mfma_f32_16x16x32_bf16: BF16 operands, FP32 accumulation): one 64 x 64
// output tile per 256-thread workgroup, 2 x 2 waves of 32 x 32, K staged
// through LDS in steps of 32 with k contiguous per lane, so every fragment is
// one 16-byte LDS read.  Transposed operands (backward pass) are transposed
// while being staged.  Epilogues fuse bias, ReLU, the ReLU mask of the
// backward pass and the BF16 conversion; weight gradients split the batch
// dimension across workgroups and add FP32 partial tiles atomically.
#include <cmath>
#include <type_traits>

#include "mf_internal.h"
#include "sf_common.h"

namespace mf {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even (finite inputs)
  return (uint16_t)(u >> 16);
}
__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

namespace {

constexpr int kTile = 64, kKStep = 32, kPad = 40;  // LDS rows of 80 bytes

// C (M x N) = op(A) (M x K) * op(B) (K x N).  A: row-major M x K (lda), or,
// with TA, stored K x M.  B: row-major K x N (ldb), or, with TB, stored N x K.
// M, N, K multiples of 8 (8-element, 16-byte staging chunks).  blockIdx.z
// takes the K range [z kchunk, (z+1) kchunk).  Output tiles are numbered with
// the M tile fastest, and workgroup b takes tile (b mod 8) c + b / 8 (c =
// gridDim.x / 8): consecutive workgroups go to different XCDs, so this gives
// each XCD a contiguous range of tiles and the few tiles that share an N slice
// of B (the long batch operand) run on one XCD, which reads that slice from
// HBM once into its L2.
template <bool TA, bool TB>
__global__ void __launch_bounds__(256)
gemm_bf16_kernel(int M, int N, int K, const uint16_t* __restrict__ A, int64_t lda,
                 const uint16_t* __restrict__ B, int64_t ldb, int kchunk, GemmEpi ep) {
  // two LDS buffers: step s is staged into buffer s mod 2 while its global
  // loads for step s + 1 are already in flight (one barrier per step)
  __shared__ __attribute__((aligned(16))) uint16_t As[2][kTile][kPad];  // [m][k]
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][kTile][kPad];  // [n][k]
  const int mtiles = (M + kTile - 1) / kTile;
  const int64_t tiles = (int64_t)mtiles * ((N + kTile - 1) / kTile);
  const int64_t lt = (int64_t)(blockIdx.x % kXcds) * (gridDim.x / kXcds) + blockIdx.x / kXcds;
  if (lt >= tiles) return;  // the few padding workgroups of the last XCD range
  const int m0 = (int)(lt % mtiles) * kTile, n0 = (int)(lt / mtiles) * kTile;
  const int kb = blockIdx.z * kchunk;
  const int ke = min(K, kb + kchunk);
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  // This thread's 16-byte staging chunk of each operand.  A transposed operand
  // is transposed while stored (eight 2-byte stores); the lanes of a
  // wavefront then span the 32 k rows, so those stores fall on 32 banks.
  // Loads read clamped (valid) addresses and a select zeroes what lies
  // outside the operand, so no load sits behind a branch.
  const uint4 zero = {0u, 0u, 0u, 0u};
  const int a_kk = TA ? (t & 31) : (t & 3) * 8, a_m = TA ? (t >> 5) * 8 : (t >> 2);
  const int b_kk = TB ? (t & 3) * 8 : (t & 31), b_n = TB ? (t >> 2) : (t >> 5) * 8;
  uint4 va, vb;
  auto gload = [&](int k0) {
    {
      const int kk = k0 + a_kk, m = m0 + a_m;
      const bool ok = kk < ke && m < M;
      const int kc = ok ? kk : kb, mc = ok ? m : m0;
      const uint4 v = TA ? *reinterpret_cast<const uint4*>(A + (int64_t)kc * lda + mc)
                         : *reinterpret_cast<const uint4*>(A + (int64_t)mc * lda + kc);
      va = ok ? v : zero;
    }
    {
      const int kk = k0 + b_kk, nn = n0 + b_n;
      const bool ok = kk < ke && nn < N;
      const int kc = ok ? kk : kb, nc = ok ? nn : n0;
      int64_t off;
      if constexpr (TB) off = (int64_t)nc * ldb + kc;
      else  // 8 columns inside one block (kb multiple of 8)
        off = ep.kb > 0 ? (int64_t)(nc / ep.kb) * ldb + (int64_t)kc * ep.kb + nc % ep.kb
                        : (int64_t)kc * ldb + nc;
      const uint4 v = *reinterpret_cast<const uint4*>(B + off);
      vb = ok ? v : zero;
    }
  };
  auto lstore = [&](int buf) {
    if constexpr (TA) {
      const uint16_t* e = reinterpret_cast<const uint16_t*>(&va);
#pragma unroll
      for (int i = 0; i < 8; ++i) As[buf][a_m + i][a_kk] = e[i];
    } else {
      *reinterpret_cast<uint4*>(&As[buf][a_m][a_kk]) = va;
    }
    if constexpr (TB) {
      *reinterpret_cast<uint4*>(&Bs[buf][b_n][b_kk]) = vb;
    } else {
      const uint16_t* e = reinterpret_cast<const uint16_t*>(&vb);
#pragma unroll
      for (int i = 0; i < 8; ++i) Bs[buf][b_n + i][b_kk] = e[i];
    }
  };
  gload(kb);
  for (int k0 = kb, step = 0; k0 < ke; k0 += kKStep, ++step) {
    const int buf = step & 1;
    lstore(buf);
    __syncthreads();
    if (k0 + kKStep < ke) gload(k0 + kKStep);
    bf16x8 a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      a[i] = *reinterpret_cast<const bf16x8*>(&As[buf][wm + i * 16 + (lane & 15)][(lane >> 4) * 8]);
      b[i] = *reinterpret_cast<const bf16x8*>(&Bs[buf][wn + i * 16 + (lane & 15)][(lane >> 4) * 8]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
  }

  // D layout of the 16 x 16 tile: lane -> column lane % 16, rows 4 (lane / 16) + r
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + i * 16 + (lane >> 4) * 4 + r;
        const int n = n0 + wn + j * 16 + (lane & 15);
        if (m >= M || n >= N) continue;
        float v = acc[i][j][r];
        if (ep.bias) v += ep.bias[m];
        if (ep.relu) v = v > 0.f ? v : 0.f;
        if (ep.mask && !(bf16_to_f32(ep.mask[(int64_t)m * ep.ldmask + n]) > 0.f)) v = 0.f;
        const int64_t nb = ep.kb > 0 ? (int64_t)(n / ep.kb) : 0, nr = ep.kb > 0 ? n % ep.kb : n;
        if (ep.out_f32) {
          float* o = ep.out_f32 + (ep.kb > 0 ? nb * ep.ld_f32 + (int64_t)m * ep.kb + nr
                                             : (int64_t)m * ep.ld_f32 + n);
          if (ep.atomic) unsafeAtomicAdd(o, v);
          else *o = v;
        }
        if (ep.out_bf16)
          ep.out_bf16[ep.kb > 0 ? nb * ep.ld_bf16 + (int64_t)m * ep.kb + nr
                                : (int64_t)m * ep.ld_bf16 + n] = f32_to_bf16(v);
      }
}

// Partition-of-unity weight of a free node: 1 / (number of (cell, local
// node) occurrences), per direction 2 on a shared cell face, 1 otherwise.
__device__ inline double pou_weight(const GridDesc& g, int i1, int i2, int i3, int cx, int cy,
                                    int cz) {
  const int li[3] = {i1, i2, i3}, c[3] = {cx, cy, cz};
  double w = 1.0;
  for (int d = 0; d < 3; ++d) {
    const bool periodic = g.N[d] == g.n[d] * g.p;
    const bool lo = li[d] == 0, hi = li[d] == g.p;
    if (!(lo || hi)) continue;
    const bool outer = !periodic && ((lo && c[d] == 0) || (hi && c[d] == g.n[d] - 1));
    if (!outer) w *= 0.5;
  }
  return w;
}

// One workgroup per (cell, chunk of 64 columns); thread t: column t % 64,
// node phase t / 64.  rho = RMS of the cell's residual column (over the
// cell's F = np^3 node values, constrained nodes as 0); X0t[i][row] =
// R[node_i][j] / rho as BF16 (rows i in [F, Fp) zero), Tt[i][row] =
// E[node_i][j] / rho in FP32 when E is given (training targets).  The node
// numbers and the per-node input and target factors of the cell are formed
// once per workgroup in LDS (kMaxCellNodes entries), so the column loops only
// load, scale and store.
constexpr int kCols = 64;
constexpr int kMaxCellNodes = 11 * 11 * 11;

// Per (cell, local node): the node number (-1 constrained), the input factor
// sqrt(w)^[pou_sqrt] / sqrt(d) and sqrt(d) (d = dsc[node], 1 without dsc).
__device__ inline void cell_node_factors(const GridDesc& g, int np, int cx, int cy, int cz,
                                         int pou_sqrt, const double* __restrict__ dsc, int* snode,
                                         double* sfin, double* sdh) {
  const int F = np * np * np;
  for (int i = threadIdx.x; i < F; i += blockDim.x) {
    const int i1 = i % np, i2 = (i / np) % np, i3 = i / (np * np);
    const int node = grid_node(g, cx, cy, cz, i1, i2, i3);
    double fi = 0.0, dh = 1.0;
    if (node >= 0) {
      const double ws = pou_sqrt ? sqrt(pou_weight(g, i1, i2, i3, cx, cy, cz)) : 1.0;
      dh = dsc ? sqrt(dsc[node]) : 1.0;
      fi = ws / dh;
    }
    snode[i] = node;
    sfin[i] = fi;
    if (sdh) sdh[i] = dh;
  }
}

__global__ void __launch_bounds__(256)
cell_gather_kernel(GridDesc g, int np, int k, const double* __restrict__ R, int64_t ldr,
                   const double* __restrict__ E, int64_t lde, int Fp, uint16_t* __restrict__ X0t,
                   float* __restrict__ Tt, int64_t ldx, float* __restrict__ rho, int pou_sqrt,
                   const double* __restrict__ dsc, int blocked) {
  __shared__ double part[256];
  __shared__ int snode[kMaxCellNodes];
  __shared__ double sfin[kMaxCellNodes], sdh[kMaxCellNodes];
  const int e = blockIdx.x;
  const int j0 = blockIdx.y * kCols;
  const int t = threadIdx.x, jj = t % kCols, ph = t / kCols;
  const int j = j0 + jj;
  const int F = np * np * np;
  const int cx = e % g.n[0], cy = (e / g.n[0]) % g.n[1], cz = e / (g.n[0] * g.n[1]);
  cell_node_factors(g, np, cx, cy, cz, pou_sqrt, dsc, snode, sfin, sdh);
  __syncthreads();
  // Loads never sit behind a branch: constrained nodes and the padding rows
  // read a valid element (clamped index) whose value a select then drops, and
  // lanes past the last column read column k - 1 and store nothing; batches
  // of kGatherBatch rows are loaded before they are used.
  const bool jok = j < k;
  const int jc = jok ? j : k - 1;
  constexpr int kGatherBatch = 8;
  const int nrows = (Fp - ph + 3) / 4;  // rows i = ph, ph + 4, ... < Fp of this wavefront
  auto node_of = [&](int i) { return snode[i < F ? i : F - 1]; };
  double s = 1.0;  // without rho: no normalisation
  if (rho) {
    double ss = 0.0;
    for (int r0 = 0; r0 < nrows; r0 += kGatherBatch) {
      double xv[kGatherBatch];
#pragma unroll
      for (int u = 0; u < kGatherBatch; ++u) {
        const int node = node_of(ph + 4 * (r0 + u));
        xv[u] = R[(int64_t)(node >= 0 ? node : 0) * ldr + jc];
      }
#pragma unroll
      for (int u = 0; u < kGatherBatch; ++u) {
        const int i = ph + 4 * (r0 + u);
        const double f = i < F ? sfin[i] : 0.0;  // 0 for constrained nodes and padding
        const double x = f != 0.0 ? xv[u] * f : 0.0;
        ss = fma(x, x, ss);
      }
    }
    part[t] = ss;
    __syncthreads();
    double tot = part[jj] + part[jj + 64] + part[jj + 128] + part[jj + 192];
    const double r = sqrt(tot / F);
    s = r > 0.0 ? 1.0 / r : 0.0;
    if (jok && ph == 0) rho[(int64_t)e * k + j] = (float)r;
  }
  if (!jok) return;
  const int64_t row = (int64_t)e * k + j;
  // element (i, row) at i * istep + base
  const int64_t base = blocked ? (int64_t)e * ldx + j : row, istep = blocked ? k : ldx;
  auto rows = [&](auto with_e) {
    constexpr bool WE = decltype(with_e)::value;
    for (int r0 = 0; r0 < nrows; r0 += kGatherBatch) {
      double xv[kGatherBatch], yv[kGatherBatch];
#pragma unroll
      for (int u = 0; u < kGatherBatch; ++u) {
        const int node = node_of(ph + 4 * (r0 + u));
        const int64_t nc = node >= 0 ? node : 0;
        xv[u] = R[nc * ldr + j];
        if constexpr (WE) yv[u] = E[nc * lde + j];
      }
#pragma unroll
      for (int u = 0; u < kGatherBatch; ++u) {
        if (r0 + u >= nrows) break;  // uniform across the wavefront
        const int i = ph + 4 * (r0 + u);
        const double f = i < F ? sfin[i] : 0.0;
        const double x = f != 0.0 ? xv[u] * s * f : 0.0;
        X0t[i * istep + base] = f32_to_bf16((float)x);
        if constexpr (WE) Tt[i * istep + base] = f != 0.0 ? (float)(yv[u] * s * sdh[i]) : 0.0f;
      }
    }
  };
  if (E) rows(std::true_type{});
  else rows(std::false_type{});
}

// The incidences of grid node g (0 <= g < N) along one direction: the cells
// c[0..cnt) holding it and its local index l[] there, with the
// partition-of-unity factor of the direction (1/2 when two cells share the
// node, 1 otherwise, as pou_weight).  Periodic directions have N = n p (node
// n p is node 0); with n = 1 a vertex node meets the one cell twice.
__device__ inline int node_incidences(int g, int n, int N, int p, int* c, int* l, double* w) {
  const bool periodic = N == n * p;
  const int cq = g / p, r = g - cq * p;
  if (r != 0) {
    c[0] = cq;
    l[0] = r;
    *w = 1.0;
    return 1;
  }
  int cnt = 0;
  if (cq < n) {  // the cell starting at the node
    c[cnt] = cq;
    l[cnt++] = 0;
  }
  if (cq > 0 || periodic) {  // the cell ending at the node
    c[cnt] = cq > 0 ? cq - 1 : n - 1;
    l[cnt++] = p;
  }
  *w = cnt == 2 ? 0.5 : 1.0;
  return cnt;
}

// Z[node][j] = (R[node][j] / diag[node] or 0) + sum over the node's
// incidences (cell e, local node i) of w^[1/2] rho[e k + j] Yt(i, e k + j)
// (divided by sqrt(dsc[node])): the partition-of-unity assembly taken node by
// node, so every Z element is written once by one lane, with a fixed order of
// its up to eight terms (no atomics; bitwise reproducible).  Constrained nodes
// get only the Jacobi term, as the scattered form never adds to them.
//
// One wavefront per (x-line of a cell, 64 columns): the nodes gx = cx p + l,
// l = 0 .. p - 1 (and l = p in the last cell of a non-periodic direction), at
// fixed (gy, gz), lanes over the columns.  Along the line only l = 0 can have
// a second x-incidence, and the y, z incidences are the same for every node,
// so with p and their counts as template parameters all the line's loads are
// independent and in flight together (one node per wavefront left the kernel
// bound by memory latency).
constexpr int kAsmLines = 4;  // lines (wavefronts) per workgroup

struct AsmArgs {
  GridDesc g;
  int k;
  const float* Yt;
  int64_t ldy;
  const float* rho;
  const double* diag;
  const double* R;
  int64_t ldr;
  double* Z;
  int64_t ldz;
  int pou_sqrt;
  const double* dsc;
  int blocked;
};

// lane l's value of v, as a wave-uniform value
__device__ __forceinline__ double wave_bcast(double v, int l) {
  const int2 h = __builtin_bit_cast(int2, v);
  const int2 r{__builtin_amdgcn_readlane(h.x, l), __builtin_amdgcn_readlane(h.y, l)};
  return __builtin_bit_cast(double, r);
}

template <int P, int NY, int NZ, bool BLK, bool RHO, bool DIAG>
__device__ __forceinline__ void assemble_line(const AsmArgs& a, int cx, int gy, int gz,
                                              const int* cy, const int* ly, double wy,
                                              const int* cz, const int* lz, double wz, int j,
                                              bool jok) {
  constexpr int NP = P + 1;
  const GridDesc& g = a.g;
  const int n0 = g.n[0], N0 = g.N[0];
  const bool periodic_x = N0 == n0 * P;
  const bool has_left = periodic_x || cx > 0;   // a cell ends at gx = cx p
  const bool extra = !periodic_x && cx == n0 - 1;  // node l = p is this line's too
  const int cxl = cx > 0 ? cx - 1 : n0 - 1;
  const bool line_constrained =
      g.dirichlet && (gy == 0 || gy == g.N[1] - 1 || gz == 0 || gz == g.N[2] - 1);
  int64_t eyz[NY * NZ];
  int iyz[NY * NZ];
#pragma unroll
  for (int c = 0; c < NZ; ++c)
#pragma unroll
    for (int b = 0; b < NY; ++b) {
      eyz[c * NY + b] = (int64_t)n0 * (cy[b] + (int64_t)g.n[1] * cz[c]);
      iyz[c * NY + b] = NP * (ly[b] + NP * lz[c]);
    }
  auto yload = [&](int64_t e, int i) -> float {
    return BLK ? a.Yt[e * a.ldy + (int64_t)i * a.k + j] : a.Yt[(int64_t)i * a.ldy + e * a.k + j];
  };
  auto rload = [&](int64_t e) -> float {
    if constexpr (RHO) return a.rho[e * a.k + j];
    return 1.0f;
  };
  // all the line's loads first (independent, in flight together), then the sums
  constexpr int Q = NY * NZ;
  float yv[P + 2][Q], rv[3][Q];  // rows: l = 0 .. p - 1, the left cell's p, this cell's p
#pragma unroll
  for (int q = 0; q < Q; ++q) {
#pragma unroll
    for (int l = 0; l < P; ++l) yv[l][q] = yload(cx + eyz[q], l + iyz[q]);
    yv[P][q] = yload(cxl + eyz[q], P + iyz[q]);
    yv[P + 1][q] = yload(cx + eyz[q], P + iyz[q]);
    rv[0][q] = rload(cx + eyz[q]);
    rv[1][q] = rload(cxl + eyz[q]);
  }
  double acc[P + 1];
#pragma unroll
  for (int l = 0; l < P; ++l) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) s += (double)rv[0][q] * (double)yv[l][q];
    if (l == 0) {  // the cell to the left, local node p (added if it exists)
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < Q; ++q) t += (double)rv[1][q] * (double)yv[P][q];
      s += has_left ? t : 0.0;
    }
    acc[l] = s;
  }
  acc[P] = 0.0;
#pragma unroll
  for (int q = 0; q < Q; ++q) acc[P] += (double)rv[0][q] * (double)yv[P + 1][q];
  if (!extra) acc[P] = 0.0;
  // per-node factors of the line, one node per lane (lanes 0 .. p), then read
  // back as wave-uniform values: 1 / diag and w^[1/2] / sqrt(dsc)
  const double wyz = wy * wz;
  const int64_t row0 = (int64_t)N0 * (gy + (int64_t)g.N[1] * gz);
  const int lane = threadIdx.x & 63;
  double invd = 0.0, fac = 0.0;
  if (lane <= P) {
    const int gx = cx * P + (lane < P || extra ? lane : 0);
    const int64_t node = row0 + gx;
    if constexpr (DIAG) invd = 1.0 / a.diag[node];
    const double pw = ((lane == 0 && has_left) ? 0.5 : 1.0) * wyz;
    fac = a.pou_sqrt ? sqrt(pw) : pw;
    if (a.dsc) fac /= sqrt(a.dsc[node]);
  }
  double rj[P + 1];  // the Jacobi term's R values (l = p: a valid node when not this line's)
  if constexpr (DIAG) {
#pragma unroll
    for (int l = 0; l <= P; ++l) {
      const int gx = cx * P + (l < P || extra ? l : 0);
      rj[l] = a.R[(row0 + gx) * a.ldr + j];
    }
  }
#pragma unroll
  for (int l = 0; l <= P; ++l) {
    if (l == P && !extra) break;
    const int gx = cx * P + l;
    const int64_t node = row0 + gx;
    const double il = wave_bcast(invd, l), fl = wave_bcast(fac, l);
    double z = 0.0;
    if constexpr (DIAG) z = rj[l] * il;
    const bool constrained = line_constrained || (g.dirichlet && (gx == 0 || gx == N0 - 1));
    if (!constrained) z = fma(fl, acc[l], z);
    if (jok) a.Z[node * a.ldz + j] = z;
  }
}

// BLK: cell-blocked Yt; RHO: rho given; DIAG: the Jacobi term (compile-time,
// so that no load sits behind a branch and the line's loads issue together)
template <int P, bool BLK, bool RHO, bool DIAG>
__global__ void __attribute__((amdgpu_flat_work_group_size(1, 64 * kAsmLines),
                               amdgpu_waves_per_eu(1, 4)))
node_assemble_kernel(AsmArgs a, int nlines, int nchunks) {
  // the column chunk varies fastest, so the halves of a Z row (and of an R
  // row) are written and read together
  const int chunk = (int)(blockIdx.x % nchunks);
  const int line = (int)(blockIdx.x / nchunks) * kAsmLines + (int)(threadIdx.x >> 6);  // < 2^31
  // every lane stays (lanes 0 .. p form the line's node factors); lanes past
  // the last column read column k - 1 and store nothing
  const int jl = chunk * 64 + (threadIdx.x & 63);
  const bool jok = jl < a.k;
  const int j = jok ? jl : a.k - 1;
  if (line >= nlines) return;
  const GridDesc& g = a.g;
  const int cx = line % g.n[0];
  const int rest = line / g.n[0];
  const int gy = rest % g.N[1], gz = rest / g.N[1];
  int cy[2], cz[2], ly[2], lz[2];
  double wy, wz;
  const int ny = node_incidences(gy, g.n[1], g.N[1], P, cy, ly, &wy);
  const int nz = node_incidences(gz, g.n[2], g.N[2], P, cz, lz, &wz);
  if (ny == 1 && nz == 1) assemble_line<P, 1, 1, BLK, RHO, DIAG>(a, cx, gy, gz, cy, ly, wy, cz, lz, wz, j, jok);
  else if (ny == 2 && nz == 1) assemble_line<P, 2, 1, BLK, RHO, DIAG>(a, cx, gy, gz, cy, ly, wy, cz, lz, wz, j, jok);
  else if (ny == 1) assemble_line<P, 1, 2, BLK, RHO, DIAG>(a, cx, gy, gz, cy, ly, wy, cz, lz, wz, j, jok);
  else assemble_line<P, 2, 2, BLK, RHO, DIAG>(a, cx, gy, gz, cy, ly, wy, cz, lz, wz, j, jok);
}

// dYt = 2 scale w[n] (Yt - Tt) for features < F (0 for the padding), as
// BF16; loss += scale sum w[n] (Yt - Tt)^2 (w = 1 when the row weights are
// null).
__global__ void __launch_bounds__(256)
mse_grad_kernel(int F, int Fp, int64_t nrows, const float* __restrict__ Yt,
                const float* __restrict__ Tt, int64_t ld, const float* __restrict__ roww,
                float scale, uint16_t* __restrict__ dYt, double* __restrict__ loss) {
  __shared__ double part[256];
  double acc = 0.0;
  const int64_t total = (int64_t)Fp * nrows;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx / nrows);
    const int64_t n = idx % nrows;
    const float w = roww ? roww[n] : 1.0f;
    float d = 0.f;
    if (i < F) {
      d = Yt[(int64_t)i * ld + n] - Tt[(int64_t)i * ld + n];
      acc += (double)w * d * d;
    }
    dYt[(int64_t)i * ld + n] = f32_to_bf16(2.0f * scale * w * d);
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) unsafeAtomicAdd(loss, part[0] * (double)scale);
}

// out[m] (+)= sum_n X[m][n] (BF16 rows): bias gradients.
__global__ void __launch_bounds__(256)
row_sums_kernel(int64_t N, const uint16_t* __restrict__ X, int64_t ld, float* __restrict__ out,
                int accumulate) {
  __shared__ float part[256];
  const int m = blockIdx.x;
  float acc = 0.f;
  for (int64_t n = threadIdx.x; n < N; n += blockDim.x) acc += bf16_to_f32(X[(int64_t)m * ld + n]);
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[m] = (accumulate ? out[m] : 0.f) + part[0];
}

// Adam on FP32 master parameters; writes the BF16 copy when given.
__global__ void adam_kernel(int64_t n, float* __restrict__ w, const float* __restrict__ grad,
                            float* __restrict__ m1, float* __restrict__ m2,
                            uint16_t* __restrict__ wbf, float lr, float b1, float b2, float eps,
                            float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = grad[i];
    const float a = b1 * m1[i] + (1.f - b1) * gi;
    const float b = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = b;
    const float wi = w[i] - lr * (a / c1) / (sqrtf(b / c2) + eps);
    w[i] = wi;
    if (wbf) wbf[i] = f32_to_bf16(wi);
  }
}

// S <- (S + S^T) / 2 on the leading n x n block of a row-major matrix (ld),
// with its BF16 copy (same layout) refreshed.
__global__ void symmetrize_kernel(int n, float* __restrict__ S, int64_t ld, uint16_t* __restrict__ Sbf) {
  const int64_t total = (int64_t)n * n;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx / n), j = (int)(idx % n);
    if (j < i) continue;
    const float v = 0.5f * (S[(int64_t)i * ld + j] + S[(int64_t)j * ld + i]);
    S[(int64_t)i * ld + j] = v;
    S[(int64_t)j * ld + i] = v;
    if (Sbf) {
      const uint16_t b = f32_to_bf16(v);
      Sbf[(int64_t)i * ld + j] = b;
      Sbf[(int64_t)j * ld + i] = b;
    }
  }
}

__global__ void to_bf16_kernel(int64_t n, const float* __restrict__ src, uint16_t* __restrict__ dst) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = f32_to_bf16(src[i]);
}

__global__ void fill_f32_kernel(float* __restrict__ v, int64_t n, float x) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    v[i] = x;
}

// A[i][j] = (S[i][j] + S[j][i]) / 2 in FP64.
__global__ void skip_sym_kernel(int F, const float* __restrict__ S, int64_t lds,
                                double* __restrict__ A) {
  const int64_t total = (int64_t)F * F;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx / F), j = (int)(idx - (int64_t)i * F);
    A[idx] = 0.5 * ((double)S[(int64_t)i * lds + j] + (double)S[(int64_t)j * lds + i]);
  }
}

// S[i][j] = sum_r V[i][r] max(w_r, floor) V[j][r], written to S (FP32) and
// Sbf (BF16), floor = -1 + margin + 2^-8 (||w||_2 + sqrt(F)) (every thread
// forms it in the same order).  The product V[i][r] V[j][r] is formed first,
// so (i, j) and (j, i) take identical operations: exactly symmetric.
__global__ void skip_rebuild_kernel(int F, const double* __restrict__ V,
                                    const double* __restrict__ w, double margin,
                                    float* __restrict__ S, int64_t lds, uint16_t* __restrict__ Sbf,
                                    int64_t ldsb) {
  double n2 = 0.0;
  for (int r = 0; r < F; ++r) n2 = fma(w[r], w[r], n2);
  const double floor = -1.0 + margin + 0.00390625 * (sqrt(n2) + sqrt((double)F));
  const int64_t total = (int64_t)F * F;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx / F), j = (int)(idx - (int64_t)i * F);
    double acc = 0.0;
    for (int r = 0; r < F; ++r) {
      const double lam = w[r] > floor ? w[r] : floor;
      acc = fma(V[(int64_t)i * F + r] * V[(int64_t)j * F + r], lam, acc);
    }
    S[(int64_t)i * lds + j] = (float)acc;
    Sbf[(int64_t)i * ldsb + j] = f32_to_bf16((float)acc);
  }
}

unsigned blocks_for(int64_t total) {
  int64_t b = (total + 255) / 256;
  if (b > 65536) b = 65536;
  return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

hipError_t launch_gemm_bf16(int M, int N, int K, bool ta, bool tb, const uint16_t* A, int64_t lda,
                            const uint16_t* B, int64_t ldb, int kchunk, const GemmEpi& ep,
                            hipStream_t s) {
  if (kchunk <= 0 || kchunk > K) kchunk = K;
  kchunk = (kchunk + kKStep - 1) / kKStep * kKStep;
  const int kz = (K + kchunk - 1) / kchunk;
  const int64_t tiles = ((int64_t)N + kTile - 1) / kTile * ((M + kTile - 1) / kTile);
  dim3 grid((unsigned)((tiles + kXcds - 1) / kXcds * kXcds), 1, kz);
  if (!ta && !tb)
    hipLaunchKernelGGL((gemm_bf16_kernel<false, false>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, kchunk, ep);
  else if (ta && !tb)
    hipLaunchKernelGGL((gemm_bf16_kernel<true, false>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, kchunk, ep);
  else if (!ta && tb)
    hipLaunchKernelGGL((gemm_bf16_kernel<false, true>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, kchunk, ep);
  else
    hipLaunchKernelGGL((gemm_bf16_kernel<true, true>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, kchunk, ep);
  return hipGetLastError();
}

hipError_t launch_cell_gather(const Operator& op, int k, const double* R, int64_t ldr,
                              const double* E, int64_t lde, int Fp, uint16_t* X0t, float* Tt,
                              int64_t ldx, float* rho, int pou_sqrt, const double* dsc,
                              int blocked, hipStream_t s) {
  dim3 grid((unsigned)op.ncells, (k + kCols - 1) / kCols);
  hipLaunchKernelGGL(cell_gather_kernel, grid, dim3(256), 0, s, op.grid, op.np, k, R, ldr, E, lde,
                     Fp, X0t, Tt, ldx, rho, pou_sqrt, dsc, blocked);
  return hipGetLastError();
}

hipError_t launch_skip_sym(int F, const float* S, int64_t lds, double* A, hipStream_t s) {
  hipLaunchKernelGGL(skip_sym_kernel, dim3(blocks_for((int64_t)F * F)), dim3(256), 0, s, F, S, lds,
                     A);
  return hipGetLastError();
}

hipError_t launch_skip_rebuild(int F, const double* V, const double* w, double margin, float* S,
                               int64_t lds, uint16_t* Sbf, int64_t ldsb, hipStream_t s) {
  hipLaunchKernelGGL(skip_rebuild_kernel, dim3(blocks_for((int64_t)F * F)), dim3(256), 0, s, F, V,
                     w, margin, S, lds, Sbf, ldsb);
  return hipGetLastError();
}

hipError_t launch_cell_scatter(const Operator& op, int k, const float* Yt, int64_t ldy,
                               const float* rho, const double* diag, const double* R, int64_t ldr,
                               double* Z, int64_t ldz, int pou_sqrt, const double* dsc,
                               int blocked, hipStream_t s) {
  const AsmArgs a{op.grid, k, Yt, ldy, rho, diag, R, ldr, Z, ldz, pou_sqrt, dsc, blocked};
  const int nlines = (int)((int64_t)op.grid.n[0] * op.grid.N[1] * op.grid.N[2]);  // <= ndofs
  const int nch = (k + 63) / 64;
  dim3 grid((unsigned)(((int64_t)nlines + kAsmLines - 1) / kAsmLines * nch));
  dim3 block(64 * kAsmLines);
  auto go = [&](auto pc) {
    constexpr int P = decltype(pc)::value;
    const int v = (blocked ? 4 : 0) + (rho ? 2 : 0) + (diag ? 1 : 0);
#define MF_ASM(B, Rh, D) \
  hipLaunchKernelGGL((node_assemble_kernel<P, B, Rh, D>), grid, block, 0, s, a, nlines, nch)
    switch (v) {
      case 0: MF_ASM(false, false, false); break;
      case 1: MF_ASM(false, false, true); break;
      case 2: MF_ASM(false, true, false); break;
      case 3: MF_ASM(false, true, true); break;
      case 4: MF_ASM(true, false, false); break;
      case 5: MF_ASM(true, false, true); break;
      case 6: MF_ASM(true, true, false); break;
      default: MF_ASM(true, true, true); break;
    }
#undef MF_ASM
  };
  switch (op.p) {
    case 1: go(std::integral_constant<int, 1>{}); break;
    case 2: go(std::integral_constant<int, 2>{}); break;
    case 3: go(std::integral_constant<int, 3>{}); break;
    case 4: go(std::integral_constant<int, 4>{}); break;
    case 5: go(std::integral_constant<int, 5>{}); break;
    case 6: go(std::integral_constant<int, 6>{}); break;
    case 7: go(std::integral_constant<int, 7>{}); break;
    case 8: go(std::integral_constant<int, 8>{}); break;
    case 9: go(std::integral_constant<int, 9>{}); break;
    case 10: go(std::integral_constant<int, 10>{}); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_mse_grad(int F, int Fp, int64_t nrows, const float* Yt, const float* Tt,
                           int64_t ld, const float* roww, float scale, uint16_t* dYt, double* loss,
                           hipStream_t s) {
  unsigned blocks = blocks_for((int64_t)Fp * nrows);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(mse_grad_kernel, dim3(blocks), dim3(256), 0, s, F, Fp, nrows, Yt, Tt, ld, roww,
                     scale, dYt, loss);
  return hipGetLastError();
}

hipError_t launch_row_sums(int M, int64_t N, const uint16_t* X, int64_t ld, float* out,
                           bool accumulate, hipStream_t s) {
  hipLaunchKernelGGL(row_sums_kernel, dim3(M), dim3(256), 0, s, N, X, ld, out, accumulate ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_adam(int64_t n, float* w, const float* g, float* m1, float* m2, uint16_t* wbf,
                       float lr, float b1, float b2, float eps, int step, hipStream_t s) {
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n)), dim3(256), 0, s, n, w, g, m1, m2, wbf, lr,
                     b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_symmetrize(int n, float* S, int64_t ld, uint16_t* Sbf, hipStream_t s) {
  hipLaunchKernelGGL(symmetrize_kernel, dim3(blocks_for((int64_t)n * n)), dim3(256), 0, s, n, S, ld,
                     Sbf);
  return hipGetLastError();
}

hipError_t launch_to_bf16(int64_t n, const float* src, uint16_t* dst, hipStream_t s) {
  hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks_for(n)), dim3(256), 0, s, n, src, dst);
  return hipGetLastError();
}

hipError_t launch_fill_f32(float* v, int64_t n, float x, hipStream_t s) {
  hipLaunchKernelGGL(fill_f32_kernel, dim3(blocks_for(n)), dim3(256), 0, s, v, n, x);
  return hipGetLastError();
}

}  // namespace mf
