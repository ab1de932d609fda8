// Internal declarations shared by the host setup, the C ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "mfmv.h"  // from the repository include directory (-I)

namespace mf {

constexpr int kMaxP = 10;
constexpr int kMaxQExtra = 3;  // q in [p+1, p+3]
// Launch shapes of the box-cell kernel: 0 .. 9, 11, 12 on the vector ALUs,
// 10 the FP64 matrix-core body (q = p + 1 <= 8)
constexpr int kBoxMfmaCfg = 10;
constexpr int kBoxCfgs = 13;
constexpr int kMfmaMaxN = 8;     // points per direction the matrix-core body handles
constexpr int kMixedCfgs = 7;  // launch shapes of the mixed-precision apply (4..6: FP32 vector)
constexpr int kBatchCfgs = 6;  // launch shapes of the batched apply (3..5: one launch per kind)
constexpr int kMaxBatch = 64;  // operators per batch (operator indices fit in a byte)

// Error reporting: every entry point returns a status and stores a message.
int fail(int status, const std::string& msg);
int hip_fail(hipError_t err, const char* what);

// ---------------------------------------------------------------- host setup
struct Rule1D {
  std::vector<double> x, w;
};
Rule1D gauss_rule(int n);
std::vector<double> gll_points(int p);

// Unfolded 1D tables (row-major, quadrature point major).
struct Tables1D {
  int np = 0, nq = 0;
  std::vector<double> xq, wq, xn;
  std::vector<double> N;   // nq x np
  std::vector<double> D;   // nq x np
  std::vector<double> Dt;  // nq x nq
  std::vector<double> Nf;  // folded: N(a,i) sqrt(w_a)
  std::vector<double> Dtf; // folded: Dt(a,b) sqrt(w_a / w_b)
};
Tables1D make_tables(int p, int q);

int validate_mesh(const mf_box_mesh* m);
int64_t nodes_per_dir(const mf_box_mesh& m, int p, int d);
void lin_matrix(const mf_box_mesh& m, double L[9]);

// --------------------------------------------------------------- operator
// Structured node grid of a box mesh: cells n[], nodes N[] per direction,
// degree p; node numbers follow from index arithmetic (periodic wrap when
// N = n p, boundary nodes constrained when dirichlet).
struct GridDesc {
  int n[3];
  int N[3];
  int p;
  int dirichlet;
};

// One set I of hanging-node constraints (Sec. 3.2.2): slaves [s0, s0+ns) and
// masters [m0, m0+nm) of the operator's index array, W_I row-major at w0.
struct ConstraintSet {
  int32_t s0, ns, m0, nm;
  int64_t w0;
};

struct Operator {
  int device = 0;
  int p = 0, q = 0, np = 0, nq = 0;
  int64_t ncells = 0, ndofs = 0;
  double mu = 0.0, sigma = 0.0;
  // device arrays
  int64_t nodes[3] = {0, 0, 0};  // nodes per direction of the full numbering
  GridDesc grid{};
  bool box = false;           // every cell axis-aligned: diagonal 3x3 factor
  int cfg = 0;                // launch shape of the box kernel set by mf_set_launch (-1: none)
  int mcfg = -1;              // launch shape of the mixed-precision kernel (-1: none)
  // shapes chosen by mf_tune, per (precision, columns); used when no shape is set
  std::map<std::pair<int, int>, int> tuned;
  std::map<std::pair<int, int>, std::vector<double>> tuned_ms;  // median ms per shape (-1: not timed)
  int32_t* d_map = nullptr;   // E x np^3, -1 = constrained
  int32_t* d_order = nullptr; // E: processing order of the cells
  // deterministic assembly (mf_set_deterministic): the cells sorted by colour
  // (cells of one colour share no node), colour c at [coff[c], coff[c+1])
  bool deterministic = false;
  int32_t* d_colour_order = nullptr;
  std::vector<int64_t> coff;
  double* d_geo = nullptr;    // E x 6: mu det J (J^-1 J^-T), (00,01,02,11,12,22)
  double* d_vq = nullptr;     // E x nq^3: det J (V + sigma)
  double* d_dtab = nullptr;   // 1D sums of the diagonal (nq np + 3 np)
  double detj = 0.0;          // det J of every cell (the cell map is affine and uniform)
  double wgll[kMaxP + 1] = {};  // GLL weights of the np nodes (lumped mass)
  Tables1D t;
  // hanging-node constraints of a refined mesh (mf_create_refined_operator):
  // the grid fields above do not describe it, so the grid-based calls refuse it
  bool refined = false;
  bool map_box = false;       // refined and every cell axis-aligned: the map-based box kernel
  int64_t nsets = 0;
  int max_slaves = 0, max_masters = 0;
  ConstraintSet* d_sets = nullptr;
  int32_t* d_cidx = nullptr;  // slave and master node indices (-1: zero-Dirichlet master)
  double* d_cw = nullptr;     // the W_I, concatenated
  int32_t* d_zrows = nullptr; // rows that are not cell-interior (the map kernel's zero fill)
  double* d_detj = nullptr;   // det J per cell (refined meshes: cells of two sizes)
  int64_t nzrows = 0;
  // optional per-launch timing (diagnostics): event triples around the zero
  // fill and the fused kernel of each apply, in a ring
  std::vector<hipEvent_t> ev;
  int ev_slots = 0, ev_next = 0, ev_count = 0;
};

// ----------------------------------------------------------------- kernels
struct ApplyLaunch {
  GridDesc grid;
  const int32_t* map;
  const int32_t* order;
  const double* geo;
  const double* vq;
  const double* X;
  double* Y;
  int64_t ldx, ldy;
  int64_t ncells;
  int nvec;
  int vtile;    // vectors per workgroup tile (general kernel)
  int threads;  // workgroup size (general kernel)
  int cfg;      // launch shape index (box kernel)
  bool accumulate;
};

// Arguments of a fused Chebyshev filter step, Out := a D A (D Y) + b Y + c Xp.
struct ChebArgs {
  const double* D;   // M^{-1/2} per row (0 on constrained rows)
  const double* Xp;  // may be NULL (c ignored); may equal Out
  double a, b, c;
};
hipError_t launch_apply_cheb(const Operator& op, const double* Y, double* Out, int64_t ld,
                             int nvec, const ChebArgs& ca, hipStream_t s);
// Face rows of Out := b Y + c Xp (0 on constrained rows): the part of a
// Chebyshev step that the apply's atomics add to.
hipError_t launch_cheb_init(const Operator& op, const double* Y, const double* Xp, double* Out,
                            int64_t ld, int nvec, double b, double c, hipStream_t s);
// out[node] := GLL-lumped mass diagonal (or its inverse square root, 0 on
// constrained rows).
hipError_t launch_gll_mass(const Operator& op, int inv_sqrt, double* out, hipStream_t s);

// One operator of a batch, as the persistent kernel sees it (device array).
struct BatchOp {
  const int32_t* map;
  const int32_t* order;
  const double* geo;
  const double* vq;
  int64_t item_begin;  // first work item of this operator in the batch's list
  int64_t ncells;
  int ntiles;          // column tiles
  int64_t plane_begin;  // first node plane gz of this operator in the batch's zero fill
  GridDesc grid;
  int p;
  int nodes[3];
};
// Per-call multivector pointers, passed by value in the kernel arguments.
struct BatchPtrs {
  const double* X[kMaxBatch];
  double* Y[kMaxBatch];
  int64_t ldx[kMaxBatch];
  int64_t ldy[kMaxBatch];
  int nvec[kMaxBatch];
};
// bounds: kXcds + 1 item indices; XCD x runs the items [bounds[x], bounds[x+1]).
// item_op[item]: index into ops of the operator that owns work item `item`.
hipError_t launch_batched(int prec, int bcfg, const BatchOp* ops, const uint8_t* item_op,
                          const int64_t* bounds, const BatchPtrs& ptrs, int grid, hipStream_t s);
int batched_blocks_per_cu(int prec, int bcfg);
hipError_t launch_batched_kind_any(int prec, int p, bool loop, const BatchOp* ops,
                                   const uint8_t* item_op,
                                   const int64_t* bounds, const BatchPtrs& ptrs, int grid,
                                   hipStream_t s);
int batched_kind_blocks_per_cu(int prec, int p);
// Batched shared-row zero fill (a kernel, graph-capturable) of the node
// planes [first, first + planes) of the concatenated gz planes of the batch;
// plane_op[plane]: the operator that owns that plane.
hipError_t launch_batch_zero(const BatchOp* ops, const uint8_t* plane_op, const BatchPtrs& ptrs,
                             int64_t first, int64_t planes, hipStream_t s);

// Hanging-node constraints: X_S := W X_M (distribute) and Y_M += W^T Y_S,
// Y_S := 0 (condense) over all sets of a refined operator.
hipError_t launch_constraints_distribute(const Operator& op, double* X, int nvec, int64_t ld,
                                         hipStream_t s);
hipError_t launch_constraints_condense(const Operator& op, double* Y, int nvec, int64_t ld,
                                       hipStream_t s);
// The body of mf_apply / mf_apply_add.
int apply_dispatch(mf_operator* handle, const double* X, double* Y, int nvec, int64_t ldx,
                   int64_t ldy, int prec, void* stream, bool accumulate);
// GLL-lumped mass of a refined operator over its map (every cell, hanging
// rows included; the caller condenses it with C^T).
hipError_t launch_gll_mass_map(const Operator& op, double* out, hipStream_t s);
// out[i] := m[i] > 0 ? m[i]^{-1/2} : 0 for i < n.
hipError_t launch_inv_sqrt(double* m, int64_t n, hipStream_t s);
// W[i*nvec + j] := D[i] Y[i*ld + j].
hipError_t launch_scale_rows(int64_t n, int nvec, const double* D, const double* Y, int64_t ld,
                             double* W, hipStream_t s);
// Out[i*ld + j] := D[i] == 0 ? 0 : a D[i] V[i*nvec + j] + b Y[i*ld + j] + c Xp[i*ld + j]
// (Xp may be NULL or Out itself).
hipError_t launch_cheb_combine(int64_t n, int nvec, const double* D, const double* V,
                               const double* Y, const double* Xp, double* Out, int64_t ld,
                               double a, double b, double c, hipStream_t s);
// Y[rows[i]][0 .. ncols) := 0 for i < n (a kernel, graph-capturable).
hipError_t launch_zero_listed_rows(double* Y, const int32_t* rows, int64_t n, int ncols, int64_t ld,
                                   hipStream_t s);
// mu det J J^-1 J^-T of an affine cell with J = L diag(h / 2), as the six
// entries (00, 01, 02, 11, 12, 22); returns det J.
double cell_factor(const double L[9], const double h[3], double mu, double G6[6]);

// FP64 fused apply of axis-aligned cells through the cell-to-node map (one
// instantiation per degree; dispatcher below).
template <int P>
hipError_t launch_apply_box_map_p(const Operator& op, const ApplyLaunch& a, hipStream_t s);
hipError_t launch_apply_box_map(const Operator& op, const ApplyLaunch& a, hipStream_t s);
// The same with FP32 cell arrays (MF_FP32 on a refined operator).
template <int P>
hipError_t launch_apply_box_map32_p(const Operator& op, const ApplyLaunch& a, hipStream_t s);
hipError_t launch_apply_box_map32(const Operator& op, const ApplyLaunch& a, hipStream_t s);

// FP64 fused apply; returns hipSuccess or the launch error.
hipError_t launch_apply_f64(const Operator& op, const ApplyLaunch& a, hipStream_t s);
// X[i] := a fixed pseudo-random value in [-1, 1) for i < n (tuner input).
hipError_t launch_fill_pattern(double* X, int64_t n, hipStream_t s);
hipError_t launch_fma_probe(int blocks, int64_t iters, double* out, hipStream_t s);
// Forget (destroy) the library's cached batches of mf_apply_batched that
// reference this operator; called when the operator is destroyed.
void batch_cache_forget(const Operator* op);
// "gfx950"-style architecture name of the current device (no feature suffix).
std::string device_arch();
// The JSON launch-shape cache of mf_tune / mf_batch_tune: a flat object of
// key -> {"cfg": shape, "ms": [...]}.  cache_lookup returns the shape or -1;
// cache_store rewrites the file (through a temporary file and a rename).
int cache_lookup(const char* path, const std::string& key);
int cache_store(const char* path, const std::string& key, int cfg, const std::vector<double>& ms);
// Zero rows [0, nrows) x columns [0, ncols) of a row-major array with stride ld.
hipError_t launch_zero_rows(double* Y, int64_t nrows, int ncols, int64_t ld, hipStream_t s);
// Zero the rows of nodes on cell faces (some grid index a multiple of p) of an
// Nx x Ny x Nz node grid: the rows the box kernel assembles with atomics.
hipError_t launch_zero_shared_rows(double* Y, const int64_t nodes[3], int p, int ncols, int64_t ld,
                                   hipStream_t s);
// FP64 fused apply for box cells.
hipError_t launch_apply_box(const Operator& op, const ApplyLaunch& a, hipStream_t s);
// FP64 matrix-core body (shape 10: 8 columns per item).
hipError_t launch_apply_mfma(const Operator& op, const ApplyLaunch& a, hipStream_t s);
bool apply_box_supported(int p, int q, int cfg);
// Mixed-precision (FP32 / BF16 matrix-core) apply for box cells.
hipError_t launch_apply_mixed(const Operator& op, const ApplyLaunch& a, int prec, hipStream_t s);
bool apply_mixed_supported(int p, int q, int cfg);
int choose_cfg_mixed(int np, int nq, int nvec, int prec);
int choose_cfg_box(int np, int nq, int nvec);
// block-CG building blocks (solver.hip)
hipError_t launch_diagonal(const Operator& op, const double* d_tab, double* diag, hipStream_t s);
hipError_t launch_col_dots(int64_t n, int k, const double* A, int64_t lda, const double* B,
                           int64_t ldb, double* out, hipStream_t s);
hipError_t launch_axpby(int64_t n, int k, double a, const double* X, int64_t ldx, double b,
                        double* Y, int64_t ldy, hipStream_t s);
int64_t gram_blocks(int64_t n);
// Row chunks of a Gram block on the matrix cores (gram_blocks(n), <= 512),
// the chunk length, and the launches: partial products work[b][i k + j] of the
// rows of chunk b, and Y := beta Y + alpha P M (blas64.hip).
int64_t gram_chunks(int64_t n);
int64_t gram_partial_rows(int64_t n, int64_t nb);
hipError_t launch_gram_partial(int64_t n, int k, const double* A, int64_t lda, const double* B,
                               int64_t ldb, int64_t nb, double* work, hipStream_t s);
// Two Gram blocks with the same left operand, A^T B1 and A^T B2, in one pass
// over A (gram2_chunks(n) row chunks, each a workgroup of eight wavefronts).
int64_t gram2_chunks(int64_t n);
hipError_t launch_gram2_partial(int64_t n, int k, const double* A, int64_t lda, const double* B1,
                                int64_t ldb1, const double* B2, int64_t ldb2, int64_t nb,
                                double* work1, double* work2, hipStream_t s);
// npart non-NULL: also the per-workgroup squared column norms of the new Y,
// npart[w k + j] for the update_workgroups(n) workgroups (only where
// update_in_lds(k, kp); hipErrorInvalidValue otherwise).
hipError_t launch_block_update(int64_t n, int k, int kp, double alpha, const double* P,
                               int64_t ldp, const double* M, int ldm, double beta, double* Y,
                               int64_t ldy, hipStream_t s, double* npart = nullptr);
bool update_in_lds(int k, int kp);
int64_t update_workgroups(int64_t n);
hipError_t launch_gram_reduce(int k, int nb, const double* work, double alpha, double beta,
                              double* C, int ldc, hipStream_t s);
// C[i / cols][i % cols] := alpha sum_b work[b rows cols + i] + beta C[..]
// (i < rows cols), summed in a fixed order (solver.hip).
hipError_t launch_chunk_sum(int rows, int cols, int nb, const double* work, double alpha,
                            double beta, double* C, int ldc, hipStream_t s);
hipError_t launch_jacobi(int64_t n, int k, const double* diag, const double* R, int64_t ldr,
                         double* Z, int64_t ldz, hipStream_t s);
hipError_t launch_spd_solve(int k, int m, const double* G, const double* S, double* X, int* status,
                            hipStream_t s);
int spd_max_k();
int eig_max_k();
hipError_t launch_sym_eig(int k, const double* A, int64_t lda, double* w, double* V, int64_t ldv,
                          double vpow, int* status, hipStream_t s);
// the skip block's eigenvalue floor (mlp.hip): A = (S + S^T) / 2 in FP64, and
// S = Sbf = V max(w, floor) V^T, floor = -1 + margin + 2^-8 (||w|| + sqrt(F))
hipError_t launch_skip_sym(int F, const float* S, int64_t lds, double* A, hipStream_t s);
hipError_t launch_skip_rebuild(int F, const double* V, const double* w, double margin, float* S,
                               int64_t lds, uint16_t* Sbf, int64_t ldsb, hipStream_t s);
// block Jacobi for 64 < k <= eig_blocked_max_k() (eig.hip)
int eig_blocked_max_k();
int64_t sym_eig_blocked_work(int k);
hipError_t launch_sym_eig_blocked(int k, const double* A, int64_t lda, double* w, double* V,
                                  int64_t ldv, double vpow, int* status, double* work,
                                  hipStream_t s);
// learned-preconditioner kernels (mlp.hip)
struct GemmEpi {  // epilogue of the BF16 matrix-core GEMM (see mfmlp.h)
  const float* bias;
  int relu;
  const uint16_t* mask;
  int64_t ldmask;
  float* out_f32;
  int64_t ld_f32;
  int atomic;
  uint16_t* out_bf16;
  int64_t ld_bf16;
  int kb;  // > 0: B and the outputs in the cell-blocked layout of block width kb
};
hipError_t launch_gemm_bf16(int M, int N, int K, bool ta, bool tb, const uint16_t* A, int64_t lda,
                            const uint16_t* B, int64_t ldb, int kchunk, const GemmEpi& ep,
                            hipStream_t s);
hipError_t launch_cell_gather(const Operator& op, int k, const double* R, int64_t ldr,
                              const double* E, int64_t lde, int Fp, uint16_t* X0t, float* Tt,
                              int64_t ldx, float* rho, int pou_sqrt, const double* dsc,
                              int blocked, hipStream_t s);
hipError_t launch_cell_scatter(const Operator& op, int k, const float* Yt, int64_t ldy,
                               const float* rho, const double* diag, const double* R, int64_t ldr,
                               double* Z, int64_t ldz, int pou_sqrt, const double* dsc,
                               int blocked, hipStream_t s);
hipError_t launch_symmetrize(int n, float* S, int64_t ld, uint16_t* Sbf, hipStream_t s);
hipError_t launch_mse_grad(int F, int Fp, int64_t nrows, const float* Yt, const float* Tt,
                           int64_t ld, const float* roww, float scale, uint16_t* dYt, double* loss,
                           hipStream_t s);
hipError_t launch_row_sums(int M, int64_t N, const uint16_t* X, int64_t ld, float* out,
                           bool accumulate, hipStream_t s);
hipError_t launch_adam(int64_t n, float* w, const float* g, float* m1, float* m2, uint16_t* wbf,
                       float lr, float b1, float b2, float eps, int step, hipStream_t s);
hipError_t launch_to_bf16(int64_t n, const float* src, uint16_t* dst, hipStream_t s);
hipError_t launch_fill_f32(float* v, int64_t n, float x, hipStream_t s);


// Launch facts of one kernel on the current device: the dynamic-LDS limit is
// raised to `lds` when it exceeds 64 KiB, and the resident workgroups per CU
// (at nt threads and lds bytes) and the CU count are queried.  Cached per
// (kernel, device) under a lock, so host threads driving different devices or
// handles see their own device's values.
struct KernelFacts {
  int per_cu = 1;
  int cus = 1;
};
hipError_t kernel_facts(const void* kernel, int nt, size_t lds, KernelFacts& out);

// Two-column (16-byte) accesses need even nvec and leading dimensions and
// 16-byte aligned multivectors.
inline bool box_pairs_ok(const double* X, const double* Y, int nvec, int64_t ldx, int64_t ldy) {
  return nvec % 2 == 0 && ldx % 2 == 0 && ldy % 2 == 0 &&
         reinterpret_cast<uintptr_t>(X) % 16 == 0 && reinterpret_cast<uintptr_t>(Y) % 16 == 0;
}
// Processing order of the cells: 8 blocks by recursive bisection (one per XCD),
// Morton order inside each block.
std::vector<int32_t> cell_order(const int n[3]);
// Cell colours for the deterministic assembly: per direction cx mod 2, and 2
// for the last cell of a periodic direction with an odd count n >= 3; colour
// = c0 + 3 (c1 + 3 c2).  Fails (empty) for a periodic direction with n = 1.
std::vector<int> cell_colours(const int n[3], const bool periodic[3]);
bool apply_f64_supported(int p, int q);
// Vectors per workgroup tile of the FP64 kernel (256 threads, LDS within 64 KiB).
int choose_vtile_f64(int np, int nq, int nvec);

}  // namespace mf
