/* libmfmv: kernels of the learned cell-local preconditioner for block CG,
 *   Z = sum_e Q_e^T W_e f_theta(Q_e R),
 * with f_theta a small MLP (F = np^3 inputs and outputs, two hidden ReLU
 * layers, plus a symmetric linear skip), Q_e the extraction of cell e's nodes (Sec. 3.2.3) and W_e the
 * partition-of-unity weights (1 / number of cells sharing the node).  The
 * network is applied to every (cell, column) of a residual block and trained
 * on the GPU by these kernels; the method generates its own training pairs
 * (residual -> error) with the operator apply.
 *
 * Batches are feature-major: an activation block is features x rows with row
 * = e * k + j for cell e and column j of a k-column multivector, element
 * (i, row) at V[i * ld + row].  The cell-blocked layout (where a call takes
 * it) keeps each cell's features x k block contiguous: element (i, e k + j)
 * at V[e * ld + i * k + j], ld the block stride (>= features * k).  BF16 data are passed as uint16_t (the upper
 * half of an IEEE single, round to nearest even).  Every call is
 * stream-ordered on `stream` (hipStream_t, NULL = default), allocates nothing
 * and returns MF_OK or a negative mf_status (message in mf_last_error()).
 */
#ifndef MFMLP_H
#define MFMLP_H

#include <stdint.h>

#include "mfmv.h"

#ifdef __cplusplus
extern "C" {
#endif

/* C = op(A) op(B) on the matrix cores (BF16 operands, FP32 accumulation),
 * then the epilogue, for every (m, n) < (M, N):
 *   v = C[m][n] (+ bias[m]) (ReLU) (* [mask[m][n] > 0]),
 *   out_f32[m*ld_f32 + n] = v (or += v with atomic != 0), and/or
 *   out_bf16[m*ld_bf16 + n] = bf16(v).
 * A is M x K row-major (lda), or K x M when ta != 0; B is K x N row-major
 * (ldb), or N x K when tb != 0.  M, N, K, lda, ldb must be multiples of 8 and
 * A, B 16-byte aligned.  kchunk > 0 splits K into ceil(K / kchunk) ranges run
 * by separate workgroups (use with atomic != 0, no bias or ReLU, on a zeroed
 * out_f32); kchunk <= 0 takes K whole.  bias (FP32, M), mask (BF16, ldmask),
 * out_f32 and out_bf16 may be NULL (at least one output).  kb > 0 (a
 * multiple of 8 dividing N): B (tb = 0) and the outputs are in the
 * cell-blocked layout with blocks of kb columns, ldb, ld_f32, ld_bf16 being
 * the block strides (>= K kb, M kb, M kb); no mask then.  Workgroups take the
 * output tiles M-tile first, so the tiles sharing a slice of B run together.
 * Errors: MF_ERR_ARG, MF_ERR_HIP. */
int mf_mlp_gemm(int M, int N, int K, int ta, int tb, const uint16_t* A, int64_t lda,
                const uint16_t* B, int64_t ldb, int kchunk, const float* bias, int relu,
                const uint16_t* mask, int64_t ldmask, float* out_f32, int64_t ld_f32, int atomic,
                uint16_t* out_bf16, int64_t ld_bf16, int kb, void* stream);

/* Network input of every (cell, column): u_i = R[node_i][j], times sqrt(w_i)
 * (the square root of node i's partition-of-unity weight) when pou_sqrt != 0
 * and divided by sqrt(dscale[node_i]) when dscale != NULL (a positive
 * diagonal, e.g. mf_diagonal's: the network then works on the diagonally
 * scaled cell problem); rho[row] = RMS of u over the cell's F = np^3 nodes
 * (constrained nodes count as 0) and X0t[i][row] = bf16(u_i / rho) (0 when
 * rho = 0; rows F <= i < Fp zero).  With E != NULL also Tt[i][row] =
 * E[node_i][j] sqrt(dscale[node_i]) / rho (FP32; no partition weight): the
 * training target for the pair (R, E).  R and E are ndofs x k multivectors
 * (ldr, lde >= k); X0t and Tt are Fp x (ncells k) with leading dimension
 * ldx >= ncells k; rho has ncells k entries, or is NULL: then rho = 1 (no
 * normalisation, one pass over R; for a linear cell map, where the scale
 * cancels).  Fp >= F, multiple of 8.  blocked != 0: X0t and Tt in the
 * cell-blocked layout, ldx the block stride (>= Fp k).  Errors: MF_ERR_ARG,
 * MF_ERR_HIP. */
int mf_cell_gather(mf_operator* op, int k, const double* R, int64_t ldr, const double* E,
                   int64_t lde, int Fp, uint16_t* X0t, float* Tt, int64_t ldx, float* rho,
                   int pou_sqrt, const double* dscale, int blocked, void* stream);

/* Z := Z0 + sum_e Q_e^T W_e (rho * Yt): the partition-of-unity assembly of
 * the network outputs Yt (FP32, first F rows used, ldy >= ncells k) scaled
 * back by rho (1 when rho is NULL), with W_e the weights w_i (or sqrt(w_i)
 * when pou_sqrt != 0: with the same weighting of the input, a symmetric cell
 * map then gives a symmetric preconditioner), divided by sqrt(dscale[node])
 * when dscale != NULL, on top of Z0 = R / diag row-wise (the Jacobi term)
 * when diag != NULL, else Z0 = 0.  Taken node by node (each Z element summed
 * by one thread over the node's cells in a fixed order, no atomics), so the
 * result is bitwise reproducible.  blocked != 0: Yt in the cell-blocked
 * layout, ldy the block stride (>= np^3 k).  Z (ndofs x k, ldz >= k) is
 * overwritten; it must not be R.  Errors: MF_ERR_ARG, MF_ERR_HIP. */
int mf_cell_scatter(mf_operator* op, int k, const float* Yt, int64_t ldy, const float* rho,
                    const double* diag, const double* R, int64_t ldr, double* Z, int64_t ldz,
                    int pou_sqrt, const double* dscale, int blocked, void* stream);

/* Eigenvalue floor of the symmetric skip block S of the cell network, the
 * step that makes the deployed linear preconditioner
 *   z = D^-1 r + sum_e Q_e^T W_e^1/2 D^-1/2 S D^-1/2 W_e^1/2 Q_e r
 * symmetric positive definite: with the partition of unity sum_e Q_e^T W_e
 * Q_e = I on the free nodes this is D^-1/2 [sum_e Q_e^T W_e^1/2 (I + S)
 * W_e^1/2 Q_e] D^-1/2, whose smallest eigenvalue is at least that of I + S
 * (relative to D^-1).  S (F x F, FP32, row-major, ld lds) is symmetrised,
 * decomposed (mf_sym_eig: S = V diag(w) V^T) and rebuilt with its eigenvalues
 * raised to at least floor = -1 + margin + 2^-8 (||w||_2 + sqrt(F)): the
 * rebuilt block has Frobenius norm at most ||w||_2 + sqrt(F), so its BF16
 * copy differs from it by at most 2^-9 of that in 2-norm, and I + S stays
 * definite, with smallest eigenvalue above margin, after the rounding.  The
 * result, exactly symmetric, is written over S and, rounded to BF16, over Sbf
 * (ld ldsb).  work: a device array of at least mf_skip_floor_work(F) doubles;
 * *status (device int): that of mf_sym_eig.  margin >= 0.  Errors: MF_ERR_ARG
 * (NULL, ld < F, short work, margin < 0), MF_ERR_UNSUPPORTED (F < 1 or
 * F > 2048), MF_ERR_HIP. */
int mf_skip_floor(int F, float* S, int64_t lds, uint16_t* Sbf, int64_t ldsb, double margin,
                  double* work, int64_t work_len, int* status, void* stream);

/* Doubles of work mf_skip_floor needs for an F x F skip block (-1 outside
 * 1..2048). */
int64_t mf_skip_floor_work(int F);

/* Weighted squared error over rows and the first F features, w = roww[n]
 * (FP32 per row; NULL means 1):
 *   *loss += scale * sum_{i<F, n<N} w (Yt - Tt)^2   (device double, accumulated)
 *   dYt = bf16(2 scale w (Yt - Tt))                 (rows F <= i < Fp written 0)
 * scale = 1 / (sum of the weights) gives the mean over the rows that count.
 * Yt, Tt, dYt share the leading dimension ld.  Errors: MF_ERR_ARG, MF_ERR_HIP. */
int mf_mse_grad(int F, int Fp, int64_t N, const float* Yt, const float* Tt, int64_t ld,
                const float* roww, float scale, uint16_t* dYt, double* loss, void* stream);

/* out[m] = (accumulate ? out[m] : 0) + sum_{n<N} X[m*ld + n] for m < M (BF16
 * X, FP32 out): bias gradients.  Errors: MF_ERR_ARG, MF_ERR_HIP. */
int mf_row_sums(int M, int64_t N, const uint16_t* X, int64_t ld, float* out, int accumulate,
                void* stream);

/* One Adam step (step >= 1) on n FP32 parameters w with gradient g and
 * moments m1, m2 (FP32, updated); with wbf != NULL the updated parameters are
 * also written as BF16.  Errors: MF_ERR_ARG, MF_ERR_HIP. */
int mf_adam(int64_t n, float* w, const float* g, float* m1, float* m2, uint16_t* wbf, float lr,
            float beta1, float beta2, float eps, int step, void* stream);

/* S := (S + S^T) / 2 on the leading n x n block of a row-major FP32 matrix
 * (ld >= n), and the same entries of its BF16 copy Sbf (same layout; may be
 * NULL): the projection that keeps the network's linear skip block
 * symmetric after each optimizer step.  Errors: MF_ERR_ARG, MF_ERR_HIP. */
int mf_symmetrize(int n, float* S, int64_t ld, uint16_t* Sbf, void* stream);

/* dst = bf16(src) (n values); mf_fill_f32: v[i] = x.  Errors: MF_ERR_ARG,
 * MF_ERR_HIP. */
int mf_to_bf16(int64_t n, const float* src, uint16_t* dst, void* stream);
int mf_fill_f32(int64_t n, float* v, float x, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MFMLP_H */
