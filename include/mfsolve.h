/* libmfmv: building blocks of the block-CG solve of A X = B (A from
 * mfmv.h, X and B multivectors of k columns) and of its Jacobi fallback
 * preconditioner.
 *
 * All multivectors are dof-major FP64 device arrays: column j of row i at
 * V[i * ld + j], ld >= k.  Every call is stream-ordered and asynchronous on
 * `stream` (a hipStream_t, NULL = the default stream), allocates nothing and
 * returns MF_OK or a negative mf_status (message in mf_last_error()).
 * Arguments are checked on the host: NULL pointers, n < 0, k < 1, ld < k
 * give MF_ERR_ARG; a failing HIP launch gives MF_ERR_HIP.  With
 * n = 0 the multivector pointers may be NULL (no rows to touch).
 */
#ifndef MFSOLVE_H
#define MFSOLVE_H

#include <stdint.h>

#include "mfmv.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Diagonal of the operator for point-Jacobi preconditioning of block CG: for
 * every free dof i, diag[i] = A_ii = sum_e A^(e)_ii, the diagonal of the
 * element matrices of eq. stiffnessmatinteg / eq. massmatinteg (with the
 * potential and sigma) assembled over the cells that share i; constrained
 * (Dirichlet) rows get 1.  On the affine cells of a box mesh the 3x3 factor G
 * of eq. sjacobian is constant per cell, so the stiffness part separates into
 * 1D sums of the folded basis and derivative tables (Sec. 3.2.4); the
 * potential part sums det J (V + sigma) N_I^2 over the cell's quadrature
 * points.  `diag` is a device array of mf_operator_info's ndofs entries owned
 * by the caller.  Errors: MF_ERR_ARG (NULL), MF_ERR_HIP. */
int mf_diagonal(mf_operator* op, double* diag, void* stream);

/* C := alpha * A^T B + beta * C, the k x k Gram block of two n x k
 * multivectors (block CG: P^T A P, P^T R, (A P)^T Z).  C is row-major with
 * leading dimension ldc >= k, on the device; with beta = 0 its old contents
 * are ignored.  Two stages: partial products of row chunks (FP64 matrix-core
 * kernel, 16 x 16 x 4 products over 128 x 128 blocks of C) into `work` (a
 * caller-owned device array of at least mf_block_gram_work(n, k) doubles,
 * contents undefined afterwards), then their reduction into C in a fixed
 * order (the result does not depend on scheduling).  C and work must not overlap each other or A, B.
 * Errors: MF_ERR_ARG (also for a short or overlapping work array),
 * MF_ERR_HIP. */
int mf_block_gram(int64_t n, int k, const double* A, int64_t lda, const double* B, int64_t ldb,
                  double alpha, double beta, double* C, int ldc, double* work, int64_t work_len,
                  void* stream);

/* mf_block_gram without a work array, for callers that cannot allocate
 * (code under HIP graph capture, serving loops, harnesses that forbid
 * allocation): the partial products go to a device array of the library's
 * own (512 chunks x 128 x 128 doubles, 64 MiB, held on every GPU the library
 * runs on until the process ends).  k <= 128.  No allocation and no host
 * synchronisation; calls that overlap in time on one GPU share the array and
 * race.  Same result as mf_block_gram (same kernels, same chunking).
 * Errors: MF_ERR_ARG (NULL, n < 0, k < 1, ld < k, C overlapping A or B),
 * MF_ERR_UNSUPPORTED (k > 128), MF_ERR_HIP. */
int mf_block_gram_noalloc(int64_t n, int k, const double* A, int64_t lda, const double* B,
                          int64_t ldb, double alpha, double beta, double* C, int ldc, void* stream);

/* Number of doubles the work array of mf_block_gram needs for n rows and k
 * columns (at most 512 k^2), or -1 for n < 0 or k < 1. */
int64_t mf_block_gram_work(int64_t n, int k);

/* The two Gram blocks of a block-CG step that share their left operand,
 * C1 := alpha * A^T B1 + beta * C1 and C2 := alpha * A^T B2 + beta * C2 (P^T (A P)
 * and P^T R, the blocks of the step length alpha = (P^T A P)^{-1} P^T R), in
 * one pass over A: each row of A is fetched from HBM once for both products
 * (one workgroup of eight wavefronts per row chunk, four per product).  Each
 * product is formed and reduced as by mf_block_gram (fixed summation order);
 * `work` is a caller-owned device array of at least mf_block_gram2_work(n, k)
 * doubles, contents undefined afterwards.  C1, C2 and work must not overlap
 * each other or A, B1, B2.  Errors: MF_ERR_ARG (NULL, n < 0, k < 1, ld < k,
 * short or overlapping arrays), MF_ERR_HIP. */
int mf_block_gram2(int64_t n, int k, const double* A, int64_t lda, const double* B1, int64_t ldb1,
                   const double* B2, int64_t ldb2, double alpha, double beta, double* C1,
                   int ldc1, double* C2, int ldc2, double* work, int64_t work_len, void* stream);

/* Number of doubles the work array of mf_block_gram2 needs for n rows and k
 * columns (at most 512 k^2), or -1 for n < 0 or k < 1. */
int64_t mf_block_gram2_work(int64_t n, int k);

/* Y := beta * Y + alpha * P M, with P an n x kp multivector (ldp), M a kp x k
 * row-major device matrix (ldm >= k) and Y n x k (ldy).  Y must not overlap P
 * or M.  Block-CG updates X += P alpha, R -= (A P) alpha, Z += P beta.  An
 * FP64 matrix-core kernel (16 rows x 128 columns of Y per wavefront).
 * Errors: MF_ERR_ARG (also for overlap), MF_ERR_HIP. */
int mf_block_update(int64_t n, int k, int kp, double alpha, const double* P, int64_t ldp,
                    const double* M, int ldm, double beta, double* Y, int64_t ldy, void* stream);

/* mf_block_update that also returns the squared 2-norms of the columns of the
 * updated Y: norms2[j] := sum_i Y[i*ldy + j]^2 (block CG: R -= (A P) alpha
 * together with the residual norms of its convergence test, without a second
 * pass over R).  The norms are summed from the values as stored, per
 * workgroup into `work` (a caller-owned device array of at least
 * mf_block_update_norms_work(n, k) doubles, contents undefined afterwards),
 * then over the workgroups in a fixed order.  `norms2` is a device array of k
 * doubles; n = 0 gives zeros.  Y, norms2 and work must not overlap each
 * other or P, M.  Errors: MF_ERR_ARG (NULL, bad sizes, short or overlapping
 * arrays), MF_ERR_UNSUPPORTED (k > 128 or kp > 128: use mf_block_update and
 * mf_col_dots), MF_ERR_HIP. */
int mf_block_update_norms(int64_t n, int k, int kp, double alpha, const double* P, int64_t ldp,
                          const double* M, int ldm, double beta, double* Y, int64_t ldy,
                          double* norms2, double* work, int64_t work_len, void* stream);

/* Number of doubles the work array of mf_block_update_norms needs for n rows
 * and k columns, or -1 for n < 0 or k < 1. */
int64_t mf_block_update_norms_work(int64_t n, int k);

/* out[j] := sum_i A[i*lda + j] B[i*ldb + j] for j < k: column dot products
 * (residual norms with A = B; the z_j^T r_j of a preconditioned residual).
 * `out` is a device array of k doubles.  Errors:
 * MF_ERR_ARG, MF_ERR_HIP. */
int mf_col_dots(int64_t n, int k, const double* A, int64_t lda, const double* B, int64_t ldb,
                double* out, void* stream);

/* Y := a X + b Y on n x k multivectors; with b = 0, Y is only written.  Y may
 * equal X (same ld) but not overlap it otherwise.  Errors: MF_ERR_ARG,
 * MF_ERR_HIP. */
int mf_axpby(int64_t n, int k, double a, const double* X, int64_t ldx, double b, double* Y,
             int64_t ldy, void* stream);

/* Z := R / diag row-wise (Z[i*ldz + j] = R[i*ldr + j] / diag[i]): the point
 * Jacobi preconditioner.  Z may equal R (same ld).  Errors: MF_ERR_ARG,
 * MF_ERR_HIP. */
int mf_jacobi(int64_t n, int k, const double* diag, const double* R, int64_t ldr, double* Z,
              int64_t ldz, void* stream);

/* X := G^{-1} S for a symmetric positive definite k x k block G and a k x m
 * block S (row-major, leading dimensions k and m, device): Cholesky
 * factorisation and two triangular solves, one workgroup per 64 columns of S,
 * the k x k step of block CG (alpha = (P^T A P)^{-1} P^T R).  G and S are not modified; X must
 * not overlap them.  If a pivot is not positive (G not numerically SPD),
 * *status (device int) is set to that pivot's index + 1 and X is left
 * unspecified; otherwise *status = 0.  Errors: MF_ERR_ARG (NULL, k < 1,
 * m < 1), MF_ERR_UNSUPPORTED (k > 128 or m > 256), MF_ERR_HIP. */
int mf_spd_solve(int k, int m, const double* G, const double* S, double* X, int* status,
                 void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MFSOLVE_H */
