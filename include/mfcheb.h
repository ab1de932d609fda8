/* libmfmv: the Chebyshev-filter building blocks of subspace iteration for the
 * eigenproblem H U = M U Lambda (eq. ghep), in its standard form
 *   H~ U~ = U~ Lambda,  H~ = M^{-1/2} H M^{-1/2},  U~ = M^{1/2} U  (eq. shep),
 * with M the mass matrix lumped by the Gauss-Lobatto-Legendre rule of the
 * element's own nodes (diagonal), and H the operator of mf_create_operator.
 * The filter of Alg. ChFSi repeats X := alpha1 H~ Y + alpha2 X - c alpha1 Y;
 * mf_cheb_step evaluates one such step in one fused pass over the cells.
 * Multivectors are dof-major (row i, column j at X[i*ld + j]), device memory;
 * calls are stream-ordered on `stream` (hipStream_t, NULL = default),
 * allocate nothing and return MF_OK or a negative mf_status (message in
 * mf_last_error()).  Axis-aligned cells only (MF_ERR_UNSUPPORTED otherwise).
 */
#ifndef MFCHEB_H
#define MFCHEB_H

#include <stdint.h>

#include "mfmv.h"

#ifdef __cplusplus
extern "C" {
#endif

/* out[i] := m_i, the GLL-lumped mass of node i (sum over the cells holding
 * the node of w_a w_b w_c det J, w the GLL weights of the element's nodes,
 * Sec. Helmholtz eigenvalue problem), or m_i^{-1/2} when inv_sqrt != 0;
 * constrained rows get 0.  out: device, mf_num_dofs entries.  On an operator
 * of mf_create_refined_operator: m_c = C^T m_u, the mass lumped by rows on the
 * constrained space (0 on hanging rows; see include/mfrefine.h).  Errors:
 * MF_ERR_ARG (NULL), MF_ERR_UNSUPPORTED (sheared cells of a uniform mesh),
 * MF_ERR_HIP. */
int mf_gll_mass(mf_operator* op, int inv_sqrt, double* out, void* stream);

/* Out := a D H (D Y) + b Y + c Xp, one step of the Chebyshev filter of
 * Alg. ChFSi on H~ = D H D (D = M^{-1/2} from mf_gll_mass with inv_sqrt,
 * device, one entry per row, 0 on constrained rows).  Y, Xp, Out: ndofs x
 * nvec, common leading dimension ld >= nvec.  Xp may be NULL (the c term is
 * dropped) and may be Out itself (the in-place recurrence of Alg. ChFSi);
 * Out must not overlap Y or D.  Constrained rows of Out are written 0.
 * Errors: MF_ERR_ARG (NULL, nvec < 1, ld < nvec, overlap), MF_ERR_UNSUPPORTED
 * (sheared cells), MF_ERR_HIP. */
int mf_cheb_step(mf_operator* op, const double* D, const double* Y, const double* Xp, double* Out,
                 int nvec, int64_t ld, double a, double b, double c, void* stream);

/* Symmetric eigen-decomposition of a k x k block, 1 <= k <= 2048 (the
 * Rayleigh-Ritz and orthogonalisation steps of Alg. ChFSi, whose block holds
 * the wanted vectors plus a buffer: Sec. 4 runs a thousand and more):
 * A = V diag(w) V^T with w ascending and V's columns orthonormal.  k <= 64: the
 * cyclic Jacobi method in one workgroup (work unused, may be NULL).  k > 64:
 * the two-sided block Jacobi method (blocks of 32, k padded to a multiple of
 * 64; each round one Jacobi sweep per block pair, then the pairs' rotations
 * applied to the whole block and to V), in `work`, a caller-owned device
 * array of at least mf_sym_eig_work(k) doubles (contents undefined after).
 * The whole run is enqueued on the stream; the host never waits.
 * A: row-major k x k (lda >= k), only read; w: k entries; V: row-major k x k
 * (ldv >= k), V[i*ldv + j] = component i of eigenvector j.  With vpow != 0
 * every column j is scaled by w_j^vpow (vpow = -1/2: V diag(w)^{-1/2}, the
 * orthonormalising factor of a Gram block).  *status (device int): 0
 * converged (off-diagonal norm <= 1e-14 of the block's); 1 not converged in
 * 40 sweeps (results are the last iterate); 2 vpow != 0 and some w_j <= 0.
 * w, V and work must not overlap A or each other.  Errors: MF_ERR_ARG (NULL,
 * ld < k, overlap, short work), MF_ERR_UNSUPPORTED (k < 1 or k > 2048),
 * MF_ERR_HIP. */
int mf_sym_eig(int k, const double* A, int64_t lda, double* w, double* V, int64_t ldv,
               double vpow, int* status, double* work, int64_t work_len, void* stream);

/* Doubles of work mf_sym_eig needs for a k x k block (0 for k <= 64), or -1
 * for k outside 1..2048.  About 2 k^2. */
int64_t mf_sym_eig_work(int k);

#ifdef __cplusplus
}
#endif

#endif /* MFCHEB_H */
