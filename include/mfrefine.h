/* libmfmv: once-refined box meshes with hanging-node constraints.
 *
 * A refined mesh is a coarse box mesh in which the coarse cells of the index
 * box [rlo, rhi) are each split into 2 x 2 x 2 children.  The fine nodes on
 * faces between refined and unrefined cells are "hanging": the conforming
 * space fixes their values as the unrefined neighbour's degree-p polynomial
 * at that node.  These are the hanging-node constraints of Sec. 3.2.2: locally
 * dense, stored as sets I, each with its master nodes M_I (the np^2 nodes of
 * one coarse face), its slave nodes S_I (the hanging fine nodes on that face
 * not already in an earlier set) and the dense weight matrix W_I (|S_I| x
 * |M_I|, row s holds L_a(t1) L_b(t2), the coarse face's tensor-product
 * Lagrange basis at the slave's face coordinates).  The constraints are
 * homogeneous (no inhomogeneity vector).  Zero-Dirichlet masters are
 * dropped: their values are zero.
 *
 * Numbering (full, constrained nodes included):
 *   cells: the unrefined coarse cells in lexicographic order (first index
 *          fastest), then the fine cells of the refined box, lexicographic
 *          over fine cell indices; local nodes as in mfmv.h (first index
 *          fastest, Sec. 3.2.3);
 *   nodes: the coarse lattice nodes (n p + 1 per direction) that belong to an
 *          unrefined cell, lexicographic, numbered consecutively; then every
 *          node of the refined box's fine lattice (2 (rhi - rlo) p + 1 per
 *          direction), lexicographic.  A hanging fine node is a node of its
 *          own even where it coincides with a coarse node (one master, weight 1).
 *   zero-Dirichlet nodes (bc = MF_BC_DIRICHLET0): every node on the outer
 *          boundary; such a node is never a slave.
 *
 * The operator A = mu K + M_{V+sigma} on the conforming space is
 *   Y = C^T A_u C X        (eq. AU with one partition)
 * where A_u assembles every cell with hanging nodes as ordinary rows.  With
 * the handle of mf_create_refined_operator it runs as mf_apply_constrained,
 * or as three stream-ordered calls: mf_constraints_distribute (C, in place on X), mf_apply (A_u through
 * the cell-to-node map: the box kernel's body for axis-aligned cells, the
 * general-geometry kernel for sheared cells or after mf_set_launch with
 * general != 0; zero-Dirichlet rows read as zero and written as zero) and
 * mf_constraints_condense (C^T, in place on Y).  The
 * sequence allocates nothing.  Multivectors are dof-major (row i, column j at
 * X[i*ld + j]) device arrays.  Every call returns MF_OK or a negative
 * mf_status (message in mf_last_error()).
 *
 * A refined operator supports mf_apply / mf_apply_add in MF_FP64, and in
 * MF_FP32 on axis-aligned cells (FP32 cell arrays with power-of-two
 * scaling per cell and column, the FP32 vector contractions, FP64 assembly);
 * mf_gll_mass gives the constrained lumped mass (see
 * mf_cheb_step_constrained); the calls built on the uniform grid
 * (mf_diagonal, mf_cheb_step, mf_cell_gather / mf_cell_scatter, batches,
 * BF16) return MF_ERR_UNSUPPORTED for it.
 */
#ifndef MFREFINE_H
#define MFREFINE_H

#include <stdint.h>

#include "mfmv.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    mf_box_mesh coarse;       /* bc: MF_BC_NONE or MF_BC_DIRICHLET0 (periodic: unsupported) */
    int32_t rlo[3];           /* refined coarse-cell index box [rlo, rhi); 0 <= rlo <= rhi <= n; */
    int32_t rhi[3];           /* rlo[d] == rhi[d] for some d means nothing is refined */
} mf_refined_mesh;

/* Sizes of a refined mesh of degree p (host; any output may be NULL):
 * nodes of the full numbering, cells, hanging (slave) nodes, constraint sets.
 * Errors: MF_ERR_ARG (NULL mesh, invalid coarse mesh or refined box),
 * MF_ERR_UNSUPPORTED (p outside [1, 10], periodic, more than 2^31-1 nodes). */
int mf_refined_sizes(const mf_refined_mesh* mesh, int p, int64_t* ndofs, int64_t* ncells,
                     int64_t* nslaves, int64_t* nsets);

/* The cell-to-node map (host, caller-owned, ncells x (p+1)^3 int32, full
 * numbering, no -1 entries) and the node kinds (host, ndofs bytes: 0 free,
 * 1 zero-Dirichlet, 2 hanging).  Either pointer may be NULL.  Errors as for
 * mf_refined_sizes. */
int mf_refined_layout(const mf_refined_mesh* mesh, int p, int32_t* map, uint8_t* kind);

/* Physical coordinates of the q^3 Gauss points of every cell, in the cell
 * order above (host, caller-owned, ncells*q^3*3 doubles, first direction
 * fastest, xyz innermost): where V is tabulated for mf_create_refined_operator
 * (eq. mjacobian).  Errors: MF_ERR_ARG, MF_ERR_UNSUPPORTED (q out of range). */
int mf_refined_quad_points(const mf_refined_mesh* mesh, int q, double* xq);

/* Build the operator on a refined mesh: the data of mf_create_operator (map
 * with zero-Dirichlet nodes as -1, per-cell 3x3 factor and per-point det J
 * (V + sigma) for cells of two sizes, weight-folded 1D tables) plus the
 * constraint sets (slave and master indices, W_I), copied to the current
 * device once.  Vq: host, ncells*q^3 values at the points of
 * mf_refined_quad_points, NULL for V = 0.  Release with mf_destroy_operator.
 * Errors: MF_ERR_ARG (NULL, invalid mesh, non-finite input), MF_ERR_UNSUPPORTED
 * (p, q, periodic, size), MF_ERR_OOM, MF_ERR_HIP. */
int mf_create_refined_operator(const mf_refined_mesh* mesh, int p, int q, double mu,
                               const double* Vq, double sigma, mf_operator** out);

/* Y := C^T A_u C X, the constrained product of eq. AU, in one call: the three
 * steps above, in order on `stream`.  X (ldx >= nvec) is in/out: its hanging rows are
 * overwritten with C X; Y (ldy >= nvec) is overwritten (hanging and
 * zero-Dirichlet rows 0).  X and Y must not overlap.  FP64.  On an operator
 * of mf_create_operator it is mf_apply.  Allocates nothing.  Errors:
 * MF_ERR_ARG (NULL, nvec < 1, ld < nvec, overlap), MF_ERR_UNSUPPORTED (nvec
 * above 4,194,240), MF_ERR_HIP. */
int mf_apply_constrained(mf_operator* op, double* X, double* Y, int nvec, int64_t ldx,
                         int64_t ldy, void* stream);

/* One step of the Chebyshev filter of Alg. ChFSi on the constrained space of a
 * refined mesh: Out := a D C^T A_u C (D Y) + b Y + c Xp on rows with D != 0,
 * 0 on the others.  D = m_c^{-1/2} from mf_gll_mass(op, 1, ...), which on a
 * refined operator lumps the constrained mass by rows: m_c = C^T m_u, m_u the
 * GLL-lumped mass of every cell (every row of C sums to one), so D is 0 on
 * hanging and zero-Dirichlet rows.  Y, Xp, Out: ndofs x nvec, leading
 * dimension ld >= nvec; Xp may be NULL (c dropped) or Out itself; Out must
 * not overlap Y or D.  work: device, 2 ndofs nvec doubles, caller-owned (the
 * scaled input and the product), overlapping nothing else.  Runs row scaling,
 * mf_apply_constrained and a combining kernel in stream order; allocates
 * nothing.  On an operator of mf_create_operator it is the same step with C
 * the identity.  Errors: MF_ERR_ARG (NULL, nvec < 1, ld < nvec, overlap),
 * MF_ERR_UNSUPPORTED, MF_ERR_HIP. */
int mf_cheb_step_constrained(mf_operator* op, const double* D, const double* Y,
                             const double* Xp, double* Out, int nvec, int64_t ld, double a,
                             double b, double c, double* work, void* stream);

/* X_S := W_I X_M for every set I: the action of C (Sec. 3.2.2), in place on
 * the slave rows of X (columns [0, nvec), row stride ld >= nvec); every other
 * row is left unchanged.  Masters are never slaves, so the sets are applied
 * concurrently.  An operator without constraint sets returns MF_OK at once.
 * Errors: MF_ERR_ARG (NULL, nvec < 1, ld < nvec), MF_ERR_HIP. */
int mf_constraints_distribute(mf_operator* op, double* X, int nvec, int64_t ld, void* stream);

/* Y_M += W_I^T Y_S, then Y_S := 0, for every set I: the action of C^T
 * (Sec. 3.2.2), in place on Y.  Masters shared by several sets accumulate
 * with FP64 atomics (summation order unspecified).  Zero-Dirichlet rows are
 * left unchanged.  Errors as for mf_constraints_distribute. */
int mf_constraints_condense(mf_operator* op, double* Y, int nvec, int64_t ld, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MFREFINE_H */
