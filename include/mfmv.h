/*
 * mfmv.h - matrix-free finite-element matrix-multivector products on MI355X.
 *
 * C ABI of libmfmv.so.  The library evaluates Y = A X for the operator
 *
 *     A = mu K + M_{V + sigma}
 *
 * on a structured hexahedral mesh, where K is the stiffness matrix and M_kappa
 * the kappa-weighted mass matrix of the paper's model problem (Sec. 2.1,
 * eq. refprob and eq. integrals), discretised with tensor-product Lagrange
 * elements of degree p on Gauss-Lobatto-Legendre nodes (eq. NTensor) and a
 * q-point Gauss rule per direction (eq. quadTensor).  X and Y are multivectors
 * of nvec columns.  The product is evaluated matrix-free by sum factorisation
 * (Sec. 2.2.2, Alg. 1 and Alg. 2, eq. helmholtz), with cell extraction and
 * assembly through the cell-to-node map (Sec. 3.2.3, eq. AU) fused into one
 * GPU launch over (cell, vector-tile) pairs (Sec. 3.1.2, eq. basempigpu).
 *
 * Conventions shared by every entry point:
 *  - Status: MF_OK (0) on success, a negative mf_status otherwise; after an
 *    error mf_last_error() returns a message (thread-local, valid until the
 *    next call on the same thread).
 *  - Node numbering ("full numbering"): nodes of the box, x fastest:
 *    node (gx, gy, gz) -> gx + Nx*(gy + Ny*gz), with N_d = n_d*p + 1, or
 *    N_d = n_d*p on a periodic mesh (nodes identified modulo N_d).  Zero
 *    Dirichlet nodes keep their numbers; they are constrained rows.
 *  - Cells are numbered x fastest; inside a cell, nodes and quadrature points
 *    are numbered with the first reference direction fastest (Sec. 3.2.3).
 *  - Multivector layout: dof-major, the nvec values of one node contiguous
 *    (the BCV layout of Sec. 3.2.1 with one batch of all columns):
 *    entry (node i, column j) is at X[i*ldx + j], ldx >= nvec.
 *  - Device pointers are hipMalloc'd memory of the device that was current
 *    when the operator was created; that device must be current at the call.
 *  - Streams are passed as `void*` holding a hipStream_t (NULL = the null
 *    stream).  Device entry points are stream-ordered and asynchronous: they
 *    enqueue work and return without synchronising, and allocate nothing.
 *  - An operator or a batch may be used from one host thread at a time (its
 *    launch settings, timing events and the batch's side streams are shared
 *    state); distinct handles are independent.
 */
#ifndef MFMV_H
#define MFMV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MF_OK = 0,
    MF_ERR_ARG = -1,          /* null pointer, bad size, aliasing, bad mesh */
    MF_ERR_UNSUPPORTED = -2,  /* degree / quadrature / precision not built */
    MF_ERR_OOM = -3,          /* device or host allocation failed */
    MF_ERR_HIP = -4           /* a HIP runtime call failed (message has hipGetErrorString) */
} mf_status;

typedef enum {
    MF_BC_NONE = 0,           /* natural boundary: no constrained nodes */
    MF_BC_DIRICHLET0 = 1,     /* zero Dirichlet on every boundary node */
    MF_BC_PERIODIC = 2        /* periodic in all three directions */
} mf_bc;

typedef enum {
    MF_FP64 = 0,  /* all arithmetic in FP64 */
    MF_FP32 = 1,  /* contractions in FP32 (vector or matrix-core shapes), FP64 assembly */
    MF_BF16 = 2,  /* contractions on the matrix cores with BF16 operands, FP32 accumulation,
                     FP64 assembly */
    /* the same two precisions under their names in the original interface
       description (FP32 runs the vector shapes unless a matrix-core shape is set) */
    MF_FP32_MFMA = MF_FP32,
    MF_BF16_MFMA = MF_BF16
} mf_precision;

/* Structured hexahedral box mesh: n[d] cells per direction on [lo, hi], then
 * the optional linear map x = lin * y (row-major 3x3) applied to every box
 * point y.  All-zero `lin` means the identity.  With a map the cells are
 * parallelepipeds and each cell Jacobian is a full 3x3 matrix; det(lin) must
 * be positive. */
typedef struct {
    int32_t n[3];
    double lo[3];
    double hi[3];
    int32_t bc;               /* mf_bc */
    double lin[9];
} mf_box_mesh;

typedef struct mf_operator mf_operator;

/* ---------------------------------------------------------------- host ---- */

/* Number of nodes of the full numbering (constrained nodes included) of a
 * degree-p mesh.  Errors: MF_ERR_ARG for a null pointer or invalid mesh,
 * MF_ERR_UNSUPPORTED for p outside [1, 10]. */
int mf_num_dofs(const mf_box_mesh* mesh, int p, int64_t* ndofs);

/* Number of cells, n[0]*n[1]*n[2]. */
int mf_num_cells(const mf_box_mesh* mesh, int64_t* ncells);

/* Physical coordinates of the q^3 Gauss points of every cell (host memory,
 * caller-owned, E*q^3*3 doubles, cell-major, first direction fastest, xyz
 * innermost).  Used to tabulate V at the points the operator integrates with
 * (eq. mjacobian: kappa is needed at every quadrature point of every cell). */
int mf_quad_points(const mf_box_mesh* mesh, int q, double* xq);

/* 1 for constrained (zero-Dirichlet) nodes, 0 otherwise; host, ndofs bytes. */
int mf_constrained_mask(const mf_box_mesh* mesh, int p, uint8_t* mask);

/* The 1D tables of the sum factorisation, unfolded (host, caller-owned):
 *   xq[q], wq[q]   Gauss points and weights on [-1, 1];
 *   xn[p+1]        GLL nodes;
 *   N[q*(p+1)]     N1D(a, i) = L_i(xq_a), row-major (quadrature point major);
 *   D[q*(p+1)]     D1D(a, i) = L_i'(xq_a);
 *   Dt[q*q]        the collocation derivative at the Gauss points,
 *                  Dt(a, b) = l_b'(xq_a) with l_b the Lagrange basis on the
 *                  Gauss points, so that D1D = Dt * N1D (eq. DU).
 * Any output pointer may be NULL.  Requires q >= p+1 (see mf_create_operator). */
int mf_basis_1d(int p, int q, double* xq, double* wq, double* xn, double* N, double* D, double* Dt);

/* -------------------------------------------------------------- device ---- */

/* Build the operator A = mu K + M_{V+sigma} for degree p, q Gauss points.
 *   Vq:    host array of E*q^3 values V(x_Q) at the points given by
 *          mf_quad_points (same order); NULL means V = 0.
 *   sigma: constant added to V (the shift of the solve "(A + sigma M) X = B").
 * Precomputes on the host (Sec. 3.2, Alg. 4 data): the cell-to-node map with
 * constrained nodes marked, the per-cell 3x3 factor mu det(J) J^-1 J^-T
 * (eq. sjacobian), the per-point factor det(J) (V + sigma) (eq. mjacobian), and
 * the weight-folded 1D matrices (Sec. 3.2.4); copies them to the current device
 * once (synchronously).  The operator owns these device copies.
 * Errors: MF_ERR_ARG (null pointer, invalid mesh, non-finite input),
 * MF_ERR_UNSUPPORTED (p outside [1, 10]; q outside [p+1, p+3] - the
 * collocation factorisation D1D = Dt N1D of eq. DU is exact only for q >= p+1),
 * MF_ERR_OOM, MF_ERR_HIP. */
int mf_create_operator(const mf_box_mesh* mesh, int p, int q, double mu, const double* Vq,
                       double sigma, mf_operator** out);

/* Release the operator's device memory.  NULL is ignored.  Work already
 * enqueued that uses the operator must have completed. */
void mf_destroy_operator(mf_operator* op);

/* Sizes of an operator (any output pointer may be NULL). */
int mf_operator_info(const mf_operator* op, int64_t* ndofs, int64_t* ncells, int* p, int* q);

/* The order in which the fused apply takes the cells of a box-mesh operator
 * (host output, ncells int32 cell indices, cell index = cx + nx (cy + ny cz)):
 * eight blocks by recursive bisection, one per XCD, Morton order inside a
 * block.  Work item i of a launch with t column tiles is (order[i / t], tile
 * i % t), and XCD x runs the contiguous items [x c, (x+1) c), c = ceil(ncells t
 * / 8) (eq. AU's sum over cells in an order of the library's choosing).
 * Diagnostic: it lets a caller find the first and last cells of each XCD's
 * range.  Errors: MF_ERR_ARG (NULL), MF_ERR_UNSUPPORTED (refined operator). */
int mf_cell_order(const mf_operator* op, int32_t* order);

/* Measured FP64 issue rate for the roofline (the analogue of rating kernels
 * against the machine's peak, Sec. 4): `blocks` workgroups of 256 threads,
 * each thread running `iters` rounds of 8 independent FP64 FMA chains (16
 * flops per thread and round, no memory traffic), then writing one double to
 * out[blocks * 256] (device, caller-owned).  Time it with events; flops =
 * blocks * 256 * iters * 16.  Errors: MF_ERR_ARG, MF_ERR_HIP. */
int mf_fma_probe(int blocks, int64_t iters, double* out, void* stream);

/* Deterministic assembly on (on != 0) or off for mf_apply / mf_apply_add of a
 * box-mesh operator.  The paper's GPU kernel adds the cell contributions to
 * shared rows with atomics (Sec. 3.2.4), so their summation order, and the
 * last bits of those rows, vary from run to run.  With this on, the cells are
 * coloured (per direction cx mod 2, the last cell of an odd periodic
 * direction a third colour; cells of one colour share no node) and the kernel
 * runs once per colour in colour order: each shared row then receives at most
 * one addition per launch and its terms are summed in a fixed order, so
 * repeated applies give bitwise equal results (for a fixed launch shape and
 * precision).  Costs up to 27 launches of fewer cells each.  The first call
 * uploads the colour-sorted cell order (device memory held until
 * mf_destroy_operator).  Errors: MF_ERR_ARG (NULL), MF_ERR_UNSUPPORTED
 * (sheared or refined operator, or a periodic direction of one cell, which
 * meets itself), MF_ERR_OOM, MF_ERR_HIP. */
int mf_set_deterministic(mf_operator* op, int on);

/* Y := A X (overwrite, never accumulate), eq. AU with one partition.
 *   X: device, ndofs rows, row stride ldx >= nvec; constrained rows are
 *      ignored (read as zero: the action of C, Sec. 3.2.2).
 *   Y: device, ndofs rows, row stride ldy >= nvec; constrained rows are
 *      written as zero (the action of C^T).  Y must not overlap X.
 *   prec: MF_FP64 evaluates every step in FP64 (FP64 atomic assembly).
 *         MF_FP32 / MF_BF16: cell arrays are FP32 and each (cell,
 *         column) is scaled by a power of two before the conversion and
 *         unscaled before the FP64 assembly; the sum-factorised contractions
 *         run on the matrix cores (FP32 or BF16 operands, FP32 accumulation)
 *         or, for FP32 by default, as FP32 vector even-odd contractions (see
 *         mf_set_launch_mixed).  Built for axis-aligned cells only.
 * Stream-ordered on `stream`; allocates nothing, does not synchronise.
 * Errors: MF_ERR_ARG (null, nvec < 1, ld < nvec, overlap), MF_ERR_UNSUPPORTED
 * (precision not available for this p, q), MF_ERR_HIP (launch failure). */
int mf_apply(mf_operator* op, const double* X, double* Y, int nvec, int64_t ldx, int64_t ldy,
             int prec, void* stream);

/* Y += A X: the accumulating form of mf_apply (same arguments and errors).
 * Constrained rows of Y are left unchanged.  mf_apply is mf_zero on Y followed
 * by this call. */
int mf_apply_add(mf_operator* op, const double* X, double* Y, int nvec, int64_t ldx, int64_t ldy,
                 int prec, void* stream);

/* Y[i*ld + j] := 0 for i < nrows, j < ncols (device, stream-ordered; a
 * kernel, not a memset, so it can be captured in a graph).
 * Errors: MF_ERR_ARG (NULL, nrows < 0, ncols < 1, ld < ncols), MF_ERR_HIP. */
int mf_zero(double* Y, int64_t nrows, int ncols, int64_t ld, void* stream);

/* Launch-shape tuning, the analogue of the paper's sweep of its GPU kernel's
 * batch size and thread-block shape (Sec. 4, GPU benchmarks,
 * tbl:batchsizeStudy).  Every launch shape built for this operator's (p, q) and
 * precision (FP64: the axis-aligned-cell shapes of mf_set_launch; FP32: the
 * mixed shapes 0..6; BF16: 0..3) is timed on device buffers of ndofs x nvec
 * (allocated and freed here: not for use under graph capture), median of 7
 * event-timed calls after 2 warm-up calls on a stream of its own, and the
 * fastest is kept for later mf_apply calls of this operator with nvec columns
 * in this precision (it takes effect unless mf_set_launch(_mixed) sets a shape:
 * mf_tune clears that setting).
 *   cache_path: a JSON file (NULL: no cache) of entries
 *     "<arch>/p<p>q<q>/cells<E>/nvec<nvec>/<fp64|fp32|bf16>":
 *       {"cfg": <shape>, "ms": [median ms per shape, -1 if not timed]};
 *   a present entry is used without timing; a new result is added by rewriting
 *   the file through a temporary file and a rename (concurrent writers from
 *   several processes may lose each other's entries, never corrupt the file).
 * Operators with a single kernel shape (general geometry, refined meshes in
 * FP64) return MF_OK without timing.  Errors: MF_ERR_ARG (NULL, nvec < 1,
 * cache not writable), MF_ERR_UNSUPPORTED (precision not built for this
 * operator), MF_ERR_OOM, MF_ERR_HIP. */
int mf_tune(mf_operator* op, int nvec, int prec, const char* cache_path);

/* The shape mf_tune chose for (nvec, prec) (-1 if none) and, if ms is not
 * NULL, its median times per shape (nms entries; -1 for shapes not timed,
 * every entry -1 when the choice came from the cache).  Errors: MF_ERR_ARG. */
int mf_tune_info(const mf_operator* op, int nvec, int prec, int* cfg, double* ms, int nms);

/* Launch selection (used by the tuner and by tests):
 *   general != 0 forces the general-geometry kernel (full 3x3 factor, three
 *                LDS buffers) even on axis-aligned cells; it cannot be undone
 *                on this operator.
 *   cfg          launch shape of the axis-aligned-cell kernel, 0..12, or -1
 *                for the built-in choice by column count.  Shapes 2 and 4 give
 *                every thread two adjacent columns (16-byte accesses); a call
 *                with odd nvec, odd ldx or ldy, or X or Y not 16-byte aligned
 *                runs the one-column shape with the same tile instead.
 *                Shapes 3, 4, 5 and 8 use a persistent grid that prefetches
 *                the next cell's X during the current cell's contractions.
 *                Shape 10 runs the contractions on the FP64 matrix cores
 *                (q = p + 1 <= 8).  Shapes 11 and 12 take 1 and 2 columns per
 *                cell with one and two wavefronts (narrow blocks).
 * Errors: MF_ERR_ARG (NULL, cfg out of range), MF_ERR_UNSUPPORTED (shape does
 * not fit the LDS for this p, q). */
int mf_set_launch(mf_operator* op, int general, int cfg);

/* Launch shape of the mixed-precision apply, 0..6, or -1 for the built-in
 * choice (by precision and column count).  0..3: matrix-core kernels (FP32 or
 * BF16 operands by the call's precision): 0 = 16 columns and 512 threads (8
 * columns if 16 exceed 80 KiB of LDS), 1 = 16 / 256, 2 = 8 / 256, 3 = 8 / 512.
 * 4..6: FP32 vector kernels (the even-odd contractions of the FP64 box kernel
 * on FP32 cell arrays, the same per-(cell, column) power-of-two scaling):
 * 4 = 16 columns, two per thread (16-byte accesses; odd nvec, odd ldx or ldy
 * or unaligned X or Y run shape 5 instead), 5 = 8 columns, 6 = 16 columns,
 * each with the fewest whole wavefronts covering the pencil tasks.  A BF16
 * call with a shape of 4..6 runs matrix-core shape 0.  The built-in choice for
 * FP32 is shape 6 (nvec > 8, where it fits 1024 threads) or 5.  Errors as
 * mf_set_launch. */
int mf_set_launch_mixed(mf_operator* op, int cfg);

/* Per-launch timing for diagnostics and benchmarks.  mf_timing(op, slots)
 * (slots > 0) makes every following mf_apply / mf_apply_add on this operator
 * record HIP events on its stream around the zero fill and around the fused
 * kernel, in a ring of `slots` entries; slots = 0 turns it off.  Not for use
 * under graph capture.  mf_timing_read waits for the recorded events and
 * returns the number of applies recorded since the last read and the summed
 * milliseconds of the zero fill and of the fused kernel; it then clears the
 * ring.  Errors: MF_ERR_ARG, MF_ERR_HIP. */
int mf_timing(mf_operator* op, int slots);
int mf_timing_read(mf_operator* op, int* count, double* zero_ms, double* kernel_ms);
/* The same events one apply at a time, oldest first: at most cap entries of
 * the zero-fill and fused-kernel milliseconds of each recorded apply (host
 * arrays), *count set to the number written; clears the ring.  Errors:
 * MF_ERR_ARG, MF_ERR_HIP. */
int mf_timing_samples(mf_operator* op, int cap, double* zero_ms, double* kernel_ms, int* count);

/* ------------------------------------------------------------- batches ---- */

/* A batch applies a list of operators, each to its own multivector,
 *     Y_i := A_i X_i,  i = 0 .. nops-1,
 * in one launch (or one per degree): the (cell, column-tile) work items of all
 * operators form one list (heaviest degree first), cut into one contiguous
 * range per XCD of equal estimated cost that the XCD's workgroups take in an
 * interleaved order; a byte table maps each item to its operator.  This is the
 * single launch over every (cell, batch) pair of eq. basempigpu widened to
 * several meshes, degrees and column counts.  Supported operators: axis-aligned
 * cells, q = p + 1, p in [2, 8] (MF_ERR_UNSUPPORTED otherwise); at most 64 per
 * batch.  The batch references the operators: they must outlive it.  */
typedef struct mf_batch mf_batch;

/* nvec[i]: columns of X_i / Y_i; prec: as mf_apply.  Allocates the work table
 * and the per-XCD item ranges on the current device.  Errors: MF_ERR_ARG,
 * MF_ERR_UNSUPPORTED, MF_ERR_HIP. */
int mf_batch_create(int nops, mf_operator* const* ops, const int* nvec, int prec, mf_batch** out);
void mf_batch_destroy(mf_batch* b);

/* Launch shape, 0..5 (see the tuner).  0..2: one persistent kernel for every
 * degree of the batch: 0 = 512 threads, FP64 tiles filling the workgroup
 * (16 columns up to 5 points per direction, else 8 within 80 KiB of LDS, else
 * 4; mixed: the largest of 16 / 8 within 80 KiB), 1 = 512 threads with FP64
 * tiles of 8 (mixed 16), 2 = 256 threads with FP64 tiles of 4 (mixed 8).
 * 3..5: one kernel per degree present, each with that degree's own tile and
 * workgroup size: 3 = resident (persistent) grids and 4 = one workgroup per
 * item, the degrees one after another with the zero fills of the later
 * degrees overlapped on a side stream; 5 = one workgroup per item, every
 * degree (its zero fill, then its kernel) on its own side stream so that the
 * degrees run concurrently.  The items of each launch are cut into one
 * contiguous range per XCD of equal estimated cost.  Side streams are the
 * batch's own (default priority), forked from and joined back into the
 * caller's stream by events, so a call is ordered on that stream as a whole
 * (also under graph capture).
 * Rebuilds the work tables (synchronous copies; may reallocate them) and drops
 * a graph captured with the previous shape (capture again before replaying). */
int mf_batch_set_launch(mf_batch* b, int cfg);

/* Y_i := A_i X_i for every operator (arrays of nops device pointers in the
 * caller's operator order; ldx / ldy may be NULL for ld = nvec).  Enqueues the
 * zero fill of every Y_i's cell-face rows (a kernel) and the apply kernel(s)
 * on `stream`; allocates nothing.  Outputs must not overlap
 * each other or any input.  Errors: MF_ERR_ARG, MF_ERR_HIP. */
int mf_batch_apply(mf_batch* b, const double* const* X, double* const* Y, const int64_t* ldx,
                   const int64_t* ldy, void* stream);

/* Capture the launches of mf_batch_apply for these X / Y into a HIP graph
 * (stream must not be NULL) and keep its executable form; mf_batch_replay then
 * launches the graph on a stream.  The graph is bound to the pointers given
 * here; capture again for other buffers.  Errors: MF_ERR_ARG, MF_ERR_HIP. */
int mf_batch_capture(mf_batch* b, const double* const* X, double* const* Y, const int64_t* ldx,
                     const int64_t* ldy, void* stream);
int mf_batch_replay(mf_batch* b, void* stream);

/* Choose the batch's launch shape: every shape 0..5 is timed on the caller's
 * buffers (Y_i overwritten) on `stream`, median of 5 event-timed calls after 2
 * warm-up calls, and the fastest set (mf_batch_set_launch).  cache_path as
 * mf_tune, with entries keyed "<arch>/batch/<precision>/" followed by every
 * operator's p, q, cells and columns in the caller's order; the choice is also
 * remembered for batches that mf_apply_batched builds in this process.  Host
 * synchronising; not for use under graph capture.  Errors: as mf_batch_apply,
 * and MF_ERR_ARG for an unwritable cache. */
int mf_batch_tune(mf_batch* b, const double* const* X, double* const* Y, const int64_t* ldx,
                  const int64_t* ldy, const char* cache_path, void* stream);

/* One call for Y_i := A_i X_i, i < nops (ld = nvec[i]; arrays in the caller's
 * order; the same requirements as mf_batch_create and mf_batch_apply).  The
 * library keeps the batch it builds for a list of operator handles, column
 * counts, precision and device (up to 8 such lists, least recently used
 * dropped; a batch is dropped when one of its operators is destroyed), with
 * the shape mf_batch_tune chose for the same key in this process, else shape
 * 0.  The first call for a list allocates the batch's tables (synchronous
 * copies); later calls only enqueue work, so they may be captured in a graph.
 * Calls from several host threads are serialised by a lock.  Errors: as
 * mf_batch_create and mf_batch_apply. */
int mf_apply_batched(int nops, mf_operator* const* ops, const double* const* X, double* const* Y,
                     const int* nvec, int prec, void* stream);

/* Work items, launch shape and grid size of the batch (outputs may be NULL). */
int mf_batch_info(const mf_batch* b, int64_t* items, int* cfg, int* grid);

/* Message of the last error on this thread ("" if none). */
const char* mf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MFMV_H */
