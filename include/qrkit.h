/*
 * qrkit.h - C ABI of the MI355X (gfx950) structured-QR Levenberg-Marquardt step solver.
 *
 * The operation (Svoboda, Cashman & Fitzgibbon, "QRkit", Section 1, Eqs. 1-2):
 * given J, b, a positive diagonal D = diag(d) and a damping lambda >= 0, return
 *
 *     p = argmin_p || [J; sqrt(lambda) D] p - [b; 0] ||_2 = (J^T J + lambda D^2)^{-1} J^T b,
 *
 * computed by QR of the augmented matrix, so the condition number of J is never
 * squared.  Two structures of J are supported:
 *
 *   block-angular  J = [ blkdiag(A_1, ..., A_K) | B ]   (Section 4.2, horizontal
 *                  concatenation of a block-diagonal part, Section 4.1, and a dense
 *                  part B; blocks of one width or of their own widths).  The damping
 *                  rows are permuted next to their blocks as in Section 5.2 (Backtrack
 *                  LM, P_r [J; sqrt(lambda) D] = QR).
 *   banded         row i of J holds w values at columns row_start[i] .. row_start[i]+w-1
 *                  (the banded class of Section 4.4), factorised by Givens rotations or
 *                  by the block-banded compact-WY steps of Section 4.4.
 * qrk_discover_* find the row and column permutations of Section 4.3 that bring a sparse
 * J to one of these layouts; qrk_factor_vcat concatenates two factored block-angular
 * problems vertically (Section 4.5).
 *
 * The paper's interface is compute(A); Q^T b; R.solve(Q^T b) (Section 5.1).  Because
 * the step always knows b, "compute" and "Q^T b" are fused into qrk_factor_*: b rides
 * through the factorisation as one more column and Q is stored only on request
 * (qrk_set_keep_q).  "R.solve" (plus optional refinement) is qrk_solve; a new right-hand
 * side with the same factor is qrk_solve_qt (with the stored Q) or qrk_solve_rhs (with J
 * and the kept R).
 *
 * Conventions for every function below
 *   - Array arguments are DEVICE pointers unless marked [host].  The caller owns
 *     every buffer it passes.  The handle owns its workspace (R factors, coupling
 *     rows, TSQR partials, refinement scratch, status word).
 *   - A handle BORROWS the J, b and d buffers given to qrk_factor_*: qrk_solve with
 *     sweeps > 0, qrk_solve_rhs and qrk_solve_adjoint read them again, so they must stay
 *     alive and unchanged until the next factor call or qrk_destroy.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).  Calls
 *     after create only enqueue work on that stream and never synchronise, except
 *     qrk_status_get and qrk_get_factor.
 *   - Argument errors are detected on the host before anything is enqueued and
 *     return QRK_EINVAL.  Numerical conditions (tiny pivot, non-finite values) are
 *     recorded in a device status word and reported by qrk_status_get; kernels never
 *     trap.  The functions never throw.
 *   - Handles are not thread-safe; distinct handles are independent.
 *   - Row-major storage throughout.  "T" below is float for QRK_F32 handles and
 *     double for QRK_F64 handles.
 */
#ifndef QRKIT_H
#define QRKIT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QRK_OK = 0,
  QRK_EINVAL = 1,        /* bad argument or shape; nothing was enqueued            */
  QRK_ENOMEM = 2,        /* device workspace allocation failed                     */
  QRK_EHIP = 3,          /* a HIP runtime call failed                              */
  QRK_ESINGULAR = 4,     /* a pivot of R is (numerically) zero; p is undefined     */
  QRK_ENONFINITE = 5,    /* NaN or Inf met in the inputs or the factor             */
  QRK_ENODEVICE = 6,     /* no usable gfx950 device                                */
  QRK_ETOOLARGE = 7,     /* the request does not fit the fixed scratch array of
                            qrk_solve_banded_noalloc; nothing was enqueued          */
  QRK_ENOTCONVERGED = 8  /* qrk_solve_tol used all its sweeps above the tolerance;
                            p is the last iterate                                   */
} qrk_status;

typedef enum { QRK_F32 = 0, QRK_F64 = 1 } qrk_dtype;

/* How the dense-part trailing updates are multiplied (float32 handles only).
 * QRK_PLAIN: fp32 products.  QRK_BF16X3: each fp32 operand x is split into
 * hi = bf16(x), lo = bf16(x - hi) and a*b is formed as hi*hi' + hi*lo' + lo*hi'
 * on the bf16 matrix cores with fp32 accumulation (about 16 significant bits). */
typedef enum { QRK_PLAIN = 0, QRK_BF16X3 = 1 } qrk_mode;

typedef struct qrk_handle_s* qrk_handle;

/* Limits of this implementation. */
#define QRK_MAX_BLOCK_COLS 8     /* n, columns per diagonal block                 */
#define QRK_MAX_BLOCK_ROWS 56    /* m_i, rows per diagonal block                  */
#define QRK_MAX_LDB (1 << 20)    /* row stride of B (elements): a block's rows of B
                                    span less than 2^31 bytes                       */
#define QRK_MAX_DENSE_COLS 127   /* nB, columns of the dense part B               */
#define QRK_MAX_BAND 31          /* w, nonzeros per banded row                    */

/* ------------------------------------------------------------------------------
 * qrk_create_blockangular
 *   Plan a solver for block-angular J with K blocks of n columns and a dense part of
 *   nB columns.  row_off_host [host, int64, K+1]: block i owns rows
 *   [row_off_host[i], row_off_host[i+1]) of J, of B and of b; row_off_host[0] = 0,
 *   nondecreasing, 0 <= m_i = row_off[i+1]-row_off[i] <= QRK_MAX_BLOCK_ROWS.  The
 *   row structure is copied; it is fixed for the life of the handle.
 *   nB <= ldb <= QRK_MAX_LDB is the row stride (in elements) of B.  Allocates all
 *   device workspace, so later calls allocate nothing.
 *   Returns QRK_EINVAL for K < 1, n outside 1..8, nB outside 0..127, ldb outside
 *   nB..QRK_MAX_LDB, a bad
 *   row_off_host, or mode == QRK_BF16X3 with dtype == QRK_F64.
 * ------------------------------------------------------------------------------ */
qrk_status qrk_create_blockangular(int32_t K, int32_t n, int32_t nB, const int64_t* row_off_host,
                                   int64_t ldb, qrk_dtype dtype, qrk_mode mode, qrk_handle* out);

/* ------------------------------------------------------------------------------
 * qrk_create_blockangular_ncol
 *   Block-angular J whose blocks have their own column counts (Section 4.1: block i is
 *   m_i x n_i): ncol_host [host, int32, K], 1 <= ncol_host[i] <= 8; the other arguments as
 *   for qrk_create_blockangular.  The handle runs the blocks at n = max_i ncol_host[i]
 *   columns: block i's columns past n_i are zero in J and their damping values are 1, so for
 *   lambda > 0 those unknowns decouple from the rest and the solution restricted to the real
 *   unknowns is that of the problem as given.
 *   Layouts on such a handle (N' = sum_i n_i + nB unknowns): A [device] holds block i's rows
 *   row-major with n_i values per row, block after block (block i starts at
 *   sum_{k<i} m_k n_k); d [device, N' doubles] and p [N' doubles] hold block i's unknowns at
 *   sum_{k<i} n_k, then the dense part's; B and b as for qrk_create_blockangular.
 *   qrk_factor_blockangular copies A and d into the handle's layout (lambda > 0 is
 *   required: QRK_EINVAL otherwise); qrk_solve and qrk_solve_tol write p in the caller's
 *   layout; qrk_get_factor returns the factor of the handle's n-column layout.  The
 *   two-stage, batched, new-right-hand-side, adjoint, stored-Q, concatenation, column-norm
 *   and LM calls return QRK_EINVAL on this handle.
 * ------------------------------------------------------------------------------ */
qrk_status qrk_create_blockangular_ncol(int32_t K, const int32_t* ncol_host, int32_t nB,
                                        const int64_t* row_off_host, int64_t ldb, qrk_dtype dtype,
                                        qrk_mode mode, qrk_handle* out);

/* ------------------------------------------------------------------------------
 * qrk_factor_blockangular
 *   Structured QR of P_r [J; sqrt(lambda) D] with b carried along (Sections 4.1, 4.2):
 *     per block   [A_i; sqrt(lambda) D_i] = Q_i [R_i; 0]   (Householder, Section 2),
 *                 Q_i^T [B_i | b_i; 0 | 0] -> coupling rows S_i | c_i and reduced rows;
 *     dense part  QR of [all reduced rows; sqrt(lambda) D_B | 0] -> R_B | c_B
 *                 (tall-skinny QR: per-workgroup leaves, then a reduction tree).
 *   A [M x n] T, row r belongs to the block owning row r; B [M x ldb] T; b [M] T;
 *   d [N = K*n + nB] double, d_j > 0; lambda >= 0 (finite).
 *   Returns QRK_EINVAL on null pointers (B may be null iff nB == 0) or bad lambda.
 * ------------------------------------------------------------------------------ */
qrk_status qrk_factor_blockangular(qrk_handle h, const void* A, const void* B, const void* b,
                                   const double* d, double lambda, void* stream);

/* ------------------------------------------------------------------------------
 * qrk_create_blockangular_cam, qrk_factor_blockangular_cam
 *   Block-angular J whose coupled columns are cameras: the bundle-adjustment Jacobian of the
 *   experiments of Section 6.2, solved as the horizontal concatenation of Section 4.2, where
 *   every row depends on one point block (n columns) and at most one camera.  The dense part
 *   has nB = ncam * cw columns, camera c owning columns c*cw .. c*cw + cw - 1, and is passed
 *   compressed: Bv [device, M x cw] T holds row r's cw values and cam [device, int32, M] its
 *   camera, so that B[r, cam[r]*cw + k] = Bv[r*cw + k] and B is zero elsewhere in row r.
 *   A camera index outside [0, ncam) means the row touches no camera (its Bv row is not
 *   used).  The per-block QR and the refinement read the compressed rows directly.
 *   create: ncam >= 1, cw >= 1, ncam * cw <= QRK_MAX_DENSE_COLS; the other arguments as for
 *   qrk_create_blockangular (QRK_EINVAL otherwise).
 *   factor: A, b, d, lambda as for qrk_factor_blockangular; Bv and cam are borrowed like A
 *   (the refinement of qrk_solve, qrk_solve_tol, qrk_solve_rhs and qrk_solve_qt reads them,
 *   so they must stay valid and unchanged until the next factor).  QRK_EINVAL on null
 *   pointers, bad lambda or a handle not made by qrk_create_blockangular_cam.
 *   On such a handle qrk_factor_blockangular, the batched and concatenation calls,
 *   qrk_solve_adjoint, qrk_colnorms_blockangular and the LM calls return QRK_EINVAL; the
 *   solve, two-stage, new-right-hand-side, stored-Q, autotuner and factor-readback calls work
 *   as on a dense-B handle.
 * ------------------------------------------------------------------------------ */
qrk_status qrk_create_blockangular_cam(int32_t K, int32_t n, int32_t ncam, int32_t cw,
                                       const int64_t* row_off_host, qrk_dtype dtype, qrk_mode mode,
                                       qrk_handle* out);
qrk_status qrk_factor_blockangular_cam(qrk_handle h, const void* A, const void* Bv, const int32_t* cam,
                                       const void* b, const double* d, double lambda, void* stream);

/* ------------------------------------------------------------------------------
 * qrk_factor_lambda  (single-problem block-angular handles)
 *   Moré's two-stage damping (Section 5.2, Eq. LMTwoStep): with J = Q R factored once by
 *   qrk_factor_blockangular(h, ..., lambda = 0, ...), each call factors [R; sqrt(lambda) D]
 *   instead of [J; sqrt(lambda) D].  The damping rows of each block are permuted next to its
 *   R_i, so the second QR is again structured: blocks [R_i; sqrt(lambda) D_i] with coupled
 *   rows [S_i | c_i; 0], and a dense part over the blocks' reduced rows, the rows of
 *   R_B | c_B and sqrt(lambda) D_B.  The result replaces the handle's factor (the factor of J
 *   is kept aside, so any number of calls may follow one factorisation of J); qrk_solve then
 *   solves the damped problem for this lambda, its refinement using the original J, b, d
 *   given to qrk_factor_blockangular (still borrowed: they must stay valid and unchanged).
 *   lambda > 0, finite.  QRK_EINVAL for a batched or banded handle, before any factor, or when
 *   the factor of J saved by an earlier call is gone (a new qrk_factor_blockangular call) and
 *   the current factor's lambda is not 0.  Allocates the kept factor and the second-stage
 *   workspace on its first call.  Not capturable on its first call after a factor of J.
 * ------------------------------------------------------------------------------ */
qrk_status qrk_factor_lambda(qrk_handle h, double lambda, void* stream);

/* ------------------------------------------------------------------------------
 * qrk_create_blockangular_batched / qrk_factor_blockangular_batched
 *   P independent block-angular problems with the same block width n, factored and solved
 *   together: every phase of qrk_factor_blockangular / qrk_solve runs over all problems in
 *   the same launches (the per-problem dense-part merge trees proceed independently inside
 *   one launch per 16-column-block count).  Problem p has K_host[p] >= 1 blocks and
 *   0 <= nB_host[p] <= 127 dense columns; N_p = K_host[p] n + nB_host[p].
 *   row_off_host [host, int64, sum_p K_p + 1]: global row offsets of all blocks, problem
 *   after problem (row_off_host[0] = 0, nondecreasing, m_i <= QRK_MAX_BLOCK_ROWS); problem p
 *   owns the rows of its blocks.  Stacked device arrays, problem after problem:
 *     A [M_tot x n] T and b [M_tot] T (global rows);
 *     B: problem p's M_p x nB_p block, row-major with row stride nB_p, starting at element
 *        sum_{q<p} M_q nB_q;
 *     d [sum_p N_p] double;  lambda_dev [P] double, >= 0, read by the kernels when they
 *        run (a captured graph picks up new values at each replay; not validated);
 *     p (qrk_solve) [sum_p N_p] double.
 *   qrk_status_get reports the worst condition over the batch (detail = OR of the bits);
 *   qrk_status_get_problems gives the bits of every problem.  qrk_solve_adjoint,
 *   qrk_colnorms_blockangular and qrk_get_factor are single-problem only (QRK_EINVAL).
 *   create returns QRK_EINVAL for P < 1, n outside 1..8, a bad K_host / nB_host /
 *   row_off_host, or mode == QRK_BF16X3 with dtype == QRK_F64.
 * ------------------------------------------------------------------------------ */
qrk_status qrk_create_blockangular_batched(int32_t P, int32_t n, const int32_t* K_host, const int32_t* nB_host,
                                           const int64_t* row_off_host, qrk_dtype dtype, qrk_mode mode,
                                           qrk_handle* out);
qrk_status qrk_factor_blockangular_batched(qrk_handle h, const void* A, const void* B, const void* b,
                                           const double* d, const double* lambda_dev, void* stream);
/* Status bits (1 singular, 2 non-finite, 4 bad input) of each of the P problems of a
 * handle into bits_host [host, int32, P]; synchronises `stream`. */
qrk_status qrk_status_get_problems(qrk_handle h, int32_t* bits_host, void* stream);

/* ------------------------------------------------------------------------------
 * qrk_create_banded / qrk_factor_banded
 *   Banded J (M x N, w values per row).  qrk_factor_banded starts from the upper
 *   triangular R = diag(sqrt(lambda) d) and rotates each row of J into R in row order
 *   with at most w Givens rotations; b rides along into c.  R has upper bandwidth w-1.
 *   row_start [M] int32, nondecreasing, 0 <= row_start[i] <= N - w (checked on the
 *   device; a violation sets QRK_EINVAL in the status word); vals [M x w] T;
 *   b [M] T; d [N] double > 0; lambda >= 0.
 *   create returns QRK_EINVAL for M < 0, N < 1, w outside 1..QRK_MAX_BAND, w > N.
 *   Out-of-range or decreasing row starts are clamped and reported as QRK_EINVAL by
 *   qrk_status_get (the factor of such a call is not meaningful).
 * ------------------------------------------------------------------------------ */
qrk_status qrk_create_banded(int64_t M, int64_t N, int32_t w, qrk_dtype dtype, qrk_handle* out);
/* P independent banded problems of the same shape in one handle (one launch per step): every
 * per-problem array is stacked, row_start [P][M], vals [P][M][w], b [P][M], d and p [P][N];
 * qrk_solve, qrk_solve_adjoint (dlambda [P]) and qrk_get_factor (R [P][N][w], c [P][N])
 * follow the same stacking.  QRK_EINVAL for P < 1 or the shape errors above. */
qrk_status qrk_create_banded_batched(int32_t P, int64_t M, int64_t N, int32_t w, qrk_dtype dtype,
                                     qrk_handle* out);
qrk_status qrk_factor_banded(qrk_handle h, const int32_t* row_start, const void* vals,
                             const void* b, const double* d, double lambda, void* stream);

/* ------------------------------------------------------------------------------
 * qrk_set_banded_method
 *   How qrk_factor_banded (and the LM driver on this handle) factorises:
 *     QRK_BANDED_GIVENS (0, the default): Givens rotations row by row.
 *     QRK_BANDED_BLOCKWY (1): the block-banded factorisation of Section 4.4 (Eq.
 *       blockBandedYTY): columns in blocks of 16, each step a dense QR of the rows carried from
 *       the previous step, the next block's damping rows and the rows whose first nonzero lies
 *       in the block, over two column blocks and the right-hand side, its Householder
 *       vectors local to those rows and applied in the compact WY form on the matrix cores.
 *     QRK_BANDED_BLOCKWY_BF16X3 (2): the same with BF16x3 products in the WY updates.
 *   The factor's outputs (R, c) and every later call are the same for all methods (R is
 *   unique up to row signs).  Methods 1 and 2 need a QRK_F32 handle with w <= 15
 *   (QRK_EINVAL otherwise, or for a block-angular handle).  Takes effect at the next factor.
 * ------------------------------------------------------------------------------ */
#define QRK_BANDED_GIVENS 0
#define QRK_BANDED_BLOCKWY 1
#define QRK_BANDED_BLOCKWY_BF16X3 2
qrk_status qrk_set_banded_method(qrk_handle h, int32_t method);

/* ------------------------------------------------------------------------------
 * qrk_solve
 *   Back-substitution through the stored R (Section 4.2: R = [[blkdiag(R_i), S],
 *   [0, R_B]] for block-angular J, banded R otherwise), then `sweeps` (0..8) sweeps of
 *   corrected semi-normal-equation refinement against the same R:
 *       r = b - J p,  g = J^T r - lambda D^2 p      (float64 on the device),
 *       R^T R delta = g (two triangular solves),    p <- p + delta   (p in float64).
 *   p [N] double (written).  Needs a preceding qrk_factor_* on this handle.
 * ------------------------------------------------------------------------------ */
qrk_status qrk_solve(qrk_handle h, double* p, int32_t sweeps, void* stream);

/* ------------------------------------------------------------------------------
 * qrk_solve_tol
 *   qrk_solve with an early stop: the back-substitution, then up to max_sweeps (0..8)
 *   refinement sweeps, stopping after the first sweep whose correction satisfies
 *   ||delta||_2 <= rel_tol ||p||_2 for every problem of the handle (rel_tol >= 0, finite).
 *   p as for qrk_solve.  *sweeps_host [host, may be NULL] receives the sweeps run.  Returns
 *   QRK_OK when the tolerance was met (or max_sweeps == 0), QRK_ENOTCONVERGED when the sweeps
 *   ran out first (p is then the last iterate, and the problems still above the tolerance
 *   carry the status bit 16, which qrk_status_get reports as QRK_ENOTCONVERGED until the next
 *   factor call).  The norms are summed on the device and read by the host after each sweep,
 *   so this call synchronises `stream` once per sweep and is not capturable (qrk_solve with a
 *   fixed sweep count is).  It allocates two small buffers on its first call on a handle.
 *   QRK_EINVAL for a NULL handle or p, a handle without a factor, or bad max_sweeps / rel_tol.
 * ------------------------------------------------------------------------------ */
qrk_status qrk_solve_tol(qrk_handle h, double* p, int32_t max_sweeps, double rel_tol, int32_t* sweeps_host,
                         void* stream);

/* ------------------------------------------------------------------------------
 * qrk_solve_rhs
 *   The step for a new right-hand side with the stored factor (the paper applies the kept
 *   Q^T to each new b, Section 5.1; here Q is not stored): p = argmin
 *   || [J; sqrt(lambda) D] p - [b; 0] || for the J, d and lambda of the last qrk_factor_*
 *   call and the given b, by `sweeps` (1..8) corrected semi-normal sweeps from p = 0:
 *       r = b - J p,  g = J^T r - lambda D^2 p,  R^T R delta = g,  p <- p + delta.
 *   The first sweep gives the semi-normal solution R^{-1} R^{-T} J^T b; each further sweep
 *   reduces the error by about cond(J) times the factor's relative accuracy (float32
 *   factors, fp32 or BF16x3 updates: four sweeps reach 1e-10 at cond(J) <= 1e3).
 *   b: device, the layout and type of the factor call's b (block-angular [M] stacked over
 *   the problems, banded [P][M]); p [N] double (block-angular: sum_p N_p; banded: P * N),
 *   written.  Neither the handle's borrowed b nor its factor is changed: qrk_solve still
 *   solves for the factor call's b.  Errors: QRK_EINVAL for a NULL handle, b or p, a
 *   handle without a factor, or sweeps outside 1..8.
 * ------------------------------------------------------------------------------ */
qrk_status qrk_solve_rhs(qrk_handle h, const void* b, double* p, int32_t sweeps, void* stream);

/* ------------------------------------------------------------------------------
 * qrk_factor_vcat (Section 4.5, Eq. vcatDecomp: vertical concatenation)
 *   Replaces the factor of h by that of the problem with the rows of both handles, from the two
 *   kept factors alone: [A1; A2] = blkdiag(Q1, Q2) [R1; R2], and the row permutation that
 *   interleaves R1 and R2 block by block makes P [R1; R2] block-angular again (blocks
 *   [R1_i; R2_i], coupled rows [S1_i | c1_i; S2_i | c2_i], dense part [R1_B | c1_B; R2_B | c2_B]),
 *   which the factor call's own kernels factor once more.  The result is the factor of
 *       min_p || [J1; sqrt(lambda1) D1; J2; sqrt(lambda2) D2] p - [b1; 0; b2; 0] ||
 *   for the inputs and damping of the two handles' last factor calls (lambda2 = 0 adds rows
 *   without a second damping).  Both handles single-problem block-angular with equal K, n, n_B and
 *   dtype (h's mode is used); the rows per block may differ.  h may already hold a concatenation
 *   (up to 64 added handles); h2 may not.  h2 and its borrowed J, b, d must stay alive and
 *   unchanged while h holds the concatenation (until h's next factor call): qrk_solve and
 *   qrk_solve_tol on h refine against every part's rows.  qrk_solve_rhs, qrk_solve_adjoint,
 *   qrk_factor_lambda and qrk_apply_qt return QRK_EINVAL on a handle holding a concatenation.
 *   Allocates the merge's workspace on its first call on h (not capturable then), enqueues only
 *   afterwards.  QRK_EINVAL for mismatched or unfactored handles, h == h2, or h2 itself holding
 *   a concatenation.
 * ------------------------------------------------------------------------------ */
qrk_status qrk_factor_vcat(qrk_handle h, qrk_handle h2, void* stream);

/* ------------------------------------------------------------------------------
 * Stored Q (Section 2: Q kept as the object that applies its Householder reflectors;
 * Sections 5.1 and 5.2: Q^T applied to each new right-hand side with the same factor).
 * Float32 block-angular handles (single or batched) whose blocks all have m_i >= n.
 *
 * qrk_set_keep_q(h, keep)
 *   keep != 0: every following factor call also stores Q: for each block its n reflectors
 *   H_j = I - g_j z_j z_j^T over the block's data and damping rows (M n + K n n + K n floats),
 *   and for the dense part the compact-WY panels (T and the column scales) of every tile each
 *   leaf merged, whose reflector columns overwrite the reduced rows in the handle's workspace,
 *   and the panels (T, scales and reflector blocks) of every merge of two triangles.  Together
 *   about 1.4 times the reduced rows' bytes.  The storage is allocated here and when the leaf
 *   layout changes (qrk_set_tsqr_shape, autotuning); the factor calls stay capturable.  An LM
 *   driver graph captured before the call is captured again at its next qrk_lm_run.  A factor
 *   that stores Q gives the same per-block factor, bit for bit, as one that does not; its dense
 *   part may take tiles of another height (64 rows at 6 column blocks instead of 128), so R_B |
 *   c_B agree up to row signs and rounding.
 *   keep == 0: later factor calls store nothing (the storage is kept until qrk_destroy).
 *   QRK_EINVAL: NULL handle; keep != 0 on a banded or float64 handle, or with a block of
 *   fewer rows than columns.  QRK_ENOMEM if the storage cannot be allocated.
 *
 * qrk_apply_qt(h, b, c, stream)
 *   c = the first N entries of Q^T [b; 0] for the stored Q of the last factor call, where
 *   [J; sqrt(lambda) D] = Q [R; 0] with the damping rows of each block and of the dense part
 *   in the order the factorisation places them (their right-hand side is zero): c_i of every
 *   block (n entries each), then c_B (nB), per problem, laid out like p.  R and c are unique up
 *   to the sign of each row of R (qrk_get_factor gives R).  b [M] float (the factor call's b
 *   layout); c [N] double, written (computed in float32 except the per-block stage, float64).
 *   Work space is the handle's; calls on one handle must not overlap.  QRK_EINVAL: NULL
 *   argument, or the last factor call did not store Q.
 *
 * qrk_solve_qt(h, b, p, sweeps, stream)
 *   The step for a new right-hand side by the stored Q: p = R^{-1} (Q^T b) as qrk_apply_qt
 *   computes it, then `sweeps` (0..8) refinement sweeps for b as in qrk_solve_rhs.  One pass
 *   over the stored reflectors instead of qrk_solve_rhs's sweeps over J: sweeps = 0 gives the
 *   factor's own accuracy (as qrk_solve with sweeps = 0 does for the factor call's b).  The
 *   handle's borrowed b and its factor are unchanged; pivot and finiteness conditions go to
 *   the status word.  QRK_EINVAL as for qrk_apply_qt, or sweeps outside 0..8.
 * ------------------------------------------------------------------------------ */
qrk_status qrk_set_keep_q(qrk_handle h, int32_t keep);
qrk_status qrk_apply_qt(qrk_handle h, const void* b, double* c, void* stream);
qrk_status qrk_solve_qt(qrk_handle h, const void* b, double* p, int32_t sweeps, void* stream);

/* ------------------------------------------------------------------------------
 * qrk_solve_adjoint
 *   For a loss L(p) of the step p (from qrk_solve on this handle) and g = dL/dp,
 *   with u = (R^T R)^{-1} g (two triangular solves with the stored R; R^T R =
 *   J^T J + lambda D^2) and r = b - J p:
 *       dL/db = J u,   dL/dJ_ab = r_a u_b - (J u)_a p_b   (structural nonzeros only),
 *       dL/dlambda = -u^T D^2 p,   dL/dd_j = -2 lambda u_j d_j p_j.
 *   Block-angular handles: dA [M x n] T, dB [M x ldb] T, db [M] T.  Banded handles:
 *   dA is dvals [M x w] T and dB must be NULL.  p, g [N] double.  dlambda [1] double,
 *   dd [N] double.  Any output pointer may be NULL (not computed).
 * ------------------------------------------------------------------------------ */
qrk_status qrk_solve_adjoint(qrk_handle h, const double* p, const double* g, void* dA, void* dB,
                             void* db, double* dlambda, double* dd, void* stream);

/* ------------------------------------------------------------------------------
 * qrk_colnorms_blockangular
 *   d_j = ||J e_j||_2 in float64 (1 for an all-zero column), the LM choice
 *   D = diag(J^T J)^(1/2) of Section 5.2.  A, B as for qrk_factor_blockangular; d [N].
 * ------------------------------------------------------------------------------ */
qrk_status qrk_colnorms_blockangular(qrk_handle h, const void* A, const void* B, double* d,
                                     void* stream);

/* ------------------------------------------------------------------------------
 * qrk_colnorms_blockangular_cam
 *   The same column norms for a handle made by qrk_create_blockangular_cam: A, Bv, cam as for
 *   qrk_factor_blockangular_cam; d [N].  A camera column no row touches gets d_j = 1.
 * ------------------------------------------------------------------------------ */
qrk_status qrk_colnorms_blockangular_cam(qrk_handle h, const void* A, const void* Bv, const int32_t* cam,
                                         double* d, void* stream);

/* ------------------------------------------------------------------------------
 * qrk_get_factor (inspection; synchronises the stream)
 *   Copies the stored factor into caller DEVICE buffers, any of which may be NULL.
 *   Block-angular: Rblk [K x n x n] T (R_i, zeros below the diagonal);
 *   S [K x n x (nB+1)] T (coupling rows S_i with c_i as last column);
 *   RB [(nB+1) x (nB+1)] T (R_B with c_B as last column; entry [nB][nB] is +-the
 *   residual norm || [J; sqrt(lambda) D] p - [b; 0] ||).
 *   Banded: Rblk [N x w] T (row j holds R[j][j .. j+w-1]), S [N] T (c), RB unused.
 * ------------------------------------------------------------------------------ */
qrk_status qrk_get_factor(qrk_handle h, void* Rblk, void* S, void* RB, void* stream);

/* ------------------------------------------------------------------------------
 * qrk_status_get: synchronises `stream`, returns the worst numerical condition recorded
 * since the last factor call (QRK_OK, QRK_ESINGULAR, QRK_ENONFINITE, QRK_ENOTCONVERGED after a
 * qrk_solve_tol that ran out of sweeps, or QRK_EINVAL for a bad banded row_start) and clears
 * nothing.  *detail_host [host, may be NULL] receives
 * the raw status bits.
 * ------------------------------------------------------------------------------ */
qrk_status qrk_status_get(qrk_handle h, int32_t* detail_host, void* stream);

/* Set the launch shape of the dense-part leaves of a single-problem handle (0 = library
 * default): number of leaves (at most 4096 for float32 handles, 1024 for float64 ones) and,
 * for float64 handles, the tree fan-in.
 * Not capturable (it may reallocate the merge-tree workspace).  Synchronises the device
 * first (no earlier work on any stream may still read the leaf tables it rewrites).  An LM
 * driver graph captured on this handle before the call is captured again at its next
 * qrk_lm_run.  QRK_EINVAL for out-of-range values or a batched handle. */
qrk_status qrk_set_tsqr_shape(qrk_handle h, int32_t leaves, int32_t fanin);

/* ------------------------------------------------------------------------------
 * qrk_autotune_blockangular (float32 handles; not capturable; synchronises the device)
 *   Times the factorisation plus a one-sweep solve of the inputs of the last qrk_factor_*
 *   call on this handle over three launch-shape knobs, by coordinate search, and keeps the
 *   fastest: the rows per dense-part leaf (1/2, 1, 2 or 4 times the library default, capped
 *   at 1024 leaves per problem), for batches whose dense parts have several widths of at most
 *   6 column blocks one persistent leaf launch over all of them or one launch per width, and
 *   the number of refinement workgroups (1/2, 1 or 2 times the default).  The handle is left
 *   factored with the chosen shape.  The choice is remembered in the process, and in the
 *   cache file when one is set (qrk_tune_cache_file), under a key of the device architecture,
 *   dtype, mode, block width, widest dense part, number of dense-part widths, and the problem
 *   and row counts rounded up to powers of two; a handle created later for a matching key
 *   starts from it.  *scale_host [host, may be NULL] receives the chosen leaf scale.  Like
 *   qrk_set_tsqr_shape it may rewrite the leaf and refinement tables, so an LM driver graph
 *   captured on this handle is captured again at its next qrk_lm_run.  QRK_EINVAL before any
 *   factor call.
 * ------------------------------------------------------------------------------ */
qrk_status qrk_autotune_blockangular(qrk_handle h, double* scale_host, void* stream);

/* The launch-shape knobs a block-angular handle uses (from qrk_autotune_blockangular, the cache,
 * or the defaults 1, 1, 1); any pointer [host] may be NULL.  QRK_EINVAL for a banded handle. */
qrk_status qrk_tune_get(qrk_handle h, double* leaf_scale, int32_t* leaf_queue, double* refine_scale);

/* Sets the autotuner's cache file [host path, NULL: none] for the process and loads the choices
 * it holds (JSON; written again after every qrk_autotune_blockangular, best effort).  Without a
 * call, the QRK_TUNE_CACHE environment variable names the file.  QRK_EINVAL if an existing file
 * cannot be parsed. */
qrk_status qrk_tune_cache_file(const char* path);

/* ------------------------------------------------------------------------------
 * Levenberg-Marquardt driver (Backtrack LM of Section 5.2) for the synthetic model
 *     f(x) = J0 phi(x) - y,   phi(t) = t + c t^3 elementwise,   J(x) = J0 diag(phi'(x)),
 * on every problem of a block-angular handle (single or batched) or of a banded handle (P
 * stacked problems); J(x) keeps J0's pattern.
 * One iteration, per problem, entirely on the device:
 *     J(x), b = -f(x) (stored in the handle's type), d = column norms of J(x) (1 for a zero
 *     column), F = |f|^2/2;  p = the handle's factor + solve with `sweeps` refinement sweeps;
 *     pred = p^T (lambda D^2 p - J^T f)/2;  F_new = |f(x + p)|^2/2;  rho = (F - F_new)/pred;
 *     rho > 0: x += p, lambda *= max(1/3, 1 - (2 rho - 1)^3), nu = 2; else lambda *= nu,
 *     nu *= 2  (Nielsen's rule; the paper names the rule it adapts but not its constants).
 * qrk_lm_create_blockangular: A0, B0, y [device, the handle's type and layouts, borrowed
 *   for the life of the driver]; c finite; 0 <= sweeps <= 8; max_log >= 0 iterations of
 *   log kept.  The driver uses the handle's factor workspace (do not factor on the handle
 *   while a run is in flight).  Allocates its state (J(x), -f, x, p, d, damping, log).
 * qrk_lm_create_banded: row_start [device, P x M int32, nondecreasing, <= N - w], vals0
 *   [device, P x M x w] and y [device, P x M] in the handle's type, borrowed; the other
 *   arguments as above.  QRK_EINVAL for M < 1.
 * qrk_lm_reset: x0 [device, N (all problems: P x N for banded handles)] and lambda0 [device, P] doubles; nu = 2; clears the log and
 *   the iteration counter.  Stream-ordered.
 * qrk_lm_run: `iters` iterations on `stream`.  use_graph = 0 enqueues them one by one;
 *   use_graph != 0 captures one iteration into a HIP graph on the driver's own stream at
 *   the first such call (not capturable itself) and replays it `iters` times on `stream`.
 * qrk_lm_get: copies x [device, N], lambda [device, P] and the log [device,
 *   max_log x P x 4: F, F_new, lambda after, accepted (0/1)] (any may be NULL); with
 *   iters_host != NULL synchronises `stream` and returns the number of iterations run.
 * ------------------------------------------------------------------------------ */
typedef struct qrk_lm_s* qrk_lm;
qrk_status qrk_lm_create_blockangular(qrk_handle h, const void* A0, const void* B0, const void* y, double c,
                                      int32_t sweeps, int32_t max_log, qrk_lm* out);
qrk_status qrk_lm_create_banded(qrk_handle h, const int32_t* row_start, const void* vals0, const void* y, double c,
                                int32_t sweeps, int32_t max_log, qrk_lm* out);
qrk_status qrk_lm_reset(qrk_lm lm, const double* x0, const double* lambda0, void* stream);
qrk_status qrk_lm_run(qrk_lm lm, int32_t iters, int32_t use_graph, void* stream);
qrk_status qrk_lm_get(qrk_lm lm, double* x, double* lambda, double* log, int32_t* iters_host, void* stream);
void qrk_lm_destroy(qrk_lm lm);

/* ------------------------------------------------------------------------------
 * Phase timing (HIP events recorded on the call's stream around each phase).
 * qrk_profile_enable(h, max_calls): max_calls > 0 creates the events for that many
 * factor/solve calls (not capturable; call outside graph capture) and starts
 * recording; 0 stops recording and frees the events.
 * qrk_profile_read(h, ms_host, count_host, nphase): synchronises, then writes for each
 * phase the summed milliseconds [host, double] and the number of recorded launches
 * [host, int32] since enable/the previous read, and resets the sums.  Phases:
 *   0 per-block QR, 1 dense-part leaves, 2 dense-part tree, 3 back-substitution,
 *   4 refinement sweeps, 5 banded factorisation.
 * ------------------------------------------------------------------------------ */
#define QRK_NPHASES 6
qrk_status qrk_profile_enable(qrk_handle h, int32_t max_calls);
qrk_status qrk_profile_read(qrk_handle h, double* ms_host, int32_t* count_host, int32_t nphase);

/* ------------------------------------------------------------------------------
 * qrk_solve_banded_noalloc  (for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc)
 *   The banded step of qrk_create_banded_batched + qrk_factor_banded + qrk_solve in one call
 *   without a handle: Givens QR of [J; sqrt(lambda) D] for P stacked problems (M rows, N
 *   columns, w values per row), back-substitution and `sweeps` (0..8) float64-residual
 *   sweeps, with the same kernels and the same results.  Arguments as for those calls:
 *   row_start [P][M] int32, vals [P][M][w] T, b [P][M] T, d [P][N] double, lambda >= 0 (one
 *   value for every problem), p [P][N] double (written); status_dev [device, int32, 1, may be
 *   NULL] receives the status bits of qrk_status_get (1 singular, 2 non-finite, 4 bad row
 *   start).  The caller owns every buffer.
 *   No memory is allocated: the factor, the sweep buffers and the status word live in one
 *   fixed device array of QRK_NOALLOC_SCRATCH_BYTES per GPU, held from the library's first
 *   call on that GPU until the process ends.  A request whose workspace (about
 *   P N ((w + 17) sizeof(T) + 20) + 8 P M bytes) does not fit returns QRK_ETOOLARGE before
 *   anything is enqueued.  All calls on one GPU share the array: calls that overlap in time
 *   on that GPU (different streams or threads) race and must be serialised by the caller.
 *   Stream-ordered; never synchronises.  QRK_EINVAL for the argument errors of the calls it
 *   replaces; QRK_ENODEVICE on a device that is not gfx950.
 * ------------------------------------------------------------------------------ */
#define QRK_NOALLOC_SCRATCH_BYTES (32ll << 20)
qrk_status qrk_solve_banded_noalloc(int32_t P, int64_t M, int64_t N, int32_t w, qrk_dtype dtype,
                                    const int32_t* row_start, const void* vals, const void* b, const double* d,
                                    double lambda, double* p, int32_t sweeps, int32_t* status_dev, void* stream);

/* ------------------------------------------------------------------------------
 * qrk_discover_blockangular / qrk_discover_banded  [host only: no device, no handle]
 *   The row and column permutations of Section 4.3 that reveal a structure in a sparse J,
 *   J' = P_r J P_c, given J's pattern: row_ptr [host, int64, M+1] (row_ptr[0] = 0,
 *   nondecreasing) and col_idx [host, int32, row_ptr[M]] (each row's columns, 0 <= c < N, any
 *   order).  Values are not read.  Row k of J' is row row_perm[k] of J; column j of J' is
 *   column col_perm[j] of J.  All outputs are caller-allocated host arrays.
 *   Block-angular (for qrk_create_blockangular_ncol): dense_cols [host, int32, nB] are the
 *   coupled columns (distinct, nB <= 127, nB < N).  Two rows belong to the same block when they
 *   share a non-dense column, transitively; a block's columns are the non-dense columns of its
 *   rows (a column no row touches is a block of one column and no rows).  Blocks come in order
 *   of their smallest column, each block's columns and rows in increasing order, then the dense
 *   columns in the order given.  Rows that touch only dense columns go to the first blocks with
 *   fewer than QRK_MAX_BLOCK_ROWS rows.  Outputs: row_perm [M], col_perm [N], ncol [N] (the K
 *   block widths), row_off [M + 1] (the K + 1 block row offsets of J'), *K.
 *   Banded (for qrk_create_banded): rows in order of their first column (stable; the paper's
 *   as-banded-as-possible row order), columns unpermuted.  Outputs: row_perm [M], row_start [M]
 *   (the start column of each row of J', its first column clamped to N - w so that its w
 *   values lie in the matrix; nondecreasing), *w (the largest last - first + 1 over the rows).
 *   QRK_EINVAL: null pointers, bad sizes or indices, repeated dense columns; a block wider than
 *   QRK_MAX_BLOCK_COLS or taller than QRK_MAX_BLOCK_ROWS; an empty row or w > QRK_MAX_BAND
 *   (banded).
 * ------------------------------------------------------------------------------ */
qrk_status qrk_discover_blockangular(int64_t M, int64_t N, const int64_t* row_ptr, const int32_t* col_idx,
                                     int32_t nB, const int32_t* dense_cols, int64_t* row_perm,
                                     int32_t* col_perm, int32_t* ncol, int64_t* row_off, int32_t* K);
qrk_status qrk_discover_banded(int64_t M, int64_t N, const int64_t* row_ptr, const int32_t* col_idx,
                               int64_t* row_perm, int32_t* row_start, int32_t* w);

/* ------------------------------------------------------------------------------
 * Self-check entry points (for parity tests of the BF16x3 mode).  They expose, one at a
 * time, the device primitives of the dense-part trailing updates C <- C - V (T^T (V^T C))
 * (Section 2, compact WY) in QRK_BF16X3 mode, where every fp32 operand x is split as
 * hi = bf16(x), lo = bf16(x - hi) (round to nearest even) and a*b is formed as
 * hi*hi' + hi*lo' + lo*hi' on the bf16 matrix cores with fp32 accumulation.
 * qrk_check_bf16_split: x [n] float (device, read); hi, lo [n] float (device, written; the
 *   bf16 values widened exactly to float).  n >= 0.  QRK_EINVAL for n < 0 or null pointers.
 * qrk_check_bf16x3_product: C = A B with A [16 x k] and B [k x 16] float row-major (device,
 *   read) and C [16 x 16] float (device, written), with the kernels' operand layout and
 *   product order (hi*hi' in one accumulator, hi*lo' then lo*hi' in a second, summed at the
 *   end).  32 <= k <= 4096, k a multiple of 32, else QRK_EINVAL.
 * Both are stream-ordered and allocate nothing; the caller owns every buffer.
 * ------------------------------------------------------------------------------ */
qrk_status qrk_check_bf16_split(const float* x, float* hi, float* lo, int64_t n, void* stream);
qrk_status qrk_check_bf16x3_product(const float* A, const float* B, float* C, int32_t k, void* stream);

/* Device workspace held by the handle, in bytes. */
int64_t qrk_workspace_bytes(qrk_handle h);

void qrk_destroy(qrk_handle h);
const char* qrk_strerror(qrk_status s);

#ifdef __cplusplus
}
#endif

#endif /* QRKIT_H */
