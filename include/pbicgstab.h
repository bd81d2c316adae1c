/*
 * pbicgstab.h -- C ABI of the MI355X (gfx950) pipelined BiCGStab library.
 *
 * The library solves A x = b for a sparse, nonsingular N x N matrix A
 * (Section 1 of Cools, "Analyzing and improving maximal attainable accuracy
 * in the communication hiding pipelined BiCGStab method") with
 *
 *   - the preconditioned pipelined BiCGStab method, Algorithm 2, with the
 *     periodic residual replacement of Section 3.6 (eq:rr), and
 *   - the classic preconditioned BiCGStab method, Algorithm 1, for
 *     comparison,
 *
 * both with the identity or the Jacobi (diagonal) preconditioner applied as
 * the listings do (right preconditioning: r = b - A x is the unpreconditioned
 * residual, x is updated with M^-1-preconditioned directions).
 *
 * Conventions for every function
 *   - Return value: 0 (PBCG_CONVERGED) or a positive solver outcome from a
 *     solve, 0 (PBCG_OK) from other calls, or a negative error code.  After an
 *     error, pbicgstab_last_error() returns a message (per thread).
 *   - "host" pointers are CPU memory, "device" pointers are GPU memory of the
 *     device that was current when the handle was created.  All device
 *     vectors are FP64 and hold exactly N elements unless stated otherwise.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is ordered after everything already queued on `stream`, and
 *     `stream` is made to wait for the library's own work before a call
 *     returns, so device buffers may be reused on `stream` right away.
 *   - Ownership.  The caller owns every device array it passes: the matrix
 *     inputs of create (read during the call only), b, x, gradients, and the
 *     workspace: one device allocation of pbicgstab_workspace_bytes() bytes
 *     (256-byte aligned, e.g. a torch uint8 tensor) that holds all of the
 *     handle's device data -- matrix layouts, solver vectors, reduction
 *     partials, device scalars -- and must outlive the handle.  The library
 *     allocates no device memory of its own; the handle owns only its
 *     internal stream, its events, captured HIP graphs and a small pinned
 *     host buffer for polling.  A handle is not thread safe, but separate
 *     handles may be used concurrently.
 */
#ifndef PBICGSTAB_H
#define PBICGSTAB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pbcg_solver* pbcg_handle;

/* storage precision */
enum {
  PBCG_FP64 = 0,  /* everything in FP64 */
  PBCG_MIXED = 1  /* matrix and recurrence vectors stored and updated in FP32 (SPMV and
                     AXPYs in FP32); dot products accumulated in FP64, scalars alpha,
                     beta, omega in FP64, x and b in FP64, residual replacement and
                     true residuals computed in FP64 */
};

/* preconditioner M */
enum {
  PBCG_PC_NONE = 0,
  PBCG_PC_JACOBI = 1,               /* M = diag(A) */
  PBCG_PC_BLOCK_JACOBI_BASE = 256   /* see PBCG_PC_BLOCK_JACOBI */
};
/* Block-Jacobi (CSR handles; a block preconditioner of the kind Section 4.1
 * names as keeping the overlap): M = the block diagonal of A with blocks of b
 * consecutive rows and columns, 2 <= b <= 64 (the last block ragged).  The
 * handle stores A M^-1 (each diagonal block inverted on the host) and runs
 * the iteration on it from y_0 = M x_0, returning x = M^-1 y: the same
 * residuals, scalars and iterates as Algorithm 2 with PREC = M^-1 in exact
 * arithmetic.  Transposed solves, gradients, value updates and the
 * automated replacement are not supported on such handles
 * (PBCG_ERR_UNSUPPORTED). */
#define PBCG_PC_BLOCK_JACOBI(b) (PBCG_PC_BLOCK_JACOBI_BASE | (b))

/* operator formats: structured operators (pbicgstab_create_stencil) and CSR */
enum {
  PBCG_ST_2D5 = 0,  /* constant 5-point stencil, dims {nx, ny}: coef[5] = S, W, C, E, N */
  PBCG_ST_3D7 = 1,  /* constant 7-point stencil, dims {nx, ny, nz}: coef[7] = D, S, W, C, E, N, U */
  PBCG_ST_DIA5 = 2, /* variable 5-point coefficients, dims {nx, ny}: coef[5*N], row d = S, W, C, E, N */
  PBCG_CSR = 3      /* general sparse matrix (pbicgstab_create_csr) */
};

/* outcomes (>= 0) and errors (< 0) */
enum {
  PBCG_OK = 0,
  PBCG_CONVERGED = 0,         /* ||b - A x|| <= tol ||b||, confirmed on the true residual */
  PBCG_MAXIT = 1,             /* maxit iterations done; x holds the last iterate */
  PBCG_BREAKDOWN_RHO = 2,     /* (r0, r_{i+1}) = 0 or a zero denominator of alpha */
  PBCG_BREAKDOWN_OMEGA = 3,   /* omega_i = 0 and the update did not meet the tolerance */
  PBCG_NONFINITE = 4,         /* a reduction produced NaN or Inf */
  PBCG_TRUE_RES_NOT_MET = 5,  /* the recursive residual met tol but the true one did not,
                                 and residual replacement is disabled or 3 replacements
                                 forced by such failures were already made */
  PBCG_ERR_INVALID_ARG = -1,
  PBCG_ERR_HIP = -2,          /* a HIP runtime call failed */
  PBCG_ERR_ZERO_DIAG = -3,    /* Jacobi requested but a diagonal entry is zero or missing */
  PBCG_ERR_WORKSPACE_TOO_SMALL = -4, /* the workspace cannot hold the handle's device data */
  PBCG_ERR_UNSUPPORTED = -5
};

typedef struct {
  double tol;            /* stop when ||r_i|| <= tol * ||b|| (recursive residual, Section 3.5),
                            confirmed by the true residual ||b - A x_i|| */
  int32_t maxit;         /* maximum number of iterations (>= 1) */
  int32_t rr_period;     /* P > 0: residual replacement (eq:rr) in iteration i when
                            (i+1) mod P == 0 and ||r_i|| >= rr_tau ||r_0||.  Also when the
                            recursive residual meets tol but the true one does not: then a
                            replacement is made and the iteration goes on (the replaced
                            residual is not tested in that iteration), at most 3 times per
                            solve.  0 disables both.
                            Ignored by classic_bicgstab_solve. */
  double rr_tau;         /* replacement cutoff; 0 selects sqrt(2^-53) */
  int32_t check_every;   /* iterations between host polls of the device state (0: default:
                            with HIP graphs and periodic replacement as many periods as fit
                            in 128 iterations, else 32 with graphs and 8 without) */
  int32_t transpose;     /* nonzero: solve A^T x = b (the adjoint system) */
  double* history;       /* optional device buffer of 4*history_len doubles; row i (0-based)
                            holds the scalars of iteration i: ||r_{i+1}||, alpha_i,
                            omega_i, beta_{i+1} (0 when the iteration stopped before beta) */
  int32_t history_len;   /* rows */
  int32_t gap_every;     /* > 0: after every gap_every-th iteration store the residual gap
                            ||(b - A x_{i+1}) - r_{i+1}|| (eq:res_gap) in gap_history */
  double* gap_history;   /* device buffer of gap_len doubles */
  int32_t gap_len;
  int32_t use_graph;     /* nonzero: replay chunks of iterations from captured HIP graphs */
  void* stream;          /* hipStream_t */
  int32_t rr_auto;       /* automated residual replacement (Section 3.6) instead of rr_period:
                            the running bound f^r of eq:DDr_bound on the residual gap, built
                            from the local error bounds eq:errbounds1-4 with epsilon rr_eps
                            (the bound restarts after a replacement with the FP64 unit
                            roundoff, the arithmetic of the replacement), replaces in step i
                            when f^r_{i-1} <= tau ||r_{i-1}|| and f^r_i > tau ||r_i||
                            (eq:criterion), tau = rr_tau or sqrt(rr_eps).
                            1: the worst-case bound as eq:DDr_bound prints it (each gap norm
                            bounded first: products of the moduli of the error propagation
                            matrices); 2: its square-root estimate (mu sqrt(N) -> sqrt(mu),
                            mu~ sqrt(N) -> 1); 3: the moduli of the products of the error
                            propagation matrices of eq:all_error_matrices, column by column,
                            times the local error bounds (never larger than variant 1's;
                            needs bound_state); 4: 3 with the estimate's local bounds;
                            0: periodic replacement */
  double rr_eps;         /* epsilon of the bound; 0 selects the unit roundoff of the storage
                            precision (2^-53 FP64, 2^-24 mixed) */
  double* bound_history; /* optional device buffer of bound_len doubles: with rr_auto, entry i
                            (0-based) receives f^r_{i+1}, the bound after iteration i (after a
                            replacement in that iteration: its restart value) */
  int32_t bound_len;
  int32_t restarts;      /* not in the paper: after a (r0, r_{i+1}) = 0 or zero alpha-denominator
                            breakdown, start again from x_{i+1} (Algorithm 2's initialisation with
                            x_0 := x_{i+1}, which also renews the shadow residual), at most this
                            many times; the iteration count continues.  0 (default): stop with
                            PBCG_BREAKDOWN_RHO as the paper's method does. */
  const double* rhat;    /* not in the paper: optional device array of n doubles, a fixed shadow
                            vector used in place of r_0 in every (r_0, .) dot of Algorithms 1
                            and 2 (also after a restart; rounded to FP32 in mixed precision).
                            NULL (default): r_0 = b - A x_0, as in the paper.  Any vector with
                            (rhat, r_0) != 0 is admissible; r_0 breaks down when it is constant
                            and the operator's interior column sums vanish (a conservative
                            discretisation with a constant source): (r_0, r_i) then tends to 0
                            long before r_i does.  Read by the initialisation kernels only;
                            the caller keeps it alive until the solve returns. */
  double* bound_state;   /* rr_auto 3 or 4: caller-owned device scratch for the bound's state,
                            16 doubles per iteration since the last replacement: at least
                            16 * (maxit + 2) doubles (PBCG_ERR_INVALID_ARG otherwise); contents
                            on entry are ignored, on return unspecified */
  int64_t bound_state_len; /* doubles in bound_state */
  int32_t single_kernel; /* nonzero: run the whole of Algorithm 2 as one kernel in one workgroup
                            (row i of every vector in the registers of thread i, the
                            inputs of the products in LDS, the global reductions as
                            workgroup reductions, no host polls) when the system allows it:
                            at most 2048 rows (above 1024 four rows per thread), FP64,
                            rr_auto 0, or 1 or 2 up to 1024 rows (the automated
                            strategy's nested reading, its bound kept in registers; the
                            bound history is written), gap_every 0, restarts 0, not
                            transposed, not block-Jacobi, and a device with 57 KiB (105 KiB
                            above 1024 rows) of LDS per workgroup; otherwise ignored (pbcg_stats.single_kernel
                            tells which ran).  Same arithmetic per row and the
                            same stopping rules as the multi-kernel path; the sums of the
                            reductions are taken in another order (results agree to
                            rounding).  For small systems, whose solve is bound by kernel
                            launches and host polls. */
  int32_t rr_nv;         /* not in the paper: nonzero: every residual replacement (periodic,
                            automated or forced) also recomputes n_i := M^-1 z_i and
                            v_i := A n_i from the replaced z_i (one more SpMV and PREC per
                            replacement), so that the next iteration's l and z recurrences
                            use n_i and v_i of the same z_i.  0 (default): the six quantities
                            of eq:rr only, n_i and v_i keep their pre-replacement values. */
} pbcg_opts;

typedef struct {
  int32_t status;            /* outcome code, same as the return value */
  int32_t iterations;        /* completed iterations */
  int32_t replacements;      /* residual replacements performed */
  int32_t spmvs;             /* sparse matrix-vector products issued */
  double rel_res_recursive;  /* ||r|| / ||b|| of the recursively computed residual */
  double rel_res_true;       /* ||b - A x|| / ||b||, computed in FP64 at the end */
  double elapsed_ms;         /* device time from the first to the last kernel of the solve */
  double rnorm0;             /* ||r_0|| */
  double bnorm;              /* ||b|| */
  int32_t restarts;          /* restarts performed (pbcg_opts.restarts) */
  int32_t single_kernel;     /* 1: the solve ran as the one-workgroup kernel (pbcg_opts.single_kernel) */
} pbcg_stats;

/* Fills `opt` with defaults: tol 1e-10, maxit 10000, rr_period 0, rr_tau 0,
 * check_every 0, transpose 0, no history, use_graph 0, stream NULL, rr_auto 0,
 * rr_eps 0, no bound history, restarts 0, rhat NULL, no bound state, single_kernel 0,
 * rr_nv 0. */
void pbicgstab_default_opts(pbcg_opts* opt);

/*
 * Tuning switches, read from the environment when a solver is created (for
 * measurements and tests; the defaults are the measured best choices):
 *   PBCG_NBLK=n           blocks of the streaming kernels (rounded to a
 *                         multiple of 8, at most 1024)
 *   PBCG_SPMV_BLOCKS=n    work blocks of a stand-alone product (at most 2048)
 *   PBCG_VEC_NT=0..3      non-temporal vector streams (bit 0 phase A, bit 1
 *                         phase B; default on above 192 MB of vectors)
 *   PBCG_SPMV_TILED=0|1   structured products on 16-byte chunks of grid lines
 *   PBCG_FUSE=0|1         structured products inside the phase kernels
 *   PBCG_MARCH3D=0|1      the stand-alone 3D product marching through planes
 *   PBCG_MARCH_ZLEN=n     planes per work item of that product (0: sized to
 *                         the grid)
 *   PBCG_MARCH_PHASE=0|1  phase kernels visiting a 3D grid plane by plane
 *                         (FP32 storage only)
 *   PBCG_PREMULT=0|1      sliced-ELL products reading the M^-1 z, M^-1 w that
 *                         the phase kernels write (Jacobi vector)
 *   PBCG_SELL_LDS=0|1     sliced-ELL iteration products staging each 1024-row
 *                         block's column window in LDS (when it fits)
 *   PBCG_LDS_BLOCKS=n     blocks of that product (0: 256 per window that takes
 *                         more than half a block's LDS, else 512)
 *   PBCG_SMALL_RPT=1|2|4  rows per thread of the single-workgroup solve
 *                         (opt single_kernel; default 2; the automated
 *                         strategy always runs with 2, more than 1024 rows
 *                         with 4)
 * None changes a result bit except PBCG_NBLK, PBCG_MARCH_PHASE and
 * PBCG_SMALL_RPT, which set the order in which the dot products are summed.
 */

/*
 * Bytes of device workspace a handle needs (the ownership model above).
 *   format    : PBCG_CSR, PBCG_ST_2D5, PBCG_ST_3D7 or PBCG_ST_DIA5
 *   n, nnz    : dimension and stored entries (nnz is used for PBCG_CSR only)
 *   width     : PBCG_CSR: the largest number of stored entries in any row and,
 *               with with_transpose, in any column (it bounds every slice of
 *               the sliced-ELL layouts); ignored otherwise.  With
 *               PBCG_PC_BLOCK_JACOBI(b) the stored A M^-1 is bounded by
 *               width * b entries per row (no transposed layout)
 *   precision, precond : as for create
 *   with_transpose : nonzero reserves the transposed layout (PBCG_CSR, DIA5),
 *               which the first transposed solve, apply or gradient builds
 * Returns 0 (and sets the last error) on invalid arguments.  The size covers
 * the 12 solver vectors, x and b (N padded to 2048, in the storage precision
 * and FP64), the reduction partials (32 x 1024 doubles), the device scalars
 * and the matrix layouts (Section 1's A; for the adjoint solve of the
 * differentiable form, A^T).
 */
size_t pbicgstab_workspace_bytes(int format, int64_t n, int64_t nnz, int32_t width,
                                 int precision, int precond, int with_transpose);

/*
 * Create a solver for a CSR matrix (Section 1: A sparse, N x N).
 *   n, nnz          : dimension and number of stored entries (n >= 1)
 *   rowptr, col, val: device arrays, rowptr[n+1] (rowptr[0] = 0,
 *                     nondecreasing, rowptr[n] = nnz), col[nnz] in [0, n),
 *                     val[nnz]; read during the call only (copied to the host,
 *                     where the layout is built); duplicate entries are kept
 *                     and summed in stored order
 *   precision       : PBCG_FP64 or PBCG_MIXED (values rounded once to FP32)
 *   precond         : PBCG_PC_NONE, PBCG_PC_JACOBI (M^-1 = 1/diag, the
 *                     diagonal being the sum of the entries with col == row;
 *                     PBCG_ERR_ZERO_DIAG if one is zero) or
 *                     PBCG_PC_BLOCK_JACOBI(b) (PBCG_ERR_ZERO_DIAG if a
 *                     diagonal block is singular)
 *   workspace, ws_bytes : caller-owned device memory, 256-byte aligned, of at
 *                     least pbicgstab_workspace_bytes(PBCG_CSR, ...) bytes;
 *                     PBCG_ERR_WORKSPACE_TOO_SMALL if the layouts do not fit
 * The matrix is stored in the workspace as sliced ELLPACK (slice height 64)
 * in the stored column order of each row.
 */
int pbicgstab_create_csr(pbcg_handle* out, int64_t n, int64_t nnz, const int32_t* rowptr,
                         const int32_t* col, const double* val, int precision, int precond,
                         void* workspace, size_t ws_bytes, void* stream);

/*
 * Create a solver for a structured operator on a lexicographically ordered
 * grid (p = ix + nx*iy + nx*ny*iz; neighbours outside the grid have no entry,
 * i.e. homogeneous Dirichlet boundaries).
 *   kind : PBCG_ST_2D5, PBCG_ST_3D7 or PBCG_ST_DIA5
 *   dims : host int64[2] or int64[3]
 *   coef : 2D5 / 3D7: host array of the 5 / 7 constants (see the format
 *          enum, ascending column order); DIA5: device array [5*N] (row d =
 *          S, W, C, E, N), read during the call only
 *   workspace, ws_bytes : as for pbicgstab_create_csr (sized for `kind`)
 */
int pbicgstab_create_stencil(pbcg_handle* out, int kind, const int64_t* dims, const double* coef,
                             int precision, int precond, void* workspace, size_t ws_bytes,
                             void* stream);

/*
 * Solve A x = b (or A^T x = b) with pipelined BiCGStab, Algorithm 2, and
 * periodic residual replacement (Section 3.6).
 *   b : device FP64 [n]       right-hand side
 *   x : device FP64 [n]       in: x_0, out: the last iterate
 *   opt: host, see pbcg_opts (NULL = defaults); st: host, may be NULL
 * Blocks the calling thread until the solve has finished.
 */
int pbicgstab_solve(pbcg_handle h, const double* b, double* x, const pbcg_opts* opt,
                    pbcg_stats* st);

/*
 * For callers that cannot allocate (tight serving loops, harnesses that
 * forbid allocation): pbicgstab_solve that allocates nothing.  The
 * reduction scratch -- the partial sums of every global reduction (32 slots x
 * 1024 blocks of FP64, 256 KiB) and the device scalar structs -- is a static
 * device array of the library (its maximum size, about 260 KiB, does not
 * depend on N; each GPU holds one copy until the process ends) instead of
 * the handle's workspace.  Iteration chunks are launched directly (opt
 * use_graph is ignored: instantiating a graph allocates), and a transposed
 * solve needs the transposed layout built beforehand (PBCG_ERR_UNSUPPORTED
 * otherwise).  The array is cleared at the start of each call; calls that
 * overlap on one GPU (from several threads or handles) share it and race.
 * Same arguments, results and blocking behaviour as pbicgstab_solve.
 */
int pbicgstab_solve_noalloc(pbcg_handle h, const double* b, double* x, const pbcg_opts* opt,
                            pbcg_stats* st);

/* Same interface with classic BiCGStab, Algorithm 1 (three global reductions
 * per iteration on the critical path; rr_period is ignored). */
int classic_bicgstab_solve(pbcg_handle h, const double* b, double* x, const pbcg_opts* opt,
                           pbcg_stats* st);

/* y = A x (or A^T x) with FP64 accumulation; x, y device FP64 [n]. */
int pbicgstab_apply(pbcg_handle h, const double* x, double* y, int transpose, void* stream);

/*
 * Gradient of a loss with respect to the stored matrix values, given the
 * adjoint lambda (solution of A^T lambda = dL/dx) and the solution x:
 * dL/da_ij = -lambda_i x_j (from d(A^-1) = -A^-1 dA A^-1).  Output (device FP64):
 *   CSR handle : grad[nnz] in the stored CSR order
 *   DIA5       : grad[5*n], row d = S, W, C, E, N, 0 where the entry does not exist
 *   2D5 / 3D7  : grad[5] / grad[7], the derivative with respect to each
 *                constant stencil coefficient (sum over the rows having it)
 */
int pbicgstab_grad_values(pbcg_handle h, const double* lambda, const double* x, double* grad,
                          void* stream);

/*
 * Replace the matrix values, keeping the pattern (the Jacobi diagonal and the
 * transposed layout follow).  values: CSR order [nnz] (CSR handle), [5*n]
 * (DIA5) or [5]/[7] (stencils); on_device selects a device or host pointer.
 */
int pbicgstab_update_values(pbcg_handle h, const double* values, int on_device, void* stream);

/*
 * Coefficient-field operators (DIA5 handles): assemble
 * -div(kappa grad u) + (cx, cy).grad u, scaled by h^2, from node values
 * kappa (device FP64 [n]): face coefficient = mean of the two node values, a
 * boundary face takes the node's own value; E/W get +/- cx h/2, N/S +/- cy h/2.
 */
int pbicgstab_dia5_assemble_kappa(pbcg_handle h, const double* kappa, double cx, double cy,
                                  double hgrid, void* stream);

/*
 * dL/dkappa (device FP64 [n]) for the assembly above, from lambda and x:
 * an interior face contributes -(lambda_p - lambda_q)(x_p - x_q)/2 to each of
 * its nodes, a boundary face -lambda_p x_p to its node.
 */
int pbicgstab_dia5_kappa_grad(pbcg_handle h, const double* lambda, const double* x,
                              double* grad_kappa, void* stream);

/*
 * Copy an internal solver vector to `out` (device FP64 [n]) for diagnostics:
 * 0 r0 (shadow residual), 1 r, 2 g, 3 s, 4 l, 5 z, 6 k, 7 w, 8 t, 9 v,
 * 10 x (the iterate), 11 dinv (Jacobi diagonal, 1 without preconditioner).
 * For classic solves 2 holds p, 3 s and 9 y.
 */
int pbicgstab_get_vector(pbcg_handle h, int which, double* out, void* stream);

/*
 * Kernel timing for roofline measurements.  Launches one kernel of the
 * Algorithm 2 iteration `reps` times back to back on the handle's stream and
 * returns the average duration per launch, measured with HIP events recorded
 * on that stream:
 *   0 phase A (g, s, l, z recurrences + GLRED 1 partials)
 *   1 PREC + SPMV  v = A M^-1 z  (with the GLRED 1 final blocks)
 *   2 phase B (x, r, k, w recurrences + GLRED 2 partials)
 *   3 PREC + SPMV  t = A M^-1 w  (with the GLRED 2 reduction, scalars not updated)
 *   4 one full iteration (0-3)
 *   5 a plain copy of N_pad doubles (2 x 8 N bytes), the bandwidth reference
 *   6 PREC + SPMV  v = A M^-1 z  without any final reduction
 *   7 the GLRED 2 final reduction alone (scalars not updated)
 * When the iteration computes the products inside the phase kernels
 * (constant 2D stencils and DIA5; 3D stencils with FP32 storage), 0 and 2
 * time those kernels (phase B then includes the GLRED 1 final), 1 a
 * stand-alone GLRED 1 final for reference, 3 the GLRED 2 final kernel, 4
 * phase A + phase B + GLRED 2 final, and 6 the stand-alone product.
 * With a sliced-ELL matrix and a Jacobi vector the products 1, 3 and 6 read
 * the copy of their input that the phase kernels have already multiplied by
 * M^-1 (as the iteration does), not z or w and dinv.
 * The solver vectors are overwritten (run it after, not between, the solves
 * whose results are needed); every later solve reinitialises them.
 */
int pbicgstab_time_kernel(pbcg_handle h, int kernel, int reps, double* avg_ms, void* stream);

/* Problem size, stored entries, and the workspace bytes the handle uses. */
int pbicgstab_info(pbcg_handle h, int64_t* n, int64_t* nnz, int64_t* device_bytes);

void pbicgstab_destroy(pbcg_handle h);

/* Message of the last error on this thread ("" if none). */
const char* pbicgstab_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PBICGSTAB_H */
