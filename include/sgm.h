/*
 * sgm.h -- C ABI of the MI355X (gfx950) adaptive s-step GMRES library.
 *
 * Method: Z. Xu, J. J. Alonso, E. Darve, "A numerically stable communication
 * avoiding s-step GMRES algorithm" (arXiv 2303.08953): Alg. 4 (adaptive
 * s-step GMRES with BCGS2 and partial CholQR), Alg. 3 (partial Cholesky with
 * an incremental condition estimator), the scaled Newton basis of Sec. 3.4
 * (Eqs. (scalednewton), (newtonrecurrence), (scalingcoeff)) and the initial
 * step-size estimator of Sec. 3.5 (Eq. (auxiliarymatrix)).
 *
 * Conventions for every entry point:
 *  - Pointers are DEVICE pointers (hipMalloc'd or torch CUDA tensors on ROCm)
 *    unless the comment says (host).
 *  - All GPU work is enqueued on `stream` (a hipStream_t passed as void*;
 *    NULL means the default stream).  Entry points that return host-visible
 *    results (sgm_solve, sgm_block_orth, sgm_shifts) synchronise `stream`
 *    before returning, on their error returns too (SGM_EINVAL aside, which
 *    enqueues nothing); the others return after enqueueing.
 *  - The caller owns every buffer it passes.  The library allocates device
 *    memory only in sgm_matrix_create (the analysed copies of the matrix)
 *    and sgm_matrix_ilu0 (its ILU(0) factors) and frees it in
 *    sgm_matrix_destroy.  Scratch for a solve is the caller's
 *    workspace, sized by sgm_workspace_size.  The one exception is
 *    sgm_block_orth_noalloc, whose scratch is a static device array of the
 *    library (24 MiB per GPU, for the life of the process).
 *  - Arguments are validated on the host before any HIP call; invalid ones
 *    return SGM_EINVAL and enqueue nothing.  HIP errors return SGM_EHIP.
 *    sgm_last_error() gives a thread-local message for the last failure.
 *    No C++ exception crosses this interface.
 *  - One matrix handle must not be used by two concurrent calls.
 */
#ifndef SGM_H
#define SGM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SGM_OK = 0,
  SGM_NOT_CONVERGED = 1, /* caps reached; x holds the last iterate        */
  SGM_EINVAL = -1,       /* invalid argument (nothing was enqueued)       */
  SGM_EHIP = -2,         /* HIP runtime error                             */
  SGM_ENOMEM = -3,       /* device allocation failed (matrix create only) */
  SGM_ENUMERIC = -4      /* NaN/Inf in a residual or in the shifts         */
} sgm_status;

typedef enum {
  SGM_BASIS_SCALED_NEWTON = 0, /* Eq. (scalednewton), gamma = |mean - theta| */
  SGM_BASIS_NEWTON = 1,        /* Eq. (newton), gamma = 1                    */
  SGM_BASIS_MONOMIAL = 2       /* Eq. (monomial), p_j(A) = A^j               */
} sgm_basis;

typedef enum {
  SGM_PRECOND_NONE = 0,
  SGM_PRECOND_JACOBI = 1,  /* right Jacobi = column scaling A D^{-1}        */
  SGM_PRECOND_ILU0 = 2     /* right ILU(0), M = L U (the preconditioner of
                              the 2D Laplace test of Sec. 4.3); float64,
                              forward solves only; the factors come from
                              sgm_matrix_ilu0                              */
} sgm_precond;

typedef enum {
  SGM_PREPHASE_CGS2 = 0,     /* one column per step (column-wise Arnoldi)  */
  SGM_PREPHASE_MONOMIAL = 1  /* adaptive monomial-basis s-step blocks      */
} sgm_prephase;

typedef enum {
  SGM_ORTH_BCGS2 = 0,      /* Alg. 4: both BCGS passes take their Gram
                              matrix from the updated block               */
  SGM_ORTH_BCGS2_PYTH = 1  /* second pass takes it by Pythagoras,
                              G2 = Q1^T Q1 - R2^T R2 (Q1 = first-pass
                              block, R2 = its projection), so the second
                              update and triangular solve are one pass
                              over the block (not in the paper)           */
} sgm_orth;

typedef enum {
  SGM_FP64 = 0,    /* everything in double precision                        */
  SGM_FP32_IR = 1  /* float32 inner s-step cycles inside float64 refinement */
} sgm_precision;

typedef struct sgm_matrix_s* sgm_matrix;

/* ---------------------------------------------------------------- matrix */

/* Analyse a square CSR matrix (0-based, int32 indices, column indices
 * sorted or not, no duplicates required) for the solver: builds on the GPU a
 * SELL-C layout with C = 64 (one wavefront per 64-row slice) holding float64
 * and float32 values, the diagonal, and the transposed SELL structure with
 * the permutation that maps values to it (for adjoint solves).
 * row_ptr[n+1], col[nnz], val[nnz] are read (device) and not kept.
 * n >= 1, 0 <= nnz < 2^31, every column index in [0, n).  *out (host)
 * receives the handle.  The matrix-analysis step of the hot path; it is not
 * part of a solve's time. */
sgm_status sgm_matrix_create(int64_t n, int64_t nnz, const int32_t* row_ptr,
                             const int32_t* col, const double* val,
                             void* stream, sgm_matrix* out);

/* Replace the values (same sparsity): val[nnz] (device), CSR order. */
sgm_status sgm_matrix_update_values(sgm_matrix A, const double* val,
                                    void* stream);

sgm_status sgm_matrix_destroy(sgm_matrix A);

/* ILU(0) factors of A for right preconditioning (SGM_PRECOND_ILU0; the
 * preconditioner of the 2D Laplace test with an ILU preconditioner, Sec.
 * 4.3).  Zero fill-in: Gaussian elimination in row order that drops every
 * update outside the pattern of A, so L (unit lower) and U (upper) have A's
 * pattern and (L U)_ij = a_ij at every stored (i, j).  Everything runs on
 * the GPU: the levels of the forward and backward substitutions (a row's
 * level is one more than the highest among the rows it depends on), rows
 * sorted by level, and the factorisation level by level.  Needs every
 * diagonal entry stored and column indices sorted within each row
 * (SGM_EINVAL otherwise); a zero or non-finite pivot gives SGM_ENUMERIC.
 * The factors belong to the handle (device memory allocated here, freed by
 * sgm_matrix_destroy or a later call) and are recomputed by
 * sgm_matrix_update_values.  levels (host, 2 entries, may be NULL) receives
 * the level counts of the forward and backward substitutions.
 * Synchronises `stream`. */
sgm_status sgm_matrix_ilu0(sgm_matrix A, void* stream, int32_t* levels);

/* z = M^{-1} r = U^{-1} (L^{-1} r) with the ILU(0) factors: r, z double[n]
 * (device, may alias).  One workgroup walks the levels of each
 * substitution in order. */
sgm_status sgm_ilu0_apply(sgm_matrix A, const double* r, double* z,
                          void* stream);

/* Copies the ILU(0) factors into lu[nnz] (device), in the CSR order of A:
 * the multipliers of L at the strict lower entries, U on and above the
 * diagonal. */
sgm_status sgm_ilu0_factors(sgm_matrix A, double* lu, void* stream);

/* Sizes of an analysed matrix (host outputs, each may be NULL): n, nnz,
 * the padded SELL-C-64 entry count of A, and index_bytes[2] = the bytes
 * per column index the SpMV of A and of A^T reads: 2 when every group of 64
 * entries (one slice position) has its columns within 65535 of each other
 * after removing the lane offset (stencils, banded matrices), else 4. */
sgm_status sgm_matrix_info(sgm_matrix A, int64_t* n, int64_t* nnz,
                           int64_t* sell_nnz, int32_t* index_bytes);

/* y = A x (transpose = 0) or y = A^T x (transpose = 1).
 * precision SGM_FP64: x, y are double[n]; SGM_FP32_IR: float[n] with the
 * float32 values.  The single sparse mat-vec of Alg. 1/4 (MPK building
 * block). */
sgm_status sgm_spmv(sgm_matrix A, int transpose, sgm_precision precision,
                    const void* x, void* y, void* stream);

/* ---------------------------------------------------------------- solve */

typedef struct {
  int32_t s_max;          /* user initial step size s0 (Alg. 4); >= 1        */
  int32_t restart;        /* m, basis vectors per cycle (Alg. 4); >= 1       */
  int32_t max_restarts;   /* restarts after the first cycle; >= 0            */
  double tol;             /* on ||b - A x|| / ||b - A x0|| (Sec. 4); > 0     */
  sgm_precond precond;    /* right preconditioner (see sgm_precond)         */
  sgm_basis basis;
  sgm_precision precision;
  double omega;           /* Alg. 3 bound; 0 => 0.1 u^{-1/2} of the Gram's
                             precision (9.49e6 in float64, 409.6 float32)    */
  double omega_est;       /* Sec. 3.5 threshold; 0 => same rule              */
  int32_t use_estimator;  /* 1 => s_init = min(s_max, s0*) (scaled Newton)   */
  int32_t transpose;      /* 1 => solve A^T x = b (adjoint solves)           */
  double inner_tol;       /* SGM_FP32_IR: relative tolerance of an inner
                             float32 cycle (default 1e-6)                    */
  int32_t max_outer;      /* SGM_FP32_IR: refinement steps cap (default 200)*/
  int32_t ritz_reuse;     /* 1 (default): the Ritz pre-phase columns are the
                             first iterations of the first cycle             */
  const double* shifts_host; /* optional (host) Ritz values as (re, im)
                             pairs; when given, the pre-phase is skipped     */
  int32_t n_shifts;       /* number of (re, im) pairs in shifts_host         */
  sgm_prephase prephase;  /* how the Ritz pre-phase builds its m0 columns:
                             SGM_PREPHASE_CGS2 (default) one column per step
                             (column-wise CGS2 Arnoldi, Sec. 3.4);
                             SGM_PREPHASE_MONOMIAL in monomial-basis blocks
                             of Alg. 4 with partial CholQR adapting their
                             size (same Krylov space and Hessenberg matrix,
                             block-wise passes over the basis)            */
  int32_t prephase_s;     /* first block size of the monomial pre-phase
                             (default 8); >= 1                               */
  sgm_orth orth;          /* second BCGS pass of blocks with s >= 2 (the
                             column-wise s = 1 steps always use Alg. 4's);
                             default SGM_ORTH_BCGS2                          */
  int32_t mpk_depth;      /* matrix powers steps per pass over the matrix
                             (temporal blocking, 1..4; default 1 = one SpMV
                             launch per step).  Results are bitwise those
                             of depth 1; matrices with fewer than three row
                             slabs of at least their bandwidth run depth 1 */
} sgm_opts;

/* Fills *o (host) with the defaults: s_max 8, restart 64, max_restarts 100,
 * tol 1e-10, no preconditioner, scaled Newton, FP64, omega/omega_est rule,
 * estimator on, inner_tol 1e-6, max_outer 200, ritz_reuse 1, column-wise
 * pre-phase, prephase_s 8, orth SGM_ORTH_BCGS2. */
void sgm_opts_default(sgm_opts* o);

typedef struct {
  int32_t iters;          /* Hessenberg columns built, all cycles (inner
                             iterations for SGM_FP32_IR)                     */
  int32_t restarts;       /* restarts (FP64) / inner cycles - 1 (FP32_IR)    */
  int32_t outer_iters;    /* refinement steps (SGM_FP32_IR), else 0          */
  int32_t s0_est;         /* estimator's s0* (0 if not run)                  */
  int32_t s_init;         /* step size used at each cycle start              */
  int32_t n_hist;         /* full length of the residual history             */
  int32_t n_blocks;       /* full length of the step-size history            */
  int32_t n_shifts;       /* number of Ritz values used as shifts            */
  int32_t gamma_guard_hits; /* gamma_k raised by the zero guard              */
  double rel_res_true;    /* final ||b - A x|| / ||b - A x0|| (float64)      */
  double rel_res_est;     /* last Givens estimate                            */
  double t_phase_ms[8];   /* 0 setup (host wall), 1 pre-phase + shifts (host
                             wall), 2 MPK, 3 block orthogonalisation with
                             the Hessenberg recovery, Givens rotations and
                             convergence test (GPU time between HIP events on
                             the solve's stream: from a block's last matrix
                             powers step to the next block's first), 4 unused
                             (0), 5 cycle end: update + true residual (host
                             wall), 6 refinement loop (host wall), 7 total
                             (host wall)                                     */
  int64_t n_spmv;         /* SpMV launches of the matrix powers kernel       */
  double t_spmv_ms;       /* their GPU time: one HIP event pair around each
                             block's matrix powers steps (queued back to
                             back; the first few may be queued behind the
                             previous block, see sgm_solve)                  */
  int32_t mpk_depth;      /* depth the matrix powers kernel ran at           */
  int64_t mpk_slab_rows;  /* rows per slab of the fused kernel (0: depth 1) */
} sgm_info;

/* Bytes of device workspace sgm_solve needs for this matrix and options. */
sgm_status sgm_workspace_size(sgm_matrix A, const sgm_opts* o,
                              size_t* bytes /* host */);

/* Adaptive s-step GMRES(m) with restarts (Alg. 4): b[n] (device, float64),
 * x0[n] (device, may be NULL for zero, may alias x), x[n] (device output).
 * ws: device workspace of ws_bytes >= sgm_workspace_size.  res_hist (host,
 * capacity res_cap, may be NULL) receives the Givens relative-residual
 * estimate after every iteration; s_hist (host, capacity s_cap, may be NULL)
 * the accepted block size of every block (0 marks a breakdown block).
 * info (host, may be NULL).  Returns SGM_OK when the true relative residual
 * reaches tol, SGM_NOT_CONVERGED when the caps are hit first.
 * Scheduling: after each block's tail the first few matrix powers steps of
 * the next block are queued at once, on the assumption that every column
 * of the block is accepted (the next block then has the same size); each
 * of them reads a control word the tail wrote and does nothing when the
 * assumption failed or the cycle ended, and the host queues the block
 * again in full.  The host waits for a tail by polling a word the tail
 * writes into mapped host memory.  Results do not depend on this. */
sgm_status sgm_solve(sgm_matrix A, const double* b, const double* x0,
                     double* x, const sgm_opts* o, void* ws, size_t ws_bytes,
                     void* stream, double* res_hist, int32_t res_cap,
                     int32_t* s_hist, int32_t s_cap, sgm_info* info);

/* grad_val[k] = -lambda[row(k)] * x[col(k)] for every nonzero k in CSR
 * order: the gradient of a loss through x = A^{-1} b with respect to A's
 * values, given the adjoint solution lambda of A^T lambda = dL/dx.
 * lambda[n], x[n], grad_val[nnz] are device float64. */
sgm_status sgm_grad_vals(sgm_matrix A, const double* lambda, const double* x,
                         double* grad_val, void* stream);

/* ------------------------------------------------------------ hot steps
 * The steps of one s-step block, callable on their own (they are what
 * sgm_solve runs).  Q is column-major with leading dimension ldq (a multiple
 * of 64 elements, >= n, rows n..ldq-1 zero), float64 (SGM_FP64) or float32
 * (SGM_FP32_IR). */

/* Matrix powers kernel of Alg. 4 (Eq. (newtonrecurrence)): for
 * j = 0..s-1,  Q[:, c+j+1] = ((A - theta_j) Q[:, c+j] - delta_j Q[:, c+j-1])
 * / gamma_j, where records (device, double[3*n_rec]) hold (theta, gamma,
 * delta) per step and are used cyclically (j mod n_rec); delta_0 is
 * ignored.  c = start column.  transpose selects A^T. */
sgm_status sgm_mpk(sgm_matrix A, int transpose, sgm_precision precision,
                   void* Q, int64_t ldq, int32_t c, int32_t s,
                   const double* records, int32_t n_rec, void* stream);

/* sgm_mpk with the fused square-sum epilogue of the matrix powers kernel
 * (Alg. 4, Eq. (newtonrecurrence)): the same columns, bitwise, and
 * norms2[j] (device, double[s]) = sum over the rows of Q[:, c+j+1]^2 as
 * stored (float64 sums, also for SGM_FP32_IR), taken by the SpMV that
 * forms the column, with no extra pass over Q: the growth of the basis
 * vectors the paper plots for the monomial and Newton bases.  work
 * (device, double[work_len], work_len >= ceil(n / 256)) holds the
 * per-workgroup partial sums of one step at a time; results are
 * deterministic (fixed summation order).  Other arguments as in sgm_mpk;
 * NULL norms2 or work, or a shorter work, return SGM_EINVAL when s > 0. */
sgm_status sgm_mpk_norms(sgm_matrix A, int transpose, sgm_precision precision,
                         void* Q, int64_t ldq, int32_t c, int32_t s,
                         const double* records, int32_t n_rec, double* norms2,
                         double* work, int64_t work_len, void* stream);

/* The matrix powers kernel of sgm_mpk with temporal blocking (the
 * communication-avoiding matrix powers idea of Sec. 2, applied to the
 * cache hierarchy): `depth` (1..4) consecutive steps per pass over the
 * matrix.  The rows are cut into slabs of at least the matrix bandwidth
 * max |column - row|; launch L computes step j on slab L - 2 j, so every
 * slab's matrix rows serve its `depth` steps within a few launches, while
 * they are still cached.  Q, ldq, c, s, records, n_rec, transpose and
 * precision as in sgm_mpk; the results are bitwise those of sgm_mpk
 * (every row is computed by the same arithmetic).  *slab_rows (host, may
 * be NULL) receives the slab height, or 0 when the matrix has fewer than
 * three such slabs and the call ran one step per launch. */
sgm_status sgm_mpk_fused(sgm_matrix A, int transpose, sgm_precision precision,
                         void* Q, int64_t ldq, int32_t c, int32_t s,
                         const double* records, int32_t n_rec, int32_t depth,
                         void* stream, int64_t* slab_rows);

/* Block orthogonalisation of the s columns Q[:, i .. i+s-1] against the
 * orthonormal Q[:, 0 .. i-1]: BCGS2 with two partial CholQR passes
 * (Alg. 4's block orthogonalisation, Alg. 3 with the condition bound
 * omega); orth selects how the second pass forms its Gram matrix (s >= 2;
 * see sgm_orth).  On return
 * (host outputs): *p = accepted size (0 = breakdown), Q[:, i .. i+p-1] hold
 * the new orthonormal vectors, R_top (host, i x s, column-major, ld i) and
 * R_kk (host, s x s, ld s) hold R(1:i, k) and R(k, k) in their leading p
 * columns.  ws: device workspace of at least sgm_block_ws_size bytes.
 * n_rows = number of meaningful rows. */
size_t sgm_block_ws_size(int64_t n_rows, int32_t i, int32_t s);
sgm_status sgm_block_orth(sgm_precision precision, int64_t n_rows, void* Q,
                          int64_t ldq, int32_t i, int32_t s, double omega,
                          sgm_orth orth, void* ws, size_t ws_bytes,
                          void* stream, int32_t* p, double* R_top,
                          double* R_kk);

/* sgm_block_orth without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same block
 * orthogonalisation, arguments, outputs and errors as sgm_block_orth.  It
 * calls no hipMalloc/hipFree and takes no workspace: its scratch (partial
 * sums, the Gram matrices, both partial Cholesky factors and inverses, the
 * control words) is a device array of 24 MiB inside the library, one copy
 * per GPU, held until the process ends.  Limits: 1 <= s <= 64 and
 * i + s <= 256; larger blocks return SGM_EINVAL (use sgm_block_orth).
 * Every call on one GPU uses that GPU's array, and it keeps the last
 * call's contents: calls that overlap on one GPU (two host threads, or
 * two streams whose calls are not ordered) race and give wrong results.
 * Like sgm_block_orth it synchronises `stream` before returning. */
sgm_status sgm_block_orth_noalloc(sgm_precision precision, int64_t n_rows,
                                  void* Q, int64_t ldq, int32_t i, int32_t s,
                                  double omega, sgm_orth orth, void* stream,
                                  int32_t* p, double* R_top, double* R_kk);

/* Shifts from a Hessenberg matrix (Sec. 3.4-3.5) computed on the GPU:
 * H (device, leading m0 x m0 block of an upper Hessenberg matrix,
 * column-major with ld ldh, 1 <= m0 <= 1024) -> Ritz values by the Francis
 * double-shift QR iteration, modified Leja order, (scaled) Newton
 * recurrence records and the estimator's s0*.  ws: device workspace of at
 * least sgm_shifts_ws_size(m0) bytes.  Outputs (host): ritz_re/ritz_im[m0]
 * in Leja order, records[3*m0] as (theta, gamma, delta) per step, *s0 (0
 * unless basis is scaled Newton and omega_est > 0), *guard_hits.  eps =
 * unit round-off used in Eq. (auxiliarymatrix).  Returns SGM_ENUMERIC if
 * the QR iteration does not converge or a Ritz value is not finite. */
size_t sgm_shifts_ws_size(int32_t m0);
sgm_status sgm_shifts(const double* H, int32_t ldh, int32_t m0,
                      sgm_basis basis, double eps, double omega_est,
                      void* ws, size_t ws_bytes, void* stream,
                      double* ritz_re, double* ritz_im, double* records,
                      int32_t* s0, int32_t* guard_hits);

/* ---------------------------------------------------------------- misc */
const char* sgm_status_string(sgm_status s);
const char* sgm_last_error(void);
/* 1 when the library was built for gfx950 and a GPU is visible. */
int sgm_device_ok(void);

#ifdef __cplusplus
}
#endif
#endif /* SGM_H */
