/*
 * pbcgs -- pipelined BiCGStab with residual replacement on one MI355X (gfx950).
 *
 * C ABI of the HIP library libpbcgs.so.  It solves A x = b for a sparse A
 * (CSR, a matrix-free constant-coefficient 5/7-point stencil, or the
 * matrix-free variable-coefficient 27-point convection-diffusion operator) with the
 * Krylov methods of S. Cools and W. Vanroose, "The communication-hiding
 * pipelined BiCGStab method for the parallel solution of large unsymmetric
 * linear systems" (arXiv 1612.01395): the BiCGStab variants for unsymmetric
 * A, and the CG family the paper derives its framework on for symmetric
 * positive definite A:
 *
 *   PBCGS_BICGSTAB       standard BiCGStab, the paper's Algorithm 7, or its
 *                        right-preconditioned form Algorithm 10 (Section 3.6);
 *   PBCGS_PBICGSTAB      pipelined BiCGStab, Algorithm 9 (Section 3.3), or the
 *                        preconditioned pipelined form Algorithm 11 (Section 3.6);
 *   PBCGS_PBICGSTAB_RR   Algorithm 9/11 with residual replacement every k
 *                        iterations (Section 4.2);
 *   PBCGS_CA_BICGSTAB    communication-avoiding BiCGStab, Algorithm 8
 *                        (Section 3.1): two reduction phases like p-BiCGStab
 *                        but no overlap, so four kernel boundaries per
 *                        iteration.  No preconditioner, or Jacobi as
 *                        PBCGS_PRECOND_JACOBI_FOLDED; binary64; not batched;
 *   PBCGS_CG             preconditioned CG, Algorithm 2 (Section 2), three
 *                        kernel boundaries per iteration;
 *   PBCGS_CGCG           Chronopoulos & Gear CG, Algorithm 4 (Section 2): one
 *                        reduction phase, two kernel boundaries;
 *   PBCGS_PIPE_CG        pipelined CG, Algorithm 6 (Section 2): its reduction
 *                        and its SpMV both use only the previous iteration's
 *                        vectors, so one kernel boundary per iteration.
 *                        The CG family needs a symmetric positive definite A
 *                        (not checked) and takes Jacobi as PBCGS_PRECOND_JACOBI
 *                        (M^{-1} applied as the algorithms write it; the folded
 *                        form A M^{-1} is not symmetric); binary64; not batched.
 *
 * Right preconditioning solves A M^{-1} y = b, M x = y (Section 3.6).  The only
 * preconditioner is Jacobi, M = diag(A).  The stopping test is
 * ||r_i||_2 / ||r_0||_2 <= tol on the recursive residual (Section 4.1).
 *
 * Arithmetic contract (FP64): every + and * is one IEEE binary64 operation in
 * the order the paper writes it (no fused multiply-add); each SpMV row is
 * summed in stored column order from 0.0; a dot product is the sum of the
 * rounded products in pairwise order (balanced binary tree over the index
 * range padded with zeros to a power of two) plus 0.0.  Results therefore do
 * not depend on the launch configuration and are reproducible bit for bit.
 *
 * Conventions of every call:
 *  - array arguments are DEVICE pointers unless stated otherwise; the library
 *    borrows them and never frees them;
 *  - a negative return value is an API or runtime error (see pbcgs_status);
 *    then outputs are untouched and pbcgs_last_error() describes the cause;
 *  - a context serialises all work on one HIP stream; a context is not
 *    thread-safe, two contexts on the same device are independent.
 */
#ifndef PBCGS_H
#define PBCGS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pbcgs_ctx_s* pbcgs_ctx_t;
typedef struct pbcgs_op_s* pbcgs_op_t;

/* Return codes.  Non-negative: numerical outcome of a solve (x holds the last
 * iterate).  Negative: the call failed and changed nothing. */
typedef enum {
    PBCGS_SUCCESS = 0,            /* ||r_i|| / ||r_0|| <= tol (or r_0 = 0)               */
    PBCGS_MAXIT = 1,              /* maxit iterations done without meeting tol             */
    PBCGS_BREAKDOWN = 2,          /* a denominator of the method vanished, or omega = 0    */
    PBCGS_NONFINITE = 3,          /* a reduced scalar became Inf or NaN                    */
    PBCGS_ERR_INVALID_ARG = -1,   /* bad pointer, size, option or matrix structure         */
    PBCGS_ERR_ALLOC = -2,         /* device memory allocation failed                       */
    PBCGS_ERR_HIP = -3,           /* a HIP runtime call failed                             */
    PBCGS_ERR_UNSUPPORTED = -4    /* valid request the library does not implement          */
} pbcgs_status;

enum {
    PBCGS_BICGSTAB = 0,
    PBCGS_PBICGSTAB = 1,
    PBCGS_PBICGSTAB_RR = 2,
    PBCGS_CA_BICGSTAB = 3,
    PBCGS_CG = 4,
    PBCGS_CGCG = 5,
    PBCGS_PIPE_CG = 6
};
/* Preconditioners.  JACOBI applies M^{-1} = diag(dinv) inside Algorithm 10 / 11
 * (the hatted vectors of Section 3.6).  JACOBI_FOLDED is the same right
 * preconditioning with the operator formed: the unpreconditioned Algorithm 7 / 9
 * runs on A M^{-1} (entries a_ij * dinv_j) from y_0 = x_0 / dinv and returns
 * x = dinv * y.  In exact arithmetic both give the same iterates x_i; the folded
 * form moves fewer vectors per iteration (no hatted copies).  With a stencil
 * it needs a constant diagonal (ERR_UNSUPPORTED otherwise). */
enum { PBCGS_PRECOND_NONE = 0, PBCGS_PRECOND_JACOBI = 1, PBCGS_PRECOND_JACOBI_FOLDED = 2 };
/* Precision.  FP64: every operation in binary64.  FP32_RR64 (precision form,
 * p-BiCGStab with residual replacement only, preconditioner NONE or
 * JACOBI_FOLDED): binary32 vectors, SpMV on the operator rounded to binary32,
 * recurrences and dot products (binary32 pairwise sums); binary64 residual
 * replacement (Section 4.2: r = b - A x, w = A r, s = A p, z = A s, each
 * rounded once when stored), x update and alpha, beta, omega.  The setup is a
 * replacement.  When the binary32 recursive residual passes tol, the binary64
 * true residual ||b - A x|| / ||r_0|| decides: SUCCESS if it is below tol too,
 * otherwise a replacement in that iteration and the iteration goes on.
 * rr_period = 0 leaves only those confirmation replacements.  CSR operators
 * need nnz floats of context-owned workspace (plus nnz doubles when folded). */
enum { PBCGS_FP64 = 0, PBCGS_FP32_RR64 = 1 };

/* Solver options (host struct). */
typedef struct {
    int32_t variant;     /* PBCGS_BICGSTAB, PBCGS_PBICGSTAB, PBCGS_PBICGSTAB_RR,
                            PBCGS_CA_BICGSTAB, PBCGS_CG, PBCGS_CGCG or PBCGS_PIPE_CG       */
    int32_t precond;     /* PBCGS_PRECOND_NONE, _JACOBI or _JACOBI_FOLDED                  */
    int32_t precision;   /* PBCGS_FP64 or PBCGS_FP32_RR64                                   */
    int32_t maxit;       /* iteration budget, >= 0                                          */
    double tol;          /* relative tolerance on the recursive residual, >= 0              */
    int32_t rr_period;   /* k: replace in iteration i when (i+1) mod k == 0; 0 = never      */
    int32_t rr_max;      /* at most this many replacements; -1 = unlimited                  */
    int32_t check_every; /* iterations between host polls of the device status; 0 = auto   */
    int32_t flags;       /* bit 0: launch each kernel directly instead of through a
                            captured HIP graph; bit 1: time the fused kernels with events;
                            bit 2: alpha_{i+1} of PBICGSTAB(_RR) and CA_BICGSTAB by
                            eq. (5), the form without (r0, s_i), instead of eq. (3)
                            (Section 3.1); bit 3: read the caller's int32 col_idx
                            even when the operator holds a compact copy (implies
                            bit 4); bit 4: read the CSR arrays even when the
                            operator has a diagonal layout (pbcgs_op_diagonals);
                            bit 5 (a test hook): fill the solve's workspace --
                            vectors with their padding, partial sums, the
                            diagonal layout's values, A M^{-1} and binary32
                            values -- with NaN bits before the solve writes it,
                            so that a read of anything the solve did not write
                            (the index -1 vectors of the pipelined methods, say)
                            turns the results into NaN; results are otherwise
                            unchanged (pbcgs_solve, pbcgs_solve_noalloc and
                            pbcgs_solve_batched)                                   */
    double* history;     /* nullable DEVICE array of maxit+1 doubles: history[i] =
                            ||r_i|| / ||r_0|| after i iterations (history[0] = 1)           */
} pbcgs_opts;

/* Solver report (host struct), filled by pbcgs_solve. */
typedef struct {
    int32_t iters;           /* completed x-updates                                       */
    int32_t n_rr;            /* residual replacements performed                           */
    int32_t status;          /* pbcgs_status of the numerical outcome                     */
    int32_t syncs_per_iter;  /* kernel boundaries of one regular iteration (1 to 5)       */
    double relres_rec;       /* last ||r_i|| / ||r_0|| of the recurrence                  */
    double relres_true;      /* ||b - A x|| / ||r_0|| of the returned x                   */
    double ms;               /* device time (HIP events) from the setup to the last
                                reduction, ms; the true residual is not included          */
    double kernel_ms[2];     /* with flags bit 1: summed duration of two kernels of the
                                iteration -- p-BiCGStab: t-phase, v-phase; BiCGStab and
                                CA-BiCGStab: the two SpMV kernels; CG: s = A p and the
                                x, r, u update; Chronopoulos & Gear: the update and
                                w = A u; p-CG: its one kernel (slot 0)                    */
    int32_t kernel_calls[2]; /* launches timed for kernel_ms                              */
    int32_t rows_per_wave_blocks; /* the launch shape that ran: 64-row blocks per wave,  */
    int32_t workgroups;           /* and workgroups of 256 threads (the system's own in a
                                     batch)                                               */
    int32_t value_codes;          /* 1 when the solve read its diagonal layout's values
                                     (binary64, or binary32 and binary64 for the
                                     precision form) as one-byte codes into a table of
                                     each diagonal's distinct values (value indexing, used
                                     for layouts of at most 8 diagonals none of which
                                     holds more than 16 distinct values, from 2^18 rows,
                                     without a Jacobi vector; same results)             */
} pbcgs_info;

/* Create a context on HIP device `device` working on stream `hip_stream`
 * (a hipStream_t; NULL = the null stream).  *out receives the handle. */
int pbcgs_ctx_create(int device, void* hip_stream, pbcgs_ctx_t* out);

/* Free the context's workspace.  Operators made on it must be destroyed first. */
int pbcgs_ctx_destroy(pbcgs_ctx_t ctx);

/* Message describing the last error on ctx (NULL ctx: the last global error). */
const char* pbcgs_last_error(pbcgs_ctx_t ctx);

/* Static name of a status code. */
const char* pbcgs_status_str(int status);

/*
 * CSR operator (Section 2: the SPMV building block): n x n, int32 row_ptr[n+1]
 * with row_ptr[0] = 0 and row_ptr[n] = nnz, int32 col_idx[nnz] in [0, n),
 * float64 val[nnz].  Each row is applied in stored order; ascending columns
 * are the convention, not a requirement: a row stored in another order is
 * summed in that order (so the result equals a row-by-row loop over the
 * stored entries, bit for bit, but not the ascending-order sum).  The
 * arrays are borrowed and must outlive the operator.  The structure is
 * validated on the device (ERR_INVALID_ARG if malformed).
 * When every column j of a row i satisfies -32768 <= j - (i & ~63) <= 32767
 * (banded matrices such as the paper's stencil discretisations), the operator
 * also keeps a compact copy of the columns as int16 offsets from the row's
 * 64-row block start (PBCGS_COLS_BLOCK16).  Otherwise, when the matrix has at
 * most 64 distinct diagonals j - i (stencils of any size), it keeps 16-bit
 * codes of (i & 63, the diagonal's index) with a 64-entry diagonal table
 * (PBCGS_COLS_DIAG16).  Either copy takes 2 nnz bytes of device memory, freed
 * with the operator, and the solves and pbcgs_spmv read it instead of
 * col_idx: 2 instead of 4 bytes per non-zero and product, with identical
 * results.  Values may change between calls; row_ptr and col_idx must not
 * change while the operator exists.
 * One launch covers at most 1024 workgroups x 4 waves x 1024 blocks x 64 rows,
 * so n <= 268,435,456, and nnz <= 2^31 - 1025 (int32 indexing); ERR_UNSUPPORTED
 * beyond.
 */
int pbcgs_op_csr(pbcgs_ctx_t ctx, int32_t n, int64_t nnz, const int32_t* row_ptr,
                 const int32_t* col_idx, const double* val, pbcgs_op_t* out);

/*
 * Matrix-free stencil operator (the SPMV building block of Section 2 without
 * a stored matrix) on the interior nodes of an nx x ny x nz grid, rows
 * ordered x fastest, Dirichlet boundaries (entries that would leave the grid
 * are dropped).  npts = 5 (nz must be 1), 7 or 27.  The terms of a row, in
 * ascending column order: 5-point {-y, -x, centre, +x, +y}; 7-point {-z, -y,
 * -x, centre, +x, +y, +z}; 27-point the offsets (dz, dy, dx) in {-1, 0, 1}^3
 * with dz slowest and dx fastest (term 13 is the centre).
 * coef_per_row = 0: coef is a HOST array of npts constant coefficients,
 * copied.  coef_per_row = 1: coef is a DEVICE array of npts * n doubles
 * (n = nx ny nz), coefficient d of row r at coef[d * n + r] (each term's
 * coefficients contiguous over the rows, so a block of rows reads them in
 * one sweep); borrowed: it must outlive the operator and may change between
 * calls; the slots of terms that leave the grid are never read.  A row sums
 * its present terms in the order above, so applying the operator gives bit
 * for bit the product with the equivalent CSR matrix, and every solver, the
 * precision form and the allocation-free entry point accept it.  Jacobi
 * takes 1 / the centre coefficient (ERR_INVALID_ARG for a zero or non-finite
 * one); folded Jacobi on per-row coefficients forms A M^{-1} in npts * n
 * doubles of context workspace, and on constant coefficients needs a constant
 * diagonal.  Not transposable, not batched (ERR_UNSUPPORTED).  ERR_INVALID_ARG
 * for a bad size, npts or coef_per_row; ERR_UNSUPPORTED when n exceeds the
 * launch limit of pbcgs_op_csr or npts * n exceeds 2^31 - 1 per-row
 * coefficients.
 */
int pbcgs_op_stencil(pbcgs_ctx_t ctx, int32_t nx, int32_t ny, int32_t nz, int32_t npts,
                     const double* coef, int32_t coef_per_row, pbcgs_op_t* out);

/*
 * Matrix-free 27-point variable-coefficient convection-diffusion operator
 * (the SPMV building block of Section 2 without a stored matrix): exactly the
 * operator pbcgs_assemble_convdiff(ctx, 3, n, 27, beta, kappa, shift, ...)
 * assembles, applied without storing it.  n^3 interior nodes of the unit
 * cube, h = 1/(n+1), rows x fastest, Dirichlet boundaries.  kappa: DEVICE
 * array of (n+1)^3 cell coefficients, x fastest, borrowed (it must outlive the
 * operator; values may change between calls).  beta: HOST array of 3
 * convection coefficients; hb_a = beta_a / (n+1).  For each of the 26
 * neighbours p + d the coupling is -kbar_d, the mean of the cell coefficients
 * the two nodes share (4, 2 or 1 cells), minus |hb_a| on the upwind face of
 * axis a (p - e_a when beta_a >= 0, else p + e_a); the diagonal is the sum of
 * all 26 kbar_d, plus (|hb_x| + |hb_y|) + |hb_z|, plus shift.  Every entry is
 * formed in the assembly's operation order and each row is summed in
 * ascending column order, so products, solves and Jacobi (dinv = 1 / a_ii
 * from the formed diagonal) equal those on the assembled CSR matrix bit for
 * bit, while a product reads 8 bytes of kappa per row instead of about 270
 * bytes of matrix.  JACOBI_FOLDED scales each entry by dinv_j as it is formed
 * (the same single rounding as the folded CSR values).  Not transposable
 * (ERR_UNSUPPORTED), not batched.  ERR_UNSUPPORTED when n^3 exceeds the launch
 * limit of pbcgs_op_csr.
 */
int pbcgs_op_convdiff27(pbcgs_ctx_t ctx, int32_t n, const double* kappa, const double* beta, double shift,
                        pbcgs_op_t* out);

int pbcgs_op_destroy(pbcgs_op_t op);

/*
 * Transpose of a CSR operator, for the adjoint solve A^T lambda = g that
 * differentiates a loss through A x = b (lambda = A^{-T} dL/dx gives
 * dL/db = lambda and dL/da_ij = -lambda_i x_j).  *out receives a new CSR
 * operator whose arrays the library allocates and frees with it.  Row j of
 * A^T lists column j of A in ascending row order, so its products sum in
 * ascending column order like every other operator; the result does not
 * depend on the order of the device's atomic operations.  ERR_UNSUPPORTED
 * for a stencil.
 */
int pbcgs_op_transpose(pbcgs_ctx_t ctx, pbcgs_op_t A, pbcgs_op_t* out);

/*
 * grad[k] := -lambda[i] * x[j] for every stored entry k = (i, j) of the CSR
 * operator A (device arrays: lambda, x of n doubles, grad of nnz doubles).
 */
int pbcgs_csr_outer_grad(pbcgs_ctx_t ctx, pbcgs_op_t A, const double* lambda, const double* x, double* grad);

/* Number of rows of op (host), or a negative status. */
int64_t pbcgs_op_rows(pbcgs_op_t op);

/* Bytes per stored column index the solves read for op: 2 when a CSR operator
 * holds a compact copy (either form, see pbcgs_op_csr), 4 for int32 columns,
 * 0 for a stencil; ERR_INVALID_ARG for NULL. */
int pbcgs_op_index_bytes(pbcgs_op_t op);

/* Number of diagonals of op's diagonal layout, or 0 when it has none.  A CSR
 * operator with at most 32 distinct diagonals j - i, every row stored with
 * strictly ascending columns, and at most 5/4 as many layout slots (diagonals
 * x rows) as stored entries, also keeps a 32-bit mask per row of the diagonals
 * it holds (4 n bytes, freed with the operator).  Solves then read it through a
 * per-solve copy of the values laid out diagonal by diagonal (diagonals x rows
 * doubles of context workspace, or floats in the precision form): per row the
 * mask and one value per diagonal, no row pointers or column indices.  Each
 * row is still summed over its entries in ascending column order, so results
 * equal those of the CSR arrays bit for bit.  With at most 8 diagonals, each
 * holding at most 16 distinct values in the solve (after folding Jacobi in),
 * no Jacobi vector (none, folded, or a constant diagonal) and at least 2^18
 * rows (PBCGS_VALUE_CODES=1: any row count; =0: never), a solve reads the
 * laid-out values as
 * one-byte codes into per-diagonal tables instead (value indexing: one 8-byte
 * word per row and 128 bytes per diagonal of context workspace; same results;
 * pbcgs_info.value_codes).  pbcgs_spmv and pbcgs_solve_noalloc read the CSR
 * arrays; a batch reads every system's layout (values, not codes) when all
 * its systems have one. */
int pbcgs_op_diagonals(pbcgs_op_t op);

/* Which column form the solves read for op (see pbcgs_op_csr). */
enum { PBCGS_COLS_INT32 = 0, PBCGS_COLS_BLOCK16 = 1, PBCGS_COLS_DIAG16 = 2, PBCGS_COLS_NONE = 3 };
int pbcgs_op_column_form(pbcgs_op_t op);

/* y := A x (device pointers, n doubles each; x and y must not overlap). */
int pbcgs_spmv(pbcgs_ctx_t ctx, pbcgs_op_t A, const double* x, double* y);

/* (x, y) in pairwise order, written to *result (HOST double). */
int pbcgs_dot(pbcgs_ctx_t ctx, int64_t n, const double* x, const double* y, double* result);

/* Jacobi: dinv_i := 1 / a_ii (Section 3.6 with M = diag(A)); ERR_INVALID_ARG if a
 * diagonal entry is zero or missing. */
int pbcgs_jacobi_dinv(pbcgs_ctx_t ctx, pbcgs_op_t A, double* dinv);

/*
 * Solve A x = b.  b: n doubles (device, read only).  x: n doubles (device),
 * holds x_0 on entry and the final iterate on return.  dinv: n doubles
 * (device) of M^{-1} = diag(dinv) when opts->precond is JACOBI or
 * JACOBI_FOLDED, or NULL to derive dinv = 1/diag(A) inside the call; ignored
 * without a preconditioner.  With JACOBI_FOLDED the context forms A M^{-1}
 * (CSR: nnz doubles of context-owned workspace, grown on demand) and x holds
 * y = M x during the call.  relres_true is always ||b - A x|| / ||r_0|| with the
 * caller's A and the returned x.  opts and info are host structs.  The call
 * enqueues on the context's stream and returns after the solve has finished;
 * the host reads the 64-byte device status once every check_every iterations.
 */
int pbcgs_solve(pbcgs_ctx_t ctx, pbcgs_op_t A, const double* b, double* x, const double* dinv,
                const pbcgs_opts* opts, pbcgs_info* info);

/*
 * pbcgs_solve without allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Arguments, results and errors as pbcgs_solve; the
 * solve runs the same kernels and returns the same bits.  Every device buffer
 * the solve needs beyond b, x and dinv -- the state slots, the partial sums of
 * the reductions, the 14 workspace vectors and, for JACOBI_FOLDED on a CSR
 * operator, the values of A M^{-1} -- lies in one statically allocated device
 * array of the library, about 64.3 MiB, of which a pool of 2^23 doubles holds
 * the vectors and folded values: 14 per row (rows rounded up to a multiple of
 * 64) plus one per non-zero when folded must fit in it, else
 * ERR_UNSUPPORTED (e.g. up to 599,186 rows unfolded; a 64^3 7-point CSR
 * system folded).  The call calls no hipMalloc or hipFree: kernels are
 * launched directly (no HIP graph is instantiated), and it refuses the
 * precision form and kernel timing (opts.flags bit 1) with ERR_UNSUPPORTED.
 * Each device that loads the library holds one copy of the array until the
 * process ends; every call on that device shares it and leaves the last
 * call's contents there (each solve initialises what it reads), so calls that
 * overlap on one device -- from two contexts or two threads -- race.
 */
int pbcgs_solve_noalloc(pbcgs_ctx_t ctx, pbcgs_op_t A, const double* b, double* x, const double* dinv,
                        const pbcgs_opts* opts, pbcgs_info* info);

/*
 * Batched solve of nsys independent systems A[k] x[k] = b[k] with the same
 * options (the batched workload of many small and large systems).  A: HOST
 * array of nsys CSR operators of ctx; b, x: HOST arrays of nsys DEVICE
 * pointers (x[k] holds x_0 on entry, the final iterate on return); infos:
 * HOST array of nsys reports.  Every kernel launch covers all systems: each
 * workgroup belongs to one system, each system has its own scalars, status,
 * reductions and stopping test, and a system that stops leaves the later
 * launches at once.  Reductions are the same pairwise trees as in
 * pbcgs_solve, so each system's result equals that of its own pbcgs_solve
 * bit for bit.  BiCGStab and p-BiCGStab (with or without replacement) only,
 * no preconditioner, binary64, no history (ERR_UNSUPPORTED otherwise).  The
 * batch reads the compact int16 columns when every operator holds them (see
 * pbcgs_op_csr) and opts.flags bit 3 is clear, else every system's int32
 * columns.  The context keeps the batch workspace (8 vectors per system).
 * Returns the largest numerical status of the systems, or a negative error.
 */
int pbcgs_solve_batched(pbcgs_ctx_t ctx, int32_t nsys, const pbcgs_op_t* A, const double* const* b,
                        double* const* x, const pbcgs_opts* opts, pbcgs_info* infos);

/* Report of an autotuning run: candidates tried, their cost per iteration
 * and the one kept. */
typedef struct {
    int32_t best;              /* the chosen value (R, or the workgroup cap)          */
    int32_t ncand;             /* candidates tried (at most 12)                       */
    int32_t cand[12];
    double ms_per_iter[12];    /* measured wall time per iteration of each candidate  */
    double best_ms_per_iter;
} pbcgs_tune_report;

/*
 * Autotuner of the launch shape, measured on the device: runs `iters`
 * iterations (tol 0) of the solve described by opts (b: DEVICE right-hand
 * side; x is a scratch vector of its own; of opts->flags only the alpha form
 * and the read-path bits are kept: graph replay, no kernel timing) for
 * every rows-per-wave block count R whose grid fits -- once to capture the
 * graphs, then three times, the fastest counting -- and keeps the fastest R
 * on the operator for the variant, precision and read path of opts (each
 * variant's kernels have their own best shape) and in the launch-shape cache
 * below; later pbcgs_solve calls on A, or on another operator of the same
 * cache key, with that variant, precision and read path use it (the environment variables PBCGS_R
 * and PBCGS_GTARGET still take precedence).  An unknown variant or precision is PBCGS_ERR_INVALID_ARG.
 * The shape never changes a result: every reduction is the same pairwise
 * tree whatever R is.
 */
int pbcgs_tune(pbcgs_ctx_t ctx, pbcgs_op_t A, const double* b, const pbcgs_opts* opts, int32_t iters,
               pbcgs_tune_report* rep);

/*
 * The same for batched solves: tries per-system workgroup caps 8 .. 512 (a
 * system of n rows gets the smallest R with at most that many workgroups)
 * and keeps the fastest on the context for later pbcgs_solve_batched calls
 * (PBCGS_BATCH_GCAP takes precedence).  Arguments as pbcgs_solve_batched,
 * without x (scratch of its own).  iters = 0 times complete solves at
 * opts->tol and opts->maxit instead of `iters` iterations at tol 0 (then
 * ms_per_iter holds the time of one whole batched solve): systems stop at
 * different iterations, so the cap that is best for the whole solve can
 * differ from the one that is best while every system still runs.
 */
int pbcgs_tune_batched(pbcgs_ctx_t ctx, int32_t nsys, const pbcgs_op_t* A, const double* const* b,
                       const pbcgs_opts* opts, int32_t iters, pbcgs_tune_report* rep);

/*
 * Process-wide launch-shape cache.  Every shape pbcgs_tune keeps is also
 * recorded here under a key: the device (its architecture name and compute
 * unit count), the library build that measured it, the operator's rows,
 * stored non-zeros (CSR; 0 for matrix-free operators) and kind, the variant,
 * the precision and the read path.  A pbcgs_solve on an operator that has no
 * tuned shape of its own for these takes the cached shape of its key, so
 * a new operator of the same size and kind (values changed, say) is not tuned
 * again; PBCGS_R and PBCGS_GTARGET still take precedence.  The shape never
 * changes a result.  Entries can be read out and put back (to keep them in a
 * file between processes: the Python layer's save_tune_cache and
 * load_tune_cache do that as JSON).  The cache is shared by every context of
 * the process and guarded by a mutex; it holds single-system shapes only
 * (pbcgs_tune_batched keeps its cap on the context).
 */
typedef struct {
    char device[64];     /* "<architecture> <compute units>cu", NUL-terminated        */
    char build[32];      /* the library build that measured it, NUL-terminated       */
    int64_t nnz;         /* stored non-zeros of a CSR operator, 0 for matrix-free     */
    int32_t n;           /* rows                                                     */
    int32_t op_kind;     /* 0 CSR, 1 5-point stencil, 2 7-point stencil,
                            3 27-point matrix-free (pbcgs_op_convdiff27),
                            4 27-point stencil, 5 stencil with per-row
                            coefficients (pbcgs_op_stencil)                          */
    int32_t variant;     /* PBCGS_BICGSTAB .. PBCGS_PIPE_CG                          */
    int32_t precision;   /* PBCGS_FP64 or PBCGS_FP32_RR64                            */
    int32_t read_path;   /* 0 the operator's default (its diagonal layout or compact
                            columns where it has them), 1 the CSR arrays
                            (opts.flags bit 4), 2 the int32 columns (bit 3)          */
    int32_t best;        /* the shape: 64-row blocks per wave, a power of two whose
                            grid of ceil(n / (256 best)) workgroups is at most 1024 */
} pbcgs_tune_entry;

/* Number of cache entries. */
int32_t pbcgs_tune_cache_size(void);
/* Copy entry i (0 <= i < size) to *out (host struct); ERR_INVALID_ARG otherwise. */
int pbcgs_tune_cache_get(int32_t i, pbcgs_tune_entry* out);
/* Add an entry, or replace the shape of the entry with the same key.  A key
 * field out of range, an unterminated string or a shape that does not fit n
 * is ERR_INVALID_ARG (the cache is then unchanged). */
int pbcgs_tune_cache_put(const pbcgs_tune_entry* e);
/* Remove every entry. */
int pbcgs_tune_cache_clear(void);
/* Fill *out with the key of (ctx's device, this build, A, variant, precision,
 * the read path that opts.flags `flags` select) and out->best with the cached
 * shape of that key, or 0 when there is none. */
int pbcgs_tune_cache_key(pbcgs_ctx_t ctx, pbcgs_op_t A, int32_t variant, int32_t precision, int32_t flags,
                         pbcgs_tune_entry* out);

/*
 * Test hook for the residual replacement of Section 4.2.  After iteration
 * `iter` of later binary64 PBCGS_PBICGSTAB and PBCGS_PBICGSTAB_RR solves on
 * ctx -- once that iteration's reductions are taken, before the next one
 * starts -- every entry of the recursive residual r_{iter+1} is multiplied by
 * `scale` (one rounding each; r^ is left alone).  The recursive residual then
 * departs from b - A x, as accumulated rounding makes it do, and the next
 * replacement must bring the two together again.  iter = -1 switches the hook
 * off (the default); scale must be finite.  While the hook is on, solves launch
 * their kernels directly (no HIP graph), and pbcgs_solve of another variant
 * or of the precision form, and pbcgs_solve_batched, return ERR_UNSUPPORTED.
 * The setting stays on the context until changed.
 */
int pbcgs_debug_perturb(pbcgs_ctx_t ctx, int32_t iter, double scale);

/*
 * Workload builder (not part of the method): assembles on the device the
 * h^2-scaled first-order upwind convection-diffusion operator used by the
 * tests and the benchmark, h = 1/(n+1), Dirichlet boundaries, rows x fastest,
 * ascending columns.  dim 2 / npts 5, or dim 3 / npts 7 or 27.  beta: HOST
 * array of dim doubles.  kappa: DEVICE array of (n+1)^3 cell coefficients for
 * npts 27 (NULL otherwise).  shift is added to the 27-point diagonal.  The
 * caller allocates row_ptr[n^dim + 1], col_idx[nnz], val[nnz] with nnz from
 * pbcgs_convdiff_nnz().
 */
int64_t pbcgs_convdiff_nnz(int32_t dim, int32_t n, int32_t npts);
int pbcgs_assemble_convdiff(pbcgs_ctx_t ctx, int32_t dim, int32_t n, int32_t npts,
                            const double* beta, const double* kappa, double shift,
                            int32_t* row_ptr, int32_t* col_idx, double* val);

#ifdef __cplusplus
}
#endif
#endif /* PBCGS_H */
