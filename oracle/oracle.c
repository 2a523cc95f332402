/*
 * CPU oracle for the pipelined BiCGStab solvers -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct FP64 reference used by the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark.  It shares no code
 * with the HIP library and the product path never loads it.
 *
 * Source: S. Cools, W. Vanroose, "The communication-hiding pipelined BiCGStab
 * method for the parallel solution of large unsymmetric linear systems"
 * (arXiv 1612.01395).  The paper numbers its listings in order of
 * appearance; the solvers below follow them step by step, in the paper's
 * order and notation:
 *
 *   Algorithm 2   standard preconditioned CG             (Section 2)
 *   Algorithm 4   Chronopoulos & Gear CG                 (Section 2)
 *   Algorithm 6   pipelined CG                           (Section 2)
 *   Algorithm 7   standard BiCGStab                     (Section 3.1)
 *   Algorithm 8   communication-avoiding BiCGStab        (Section 3.1)
 *   Algorithm 9   pipelined BiCGStab, unpreconditioned   (Section 3.3)
 *   Algorithm 10  right-preconditioned BiCGStab          (Section 3.6)
 *   Algorithm 11  preconditioned pipelined BiCGStab      (Section 3.6)
 *
 * or_solve_mp is the precision form of Algorithm 9 with residual replacement:
 * binary32 vectors, SpMV, recurrences and dot products, binary64 replacement
 * steps, x update and scalars, and a binary64 true-residual check before any
 * SUCCESS.  Its rounding sequence is pinned operation by operation by an
 * exact-rational twin that rounds each exact result to binary32 or binary64
 * as IEEE 754 defines it (exact.py, ieee.py), besides special cases and
 * accuracy facts (exact binary32 cases, tracking of the binary64 iterates,
 * the stall without replacement, the confirmed convergence).
 *
 * Residual replacement follows Section 4.2: every k iterations r, r^, w and
 * s, s^, z are recomputed from their definitions (4 SpMVs + 2 preconditioner
 * applications).  Stopping test: ||r_i||_2 / ||r_0||_2 <= tol on the
 * recursive residual (Section 4.1).
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *  - shadow residual r~ = r_0; quantities with index -1 are zero, omega_{-1}=0;
 *  - alpha_{i+1} uses the four-dot expression (eq. 3) by default; eq. (5),
 *    the three-dot form, on request (or_set_alpha_form);
 *  - a test hook (or_set_perturb) scales the recursive residual of the
 *    pipelined solvers after one iteration, so that tests can watch the next
 *    replacement close the gap to b - A x;
 *  - residual replacement in iteration i with (i+1) mod k == 0: r, r^, w are
 *    replaced after the x-update of iteration i (so the second reduction,
 *    beta_i, alpha_{i+1}, w^ and t all see the true values) and s, s^, z
 *    are replaced at the start of iteration i+1, right after the p^ update;
 *  - breakdown: (y,y) = 0 means q = 0, i.e. exact convergence: x += alpha p^;
 *    a zero denominator elsewhere, or omega = 0, stops with BREAKDOWN;
 *  - floating point: every + and * is one binary64 operation in the written
 *    order (built with -ffp-contract=off, so no fused multiply-add);
 *    the SpMV sums each row in stored (ascending column) order starting from
 *    0.0; a dot product (x,y) is the sum of the rounded products x_i*y_i in
 *    pairwise order -- the balanced binary tree over the index range padded
 *    with zeros to a power of two -- followed by "+ 0.0" so that a zero sum
 *    is always +0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_SUCCESS 0
#define OR_MAXIT 1
#define OR_BREAKDOWN 2
#define OR_NONFINITE 3
#define OR_ERR_INVALID_ARG (-1)
#define OR_ERR_ALLOC (-2)

#define PAR _Pragma("omp parallel for schedule(static)")

/* ------------------------------------------------------------------------ */
/* counters used to check the per-iteration cost model of Table 1            */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t spmv;   /* sparse matrix-vector products                        */
    int64_t pc;     /* preconditioner applications M^{-1} v                 */
    int64_t glred;  /* global reduction phases (groups of dot products)     */
    int64_t dots;   /* dot products counted by the paper (no norm of r)     */
    int64_t flops;  /* AXPY + dot flops per vector element (the "x N")      */
    int64_t rec;    /* recurrence (AXPY) lines executed                      */
} or_counters;

static or_counters g_ctr;

/* alpha_{i+1} of the pipelined solvers: 3 = eq. (3), four dot products (the
 * default, as in Algorithms 9 and 11); 5 = eq. (5), the three-dot form that
 * is equal in exact arithmetic. */
static int g_alpha_form = 3;
void or_set_alpha_form(int32_t form) { g_alpha_form = (form == 5) ? 5 : 3; }

/* Test hook for the residual replacement of Section 4.2.  At the end of
 * iteration g_perturb_iter of the pipelined BiCGStab solvers (Algorithms 9
 * and 11), after that iteration's reductions and scalars, every entry of the
 * recursive residual r_{i+1} is multiplied by g_perturb_scale (the
 * preconditioned copy r^ is left alone).  This opens a gap between r and
 * b - A x, as accumulated rounding does, which the next replacement must
 * close.  -1 = off. */
static int32_t g_perturb_iter = -1;
static double g_perturb_scale = 1.0;
void or_set_perturb(int32_t iter, double scale) { g_perturb_iter = iter; g_perturb_scale = scale; }

void or_counters_get(int64_t* out6)
{
    out6[0] = g_ctr.spmv; out6[1] = g_ctr.pc; out6[2] = g_ctr.glred;
    out6[3] = g_ctr.dots; out6[4] = g_ctr.flops; out6[5] = g_ctr.rec;
}

void or_counters_reset(void) { memset(&g_ctr, 0, sizeof g_ctr); }

/* ------------------------------------------------------------------------ */
/* matrix assembly (the workload definition, not part of the method)         */
/* ------------------------------------------------------------------------ */

/* Number of stored entries of the convection-diffusion operator. */
int64_t or_assemble_nnz(int32_t dim, int32_t n, int32_t npts)
{
    int64_t m = n;
    if (n <= 0) return -1;
    if (dim == 2 && npts == 5) return 5 * m * m - 4 * m;
    if (dim == 3 && npts == 7) return 7 * m * m * m - 6 * m * m;
    if (dim == 3 && npts == 27) return (3 * m - 2) * (3 * m - 2) * (3 * m - 2);
    return -1;
}

/*
 * h^2-scaled upwind convection-diffusion operator on the n^dim interior
 * nodes of the unit square/cube, homogeneous Dirichlet boundaries (couplings
 * to boundary nodes are not stored), rows ordered x fastest, columns
 * ascending within a row.
 *
 *   hb_a = beta_a / (n + 1)
 *   5/7-point:  off-diagonal -1, plus -|hb_a| on the upwind neighbour of axis
 *               a (p - e_a if beta_a >= 0, else p + e_a);
 *               diagonal (4 + |hbx|) + |hby|   or   ((6 + |hbx|) + |hby|) + |hbz|
 *   27-point:   kbar_d = mean of the cell coefficients kappa shared by node p
 *               and its neighbour p + d (4, 2 or 1 cells), summed c, b, a
 *               lexicographically then scaled by 1/count; coupling -kbar_d,
 *               plus -|hb_a| on the upwind face of axis a; diagonal
 *               (sum_d kbar_d over all 26 d + ((|hbx| + |hby|) + |hbz|)) + shift.
 *
 * or_assemble_rows emits only rows [row_begin, row_end) (row pointers relative
 * to row_begin) and returns their entry count; -1 for unsupported arguments.
 */
int64_t or_assemble_rows(int32_t dim, int32_t n, int32_t npts, const double* beta,
                         const double* kappa, double shift, int64_t row_begin, int64_t row_end,
                         int32_t* row_ptr, int32_t* col, double* val)
{
    int64_t nnz_expected = or_assemble_nnz(dim, n, npts);
    if (nnz_expected < 0 || beta == NULL) return -1;
    if (npts == 27 && kappa == NULL) return -1;
    const int nz = (dim == 3) ? n : 1;
    const int64_t nn = (int64_t)n * n;
    double hb[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < dim; ++a) hb[a] = beta[a] / (double)(n + 1);
    const int64_t cn = n + 1; /* cells per axis */

    int64_t pos = 0;
    row_ptr[0] = 0;
    for (int k = 0; k < nz; ++k)
    for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
        const int64_t row = i + (int64_t)n * j + nn * k;
        if (row < row_begin || row >= row_end) continue;
        if (npts == 5 || npts == 7) {
            /* entries in ascending column order: (-z), -y, -x, diagonal, +x, +y, (+z);
             * entry e is axis ax[e] on side sd[e] (sd 0 marks the diagonal) */
            static const int ax3[7] = {2, 1, 0, 0, 0, 1, 2}, sd3[7] = {-1, -1, -1, 0, 1, 1, 1};
            static const int ax2[5] = {1, 0, 0, 0, 1}, sd2[5] = {-1, -1, 0, 1, 1};
            const int* ax = (dim == 3) ? ax3 : ax2;
            const int* sd = (dim == 3) ? sd3 : sd2;
            for (int e = 0; e < npts; ++e) {
                if (sd[e] == 0) {
                    double d;
                    if (dim == 2) d = (4.0 + fabs(hb[0])) + fabs(hb[1]);
                    else d = ((6.0 + fabs(hb[0])) + fabs(hb[1])) + fabs(hb[2]);
                    col[pos] = (int32_t)row;
                    val[pos] = d;
                    ++pos;
                    continue;
                }
                const int a = ax[e], side = sd[e];
                int ci = i, cj = j, ck = k;
                if (a == 0) ci += side;
                if (a == 1) cj += side;
                if (a == 2) ck += side;
                if (ci < 0 || ci >= n || cj < 0 || cj >= n || ck < 0 || ck >= nz) continue;
                /* upwind neighbour: p - e_a for beta_a >= 0, p + e_a otherwise */
                int upwind = (beta[a] >= 0.0) ? (side < 0) : (side > 0);
                col[pos] = (int32_t)(ci + (int64_t)n * cj + nn * ck);
                val[pos] = upwind ? (-1.0 - fabs(hb[a])) : -1.0;
                ++pos;
            }
        } else {
            /* 27-point: offsets in (dz, dy, dx) lexicographic order */
            double diag_sum = 0.0;
            int64_t diag_pos = -1;
            for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (dx == 0 && dy == 0 && dz == 0) {
                    diag_pos = pos;
                    col[pos] = (int32_t)row;
                    val[pos] = 0.0; /* filled in below */
                    ++pos;
                    continue;
                }
                /* cells shared by node p and p + d */
                int alo = (dx > 0) ? 1 : 0, ahi = (dx < 0) ? 0 : 1;
                int blo = (dy > 0) ? 1 : 0, bhi = (dy < 0) ? 0 : 1;
                int clo = (dz > 0) ? 1 : 0, chi = (dz < 0) ? 0 : 1;
                double ksum = 0.0;
                int count = 0;
                for (int c = clo; c <= chi; ++c)
                for (int b = blo; b <= bhi; ++b)
                for (int a = alo; a <= ahi; ++a) {
                    ksum = ksum + kappa[(i + a) + cn * ((j + b) + cn * (k + c))];
                    ++count;
                }
                double kbar = ksum * (1.0 / (double)count);
                diag_sum = diag_sum + kbar;
                int ci = i + dx, cj = j + dy, ck = k + dz;
                if (ci < 0 || ci >= n || cj < 0 || cj >= n || ck < 0 || ck >= n) continue;
                double v = -kbar;
                int nzc = (dx != 0) + (dy != 0) + (dz != 0);
                if (nzc == 1) {
                    int a = (dx != 0) ? 0 : ((dy != 0) ? 1 : 2);
                    int side = (dx != 0) ? dx : ((dy != 0) ? dy : dz);
                    int upwind = (beta[a] >= 0.0) ? (side < 0) : (side > 0);
                    if (upwind) v = -kbar - fabs(hb[a]);
                }
                col[pos] = (int32_t)(ci + (int64_t)n * cj + nn * ck);
                val[pos] = v;
                ++pos;
            }
            val[diag_pos] = (diag_sum + ((fabs(hb[0]) + fabs(hb[1])) + fabs(hb[2]))) + shift;
        }
        row_ptr[row - row_begin + 1] = (int32_t)pos;
    }
    return pos;
}

/* The whole operator: rows [0, n^dim). */
int64_t or_assemble(int32_t dim, int32_t n, int32_t npts, const double* beta,
                    const double* kappa, double shift,
                    int32_t* row_ptr, int32_t* col, double* val)
{
    const int64_t N = (dim == 3) ? (int64_t)n * n * n : (int64_t)n * n;
    int64_t nnz = or_assemble_rows(dim, n, npts, beta, kappa, shift, 0, N, row_ptr, col, val);
    return (nnz == or_assemble_nnz(dim, n, npts)) ? nnz : -1;
}

/* ------------------------------------------------------------------------ */
/* kernels of the method: SpMV, dot product, Jacobi                          */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t n;
    const int32_t* rp;
    const int32_t* ci;
    const double* va;
} csr_t;

/* Product with A: each row summed in stored order from 0.0 (Section 2, the SPMV kernel). */
static void spmv(const csr_t* A, const double* x, double* y)
{
    PAR for (int32_t i = 0; i < A->n; ++i) {
        double acc = 0.0;
        for (int32_t k = A->rp[i]; k < A->rp[i + 1]; ++k) acc = acc + A->va[k] * x[A->ci[k]];
        y[i] = acc;
    }
    g_ctr.spmv++;
}

void or_spmv(int32_t n, const int32_t* rp, const int32_t* ci, const double* va,
             const double* x, double* y)
{
    csr_t A = {n, rp, ci, va};
    spmv(&A, x, y);
}

/* Sum of a[0 .. len), len a power of two: left half + right half. */
static double pairwise(const double* a, int64_t len)
{
    if (len == 1) return a[0];
    return pairwise(a, len / 2) + pairwise(a + len / 2, len / 2);
}

/* The same tree with the 64 top subtrees evaluated by separate threads. */
static double pairwise_par(const double* a, int64_t len)
{
    if (len < (1 << 16)) return pairwise(a, len);
    double part[64];
    const int64_t bl = len / 64;
    PAR for (int b = 0; b < 64; ++b) part[b] = pairwise(a + b * bl, bl);
    return pairwise(part, 64);
}

static int64_t pow2_at_least(int64_t n)
{
    int64_t p = 1;
    while (p < n) p <<= 1;
    return p;
}

/* (x, y) = sum_i x_i y_i in pairwise order; prod is scratch of pow2(n). */
static double dot_ws(int64_t n, const double* x, const double* y, double* prod)
{
    const int64_t len = pow2_at_least(n);
    PAR for (int64_t i = 0; i < len; ++i) prod[i] = (i < n) ? x[i] * y[i] : 0.0;
    return pairwise_par(prod, len) + 0.0;
}

double or_dot(int64_t n, const double* x, const double* y)
{
    if (n <= 0) return 0.0;
    double* prod = (double*)malloc(sizeof(double) * (size_t)pow2_at_least(n));
    if (!prod) return NAN;
    double s = dot_ws(n, x, y, prod);
    free(prod);
    return s;
}

/* The pairwise sum of a plain array (used to check the tree order). */
double or_pairwise_sum(int64_t n, const double* a)
{
    if (n <= 0) return 0.0;
    const int64_t len = pow2_at_least(n);
    double* buf = (double*)calloc((size_t)len, sizeof(double));
    if (!buf) return NAN;
    memcpy(buf, a, sizeof(double) * (size_t)n);
    double s = pairwise_par(buf, len) + 0.0;
    free(buf);
    return s;
}

/* Jacobi: M = diag(A), dinv_i = 1 / a_ii.  Error if a diagonal is absent or 0. */
int or_jacobi_dinv(int32_t n, const int32_t* rp, const int32_t* ci, const double* va, double* dinv)
{
    for (int32_t i = 0; i < n; ++i) {
        double d = 0.0;
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
            if (ci[k] == i) d = va[k];
        if (d == 0.0 || !isfinite(d)) return OR_ERR_INVALID_ARG;
        dinv[i] = 1.0 / d;
    }
    return OR_SUCCESS;
}

/* ------------------------------------------------------------------------ */
/* solver bookkeeping                                                        */
/* ------------------------------------------------------------------------ */
typedef struct {
    double tol;
    int32_t maxit;
    int32_t rr_period;  /* k; 0 disables residual replacement */
    int32_t rr_max;     /* -1: unlimited */
    double* history;    /* NULL or maxit+1 entries: ||r_i|| / ||r_0|| */
    double* scalars;    /* NULL or 3*maxit entries: alpha_i, omega_i, beta_i */
} or_opts;

typedef struct {
    int32_t iters, n_rr, status;
    double relres_rec;
    double relres_true;
} or_info;

#define DOT(a, b) dot_ws(n, (a), (b), prod)
#define NEWVEC(p) do { (p) = (double*)calloc((size_t)n, sizeof(double)); if (!(p)) goto oom; } while (0)
#define FLOPS(k) (g_ctr.flops += (k))
#define REC(k) (g_ctr.rec += (k))

static int rr_due(const or_opts* o, int32_t i, int32_t n_rr)
{
    if (o->rr_period <= 0) return 0;
    if ((i + 1) % o->rr_period != 0) return 0;
    return (o->rr_max < 0) || (n_rr < o->rr_max);
}

static void finish(const csr_t* A, const double* b, const double* x, double rho0,
                   double* tmp, double* prod, or_info* info)
{
    const int32_t n = A->n;
    spmv(A, x, tmp);
    g_ctr.spmv--; /* the final true residual is bookkeeping, not an iteration cost */
    PAR for (int32_t j = 0; j < n; ++j) tmp[j] = b[j] - tmp[j];
    double nr = dot_ws(n, tmp, tmp, prod);
    info->relres_true = (rho0 > 0.0) ? sqrt(nr) / rho0 : 0.0;
}

/* ------------------------------------------------------------------------ */
/* Alg. 7 (standard BiCGStab) and Alg. 10 (its right-preconditioned form,    */
/* A M^{-1} y = b, M x = y).  dinv == NULL selects Alg. 7.                   */
/* ------------------------------------------------------------------------ */
static int bicgstab(const csr_t* A, const double* dinv, const double* b, double* x,
                    const or_opts* o, or_info* info)
{
    const int32_t n = A->n;
    const int pc = (dinv != NULL);
    double *r0 = 0, *r = 0, *p = 0, *ph = 0, *s = 0, *q = 0, *qh = 0, *y = 0, *tmp = 0, *prod = 0;
    NEWVEC(r0); NEWVEC(r); NEWVEC(p); NEWVEC(s); NEWVEC(q); NEWVEC(y); NEWVEC(tmp);
    if (pc) { NEWVEC(ph); NEWVEC(qh); } else { ph = p; qh = q; }
    prod = (double*)malloc(sizeof(double) * (size_t)pow2_at_least(n));
    if (!prod) goto oom;

    info->iters = 0; info->n_rr = 0; info->relres_rec = 0.0; info->relres_true = 0.0;
    /* initial residual; the first search direction is that residual */
    spmv(A, x, tmp);
    PAR for (int32_t j = 0; j < n; ++j) r0[j] = b[j] - tmp[j];
    double gamma = DOT(r0, r0); /* (r_0, r_0) = (r_0, r_i) at i = 0 */
    const double rho0 = sqrt(gamma);
    if (o->history) o->history[0] = 1.0;
    info->relres_rec = 1.0;
    if (!isfinite(rho0)) { info->status = OR_NONFINITE; goto done; }
    if (rho0 == 0.0) { info->status = OR_SUCCESS; info->relres_rec = 0.0; goto done; }
    memcpy(r, r0, sizeof(double) * (size_t)n);
    memcpy(p, r0, sizeof(double) * (size_t)n);

    for (int32_t i = 0; i < o->maxit; ++i) {
        /* preconditioned search direction (Algorithm 10 only), then its product with A */
        if (pc) { PAR for (int32_t j = 0; j < n; ++j) ph[j] = dinv[j] * p[j]; g_ctr.pc++; }
        spmv(A, ph, s);
        /* first reduction: the shadow inner product of that product gives the step length alpha */
        double delta = DOT(r0, s);
        g_ctr.glred++; g_ctr.dots++; FLOPS(2);
        if (!isfinite(delta)) { info->status = OR_NONFINITE; goto done; }
        if (delta == 0.0) { info->status = OR_BREAKDOWN; goto done; }
        double alpha = gamma / delta;
        if (!isfinite(alpha)) { info->status = OR_NONFINITE; goto done; }
        /* intermediate residual after the alpha step, preconditioned (Algorithm 10), and its product with A */
        PAR for (int32_t j = 0; j < n; ++j) q[j] = r[j] - alpha * s[j];
        FLOPS(2); REC(1);
        if (pc) { PAR for (int32_t j = 0; j < n; ++j) qh[j] = dinv[j] * q[j]; g_ctr.pc++; }
        spmv(A, qh, y);
        /* second reduction: the two inner products whose quotient is the stabilising step omega */
        double th1 = DOT(q, y), th2 = DOT(y, y);
        g_ctr.glred++; g_ctr.dots += 2; FLOPS(4);
        if (!isfinite(th1) || !isfinite(th2)) { info->status = OR_NONFINITE; goto done; }
        if (th2 == 0.0) {
            /* y_i = A q^_i = 0 means q_i = 0: x_i + alpha_i p^_i solves the system */
            PAR for (int32_t j = 0; j < n; ++j) x[j] = x[j] + alpha * ph[j];
            info->iters = i + 1; info->relres_rec = 0.0; info->status = OR_SUCCESS;
            if (o->history) o->history[i + 1] = 0.0;
            goto done;
        }
        double omega = th1 / th2;
        if (!isfinite(omega)) { info->status = OR_NONFINITE; goto done; }
        /* new iterate from both steps, and the new residual from the intermediate one */
        PAR for (int32_t j = 0; j < n; ++j) x[j] = x[j] + alpha * ph[j] + omega * qh[j];
        PAR for (int32_t j = 0; j < n; ++j) r[j] = q[j] - omega * y[j];
        FLOPS(4 + 2); REC(2);
        info->iters = i + 1;
        /* reduction (r_0, r_{i+1}) together with the norm for the stopping test */
        double gamma1 = DOT(r0, r), nu = DOT(r, r);
        g_ctr.glred++; g_ctr.dots++; FLOPS(2);
        if (o->scalars) { o->scalars[3 * i] = alpha; o->scalars[3 * i + 1] = omega; }
        if (!isfinite(gamma1) || !isfinite(nu)) { info->status = OR_NONFINITE; goto done; }
        info->relres_rec = sqrt(nu) / rho0;
        if (o->history) o->history[i + 1] = info->relres_rec;
        if (info->relres_rec <= o->tol) { info->status = OR_SUCCESS; goto done; }
        if (omega == 0.0 || gamma == 0.0) { info->status = OR_BREAKDOWN; goto done; }
        /* direction update coefficient beta from the ratio of consecutive shadow inner products */
        double beta = (alpha / omega) * (gamma1 / gamma);
        if (!isfinite(beta)) { info->status = OR_NONFINITE; goto done; }
        if (o->scalars) o->scalars[3 * i + 2] = beta;
        /* next search direction: new residual plus beta times the omega-corrected old direction */
        PAR for (int32_t j = 0; j < n; ++j) p[j] = r[j] + beta * (p[j] - omega * s[j]);
        FLOPS(4); REC(1);
        gamma = gamma1;
    }
    info->status = OR_MAXIT;
done:
    finish(A, b, x, rho0, tmp, prod, info);
    free(r0); free(r); free(p); free(s); free(q); free(y); free(tmp); free(prod);
    if (pc) { free(ph); free(qh); }
    return info->status;
oom:
    free(r0); free(r); free(p); free(s); free(q); free(y); free(tmp); free(prod);
    if (pc) { free(ph); free(qh); }
    return OR_ERR_ALLOC;
}

/* ------------------------------------------------------------------------ */
/* Alg. 9 (p-BiCGStab) and Alg. 11 (preconditioned p-BiCGStab), with the    */
/* residual replacement of Section 4.2.  dinv == NULL selects Alg. 9, where  */
/* every hatted vector is the unhatted one.                                  */
/* ------------------------------------------------------------------------ */
static int pbicgstab(const csr_t* A, const double* dinv, const double* b, double* x,
                     const or_opts* o, or_info* info)
{
    const int32_t n = A->n;
    const int pc = (dinv != NULL);
    double *r0 = 0, *r = 0, *rh = 0, *w = 0, *wh = 0, *t = 0, *ph = 0, *s = 0, *sh = 0;
    double *z = 0, *zh = 0, *v = 0, *q = 0, *qh = 0, *y = 0, *tmp = 0, *prod = 0;
    NEWVEC(r0); NEWVEC(r); NEWVEC(w); NEWVEC(t); NEWVEC(ph); NEWVEC(s); NEWVEC(z);
    NEWVEC(v); NEWVEC(q); NEWVEC(y); NEWVEC(tmp);
    if (pc) { NEWVEC(rh); NEWVEC(wh); NEWVEC(sh); NEWVEC(zh); NEWVEC(qh); }
    else { rh = r; wh = w; sh = s; zh = z; qh = q; }
    prod = (double*)malloc(sizeof(double) * (size_t)pow2_at_least(n));
    if (!prod) goto oom;

    info->iters = 0; info->n_rr = 0; info->relres_rec = 1.0; info->relres_true = 0.0;
    /* initial residual, its preconditioned copy, the product of that copy with A, and its preconditioned copy */
    spmv(A, x, tmp);
    PAR for (int32_t j = 0; j < n; ++j) r0[j] = b[j] - tmp[j];
    double gamma = DOT(r0, r0); /* (r_0, r_0) */
    const double rho0 = sqrt(gamma);
    if (o->history) o->history[0] = 1.0;
    if (!isfinite(rho0)) { info->status = OR_NONFINITE; goto done; }
    if (rho0 == 0.0) { info->status = OR_SUCCESS; info->relres_rec = 0.0; goto done; }
    memcpy(r, r0, sizeof(double) * (size_t)n);
    if (pc) { PAR for (int32_t j = 0; j < n; ++j) rh[j] = dinv[j] * r[j]; g_ctr.pc++; }
    spmv(A, rh, w);
    if (pc) { PAR for (int32_t j = 0; j < n; ++j) wh[j] = dinv[j] * w[j]; g_ctr.pc++; }
    /* auxiliary product for the first iteration; first step length from the setup's inner products; beta starts at 0 */
    spmv(A, wh, t);
    double delta = DOT(r0, w);
    if (!isfinite(delta)) { info->status = OR_NONFINITE; goto done; }
    if (delta == 0.0) { info->status = OR_BREAKDOWN; goto done; }
    double alpha = gamma / delta, beta = 0.0, omega = 0.0;
    if (!isfinite(alpha)) { info->status = OR_NONFINITE; goto done; }
    /* p^_{-1} = s_{-1} = s^_{-1} = z_{-1} = z^_{-1} = v_{-1} = 0 (calloc) */
    int rr_pending = 0;
    int32_t n_rr = 0;

    for (int32_t i = 0; i < o->maxit; ++i) {
        /* Algorithm 11: search direction from the (preconditioned) residual and the previous direction */
        PAR for (int32_t j = 0; j < n; ++j) ph[j] = rh[j] + beta * (ph[j] - omega * sh[j]);
        FLOPS(4); REC(1);
        if (rr_pending) {
            /* second half of a replacement (Section 4.2): s, its preconditioned copy and z recomputed from p */
            spmv(A, ph, s);
            if (pc) { PAR for (int32_t j = 0; j < n; ++j) sh[j] = dinv[j] * s[j]; g_ctr.pc++; }
            spmv(A, sh, z);
            rr_pending = 0;
        } else {
            /* recurrence of s, the product of A with the search direction (uses the old z) */
            PAR for (int32_t j = 0; j < n; ++j) s[j] = w[j] + beta * (s[j] - omega * z[j]);
            /* the same recurrence for the preconditioned copy of s (Algorithm 11) */
            if (pc) PAR for (int32_t j = 0; j < n; ++j) sh[j] = wh[j] + beta * (sh[j] - omega * zh[j]);
            /* recurrence of z, the product of A with the preconditioned s (uses the old v) */
            PAR for (int32_t j = 0; j < n; ++j) z[j] = t[j] + beta * (z[j] - omega * v[j]);
            FLOPS(pc ? 12 : 8); REC(pc ? 3 : 2);
        }
        /* intermediate residual q, its preconditioned copy, and y = A times that copy, all by recurrence */
        PAR for (int32_t j = 0; j < n; ++j) q[j] = r[j] - alpha * s[j];
        if (pc) PAR for (int32_t j = 0; j < n; ++j) qh[j] = rh[j] - alpha * sh[j];
        PAR for (int32_t j = 0; j < n; ++j) y[j] = w[j] - alpha * z[j];
        FLOPS(pc ? 6 : 4); REC(pc ? 3 : 2);
        /* begin reduction (q_i, y_i), (y_i, y_i) */
        double th1 = DOT(q, y), th2 = DOT(y, y);
        g_ctr.glred++; g_ctr.dots += 2; FLOPS(4);
        /* the product that the first reduction overlaps in the paper: v from the preconditioned z */
        if (pc) { PAR for (int32_t j = 0; j < n; ++j) zh[j] = dinv[j] * z[j]; g_ctr.pc++; }
        spmv(A, zh, v);
        /* first reduction finished: omega */
        if (!isfinite(th1) || !isfinite(th2)) { info->status = OR_NONFINITE; goto done; }
        if (th2 == 0.0) {
            PAR for (int32_t j = 0; j < n; ++j) x[j] = x[j] + alpha * ph[j];
            info->iters = i + 1; info->relres_rec = 0.0; info->status = OR_SUCCESS;
            if (o->history) o->history[i + 1] = 0.0;
            goto done;
        }
        omega = th1 / th2;
        if (!isfinite(omega)) { info->status = OR_NONFINITE; goto done; }
        /* iterate update by both steps */
        PAR for (int32_t j = 0; j < n; ++j) x[j] = x[j] + alpha * ph[j] + omega * qh[j];
        /* residual recurrence */
        PAR for (int32_t j = 0; j < n; ++j) r[j] = q[j] - omega * y[j];
        /* recurrence of the preconditioned residual (Algorithm 11) */
        if (pc) PAR for (int32_t j = 0; j < n; ++j) rh[j] = qh[j] - omega * (wh[j] - alpha * zh[j]);
        /* recurrence of w, the product of A with the preconditioned residual */
        PAR for (int32_t j = 0; j < n; ++j) w[j] = y[j] - omega * (t[j] - alpha * v[j]);
        FLOPS(pc ? 14 : 10); REC(pc ? 4 : 3);
        info->iters = i + 1;
        if (rr_due(o, i, n_rr)) {
            /* first half of a replacement (Section 4.2): true residual, its preconditioned copy, and w from it */
            spmv(A, x, tmp);
            PAR for (int32_t j = 0; j < n; ++j) r[j] = b[j] - tmp[j];
            if (pc) { PAR for (int32_t j = 0; j < n; ++j) rh[j] = dinv[j] * r[j]; g_ctr.pc++; }
            spmv(A, rh, w);
            rr_pending = 1;
            ++n_rr;
            info->n_rr = n_rr;
        }
        /* begin reduction (r_0,r_{i+1}), (r_0,w_{i+1}), (r_0,s_i), (r_0,z_i), plus ||r_{i+1}||^2 */
        double gamma1 = DOT(r0, r), eta = DOT(r0, w), sig_s = DOT(r0, s), sig_z = DOT(r0, z);
        double nu = DOT(r, r);
        g_ctr.glred++; g_ctr.dots += 4; FLOPS(8);
        if (o->scalars) { o->scalars[3 * i] = alpha; o->scalars[3 * i + 1] = omega; }
        if (!isfinite(gamma1) || !isfinite(eta) || !isfinite(sig_s) || !isfinite(sig_z) || !isfinite(nu)) {
            info->status = OR_NONFINITE; goto done;
        }
        info->relres_rec = sqrt(nu) / rho0;
        if (o->history) o->history[i + 1] = info->relres_rec;
        if (info->relres_rec <= o->tol) { info->status = OR_SUCCESS; goto done; }
        /* the product the second reduction overlaps: t from the preconditioned w */
        if (pc) { PAR for (int32_t j = 0; j < n; ++j) wh[j] = dinv[j] * w[j]; g_ctr.pc++; }
        spmv(A, wh, t);
        /* end reduction ; beta_i ; alpha_{i+1} by eq. (3) */
        if (omega == 0.0 || gamma == 0.0) { info->status = OR_BREAKDOWN; goto done; }
        beta = (alpha / omega) * (gamma1 / gamma);
        if (!isfinite(beta)) { info->status = OR_NONFINITE; goto done; }
        if (o->scalars) o->scalars[3 * i + 2] = beta;
        if (g_alpha_form == 5) {
            /* eq. (5): (1/omega + (r0,w)/(r0,r) - (beta omega) ((r0,z)/(r0,r)))^{-1}, three quotients
               summed in the order the equation writes them */
            if (gamma1 == 0.0) { info->status = OR_BREAKDOWN; goto done; }
            double den5 = (1.0 / omega + eta / gamma1) - (beta * omega) * (sig_z / gamma1);
            if (den5 == 0.0) { info->status = OR_BREAKDOWN; goto done; }
            alpha = 1.0 / den5;
        } else {
            double den = eta + beta * sig_s - beta * omega * sig_z;
            if (den == 0.0 || gamma1 == 0.0) { info->status = OR_BREAKDOWN; goto done; }
            alpha = gamma1 / den;
        }
        if (!isfinite(alpha)) { info->status = OR_NONFINITE; goto done; }
        gamma = gamma1;
        if (i == g_perturb_iter) PAR for (int32_t j = 0; j < n; ++j) r[j] = g_perturb_scale * r[j];
    }
    info->status = OR_MAXIT;
done:
    finish(A, b, x, rho0, tmp, prod, info);
    free(r0); free(r); free(w); free(t); free(ph); free(s); free(z); free(v); free(q); free(y);
    free(tmp); free(prod);
    if (pc) { free(rh); free(wh); free(sh); free(zh); free(qh); }
    return info->status;
oom:
    free(r0); free(r); free(w); free(t); free(ph); free(s); free(z); free(v); free(q); free(y);
    free(tmp); free(prod);
    if (pc) { free(rh); free(wh); free(sh); free(zh); free(qh); }
    return OR_ERR_ALLOC;
}

/* ------------------------------------------------------------------------ */
/* Alg. 8 (communication-avoiding BiCGStab, Section 3.1), unpreconditioned: */
/* s_i and y_i come from recurrences (eqs. (1) and (4)), so the iteration   */
/* has two reduction phases, (q,y), (y,y) and then (r_0,r_{i+1}),           */
/* (r_0,w_{i+1}), (r_0,s_i), (r_0,z_i), the second one finishing beta_i and */
/* alpha_{i+1} together.  The squared norm of r_{i+1} joins that second     */
/* phase for the stopping test.  No residual replacement.                   */
/* ------------------------------------------------------------------------ */
static int ca_bicgstab(const csr_t* A, const double* b, double* x, const or_opts* o, or_info* info)
{
    const int32_t n = A->n;
    double *r0 = 0, *r = 0, *w = 0, *p = 0, *s = 0, *z = 0, *q = 0, *y = 0, *tmp = 0, *prod = 0;
    NEWVEC(r0); NEWVEC(r); NEWVEC(w); NEWVEC(p); NEWVEC(s); NEWVEC(z); NEWVEC(q); NEWVEC(y); NEWVEC(tmp);
    prod = (double*)malloc(sizeof(double) * (size_t)pow2_at_least(n));
    if (!prod) goto oom;

    info->iters = 0; info->n_rr = 0; info->relres_rec = 1.0; info->relres_true = 0.0;
    /* initial residual, w from it, first step length from the setup's inner products; beta starts at 0 */
    spmv(A, x, tmp);
    PAR for (int32_t j = 0; j < n; ++j) r0[j] = b[j] - tmp[j];
    double gamma = DOT(r0, r0);
    const double rho0 = sqrt(gamma);
    if (o->history) o->history[0] = 1.0;
    if (!isfinite(rho0)) { info->status = OR_NONFINITE; goto done; }
    if (rho0 == 0.0) { info->status = OR_SUCCESS; info->relres_rec = 0.0; goto done; }
    memcpy(r, r0, sizeof(double) * (size_t)n);
    spmv(A, r, w);
    double delta = DOT(r0, w);
    if (!isfinite(delta)) { info->status = OR_NONFINITE; goto done; }
    if (delta == 0.0) { info->status = OR_BREAKDOWN; goto done; }
    double alpha = gamma / delta, beta = 0.0, omega = 0.0;
    if (!isfinite(alpha)) { info->status = OR_NONFINITE; goto done; }
    /* p_{-1} = s_{-1} = z_{-1} = 0 (calloc), omega_{-1} = 0 */

    for (int32_t i = 0; i < o->maxit; ++i) {
        /* search direction from the residual and the previous direction */
        PAR for (int32_t j = 0; j < n; ++j) p[j] = r[j] + beta * (p[j] - omega * s[j]);
        /* s by its recurrence, eq. (1), instead of a product with A */
        PAR for (int32_t j = 0; j < n; ++j) s[j] = w[j] + beta * (s[j] - omega * z[j]);
        FLOPS(8); REC(2);
        /* the first product of the iteration: z from s */
        spmv(A, s, z);
        /* q and y by their recurrences, eq. (4) */
        PAR for (int32_t j = 0; j < n; ++j) q[j] = r[j] - alpha * s[j];
        PAR for (int32_t j = 0; j < n; ++j) y[j] = w[j] - alpha * z[j];
        FLOPS(4); REC(2);
        /* reduction (q_i, y_i), (y_i, y_i) ; omega_i */
        double th1 = DOT(q, y), th2 = DOT(y, y);
        g_ctr.glred++; g_ctr.dots += 2; FLOPS(4);
        if (!isfinite(th1) || !isfinite(th2)) { info->status = OR_NONFINITE; goto done; }
        if (th2 == 0.0) {
            PAR for (int32_t j = 0; j < n; ++j) x[j] = x[j] + alpha * p[j];
            info->iters = i + 1; info->relres_rec = 0.0; info->status = OR_SUCCESS;
            if (o->history) o->history[i + 1] = 0.0;
            goto done;
        }
        omega = th1 / th2;
        if (!isfinite(omega)) { info->status = OR_NONFINITE; goto done; }
        /* iterate and residual updates */
        PAR for (int32_t j = 0; j < n; ++j) x[j] = x[j] + alpha * p[j] + omega * q[j];
        PAR for (int32_t j = 0; j < n; ++j) r[j] = q[j] - omega * y[j];
        FLOPS(6); REC(2);
        info->iters = i + 1;
        /* the second product of the iteration: w from the new residual */
        spmv(A, r, w);
        /* reduction (r_0,r_{i+1}), (r_0,w_{i+1}), (r_0,s_i), (r_0,z_i), plus ||r_{i+1}||^2 */
        double gamma1 = DOT(r0, r), eta = DOT(r0, w), sig_s = DOT(r0, s), sig_z = DOT(r0, z);
        double nu = DOT(r, r);
        g_ctr.glred++; g_ctr.dots += 4; FLOPS(8);
        if (o->scalars) { o->scalars[3 * i] = alpha; o->scalars[3 * i + 1] = omega; }
        if (!isfinite(gamma1) || !isfinite(eta) || !isfinite(sig_s) || !isfinite(sig_z) || !isfinite(nu)) {
            info->status = OR_NONFINITE; goto done;
        }
        info->relres_rec = sqrt(nu) / rho0;
        if (o->history) o->history[i + 1] = info->relres_rec;
        if (info->relres_rec <= o->tol) { info->status = OR_SUCCESS; goto done; }
        /* second reduction finished: beta, then the next alpha by eq. (3) or eq. (5) */
        if (omega == 0.0 || gamma == 0.0) { info->status = OR_BREAKDOWN; goto done; }
        beta = (alpha / omega) * (gamma1 / gamma);
        if (!isfinite(beta)) { info->status = OR_NONFINITE; goto done; }
        if (o->scalars) o->scalars[3 * i + 2] = beta;
        if (g_alpha_form == 5) {
            if (gamma1 == 0.0) { info->status = OR_BREAKDOWN; goto done; }
            double den5 = (1.0 / omega + eta / gamma1) - (beta * omega) * (sig_z / gamma1);
            if (den5 == 0.0) { info->status = OR_BREAKDOWN; goto done; }
            alpha = 1.0 / den5;
        } else {
            double den = eta + beta * sig_s - beta * omega * sig_z;
            if (den == 0.0 || gamma1 == 0.0) { info->status = OR_BREAKDOWN; goto done; }
            alpha = gamma1 / den;
        }
        if (!isfinite(alpha)) { info->status = OR_NONFINITE; goto done; }
        gamma = gamma1;
    }
    info->status = OR_MAXIT;
done:
    finish(A, b, x, rho0, tmp, prod, info);
    free(r0); free(r); free(w); free(p); free(s); free(z); free(q); free(y); free(tmp); free(prod);
    return info->status;
oom:
    free(r0); free(r); free(w); free(p); free(s); free(z); free(q); free(y); free(tmp); free(prod);
    return OR_ERR_ALLOC;
}

/* ------------------------------------------------------------------------ */
/* The CG family of Section 2, for symmetric positive definite A (and M):   */
/*   Alg. 2  standard preconditioned CG: two reduction phases per iteration; */
/*   Alg. 4  Chronopoulos & Gear CG: one reduction phase, w = A u by         */
/*           recurrence-free SpMV, alpha from (delta/gamma - beta/alpha)^-1; */
/*   Alg. 6  pipelined CG (p-CG): one reduction phase overlapped with the   */
/*           SpMV n = A M^{-1} w; z, q, s, p, x, r, u, w by recurrences.    */
/* M^{-1} = diag(dinv) or the identity (dinv == NULL; then u = r, and in    */
/* Alg. 6 also m = w and q = s).  The squared norm of r joins a reduction   */
/* phase for the stopping test ||r_i|| / ||r_0|| <= tol.  scalars[3i] and    */
/* scalars[3i+2] hold alpha_i and beta_{i+1} (Alg. 2) or beta_i (Alg. 4, 6). */
/* ------------------------------------------------------------------------ */
static int cg(const csr_t* A, const double* dinv, const double* b, double* x, const or_opts* o, or_info* info)
{
    const int32_t n = A->n;
    const int pc = (dinv != NULL);
    double *r = 0, *u = 0, *p = 0, *s = 0, *tmp = 0, *prod = 0;
    NEWVEC(r); NEWVEC(p); NEWVEC(s); NEWVEC(tmp);
    if (pc) NEWVEC(u); else u = r;
    prod = (double*)malloc(sizeof(double) * (size_t)pow2_at_least(n));
    if (!prod) goto oom;

    info->iters = 0; info->n_rr = 0; info->relres_rec = 1.0; info->relres_true = 0.0;
    /* initial residual, its preconditioned copy, and the first search direction equal to that copy */
    spmv(A, x, tmp);
    PAR for (int32_t j = 0; j < n; ++j) r[j] = b[j] - tmp[j];
    if (pc) { PAR for (int32_t j = 0; j < n; ++j) u[j] = dinv[j] * r[j]; }
    memcpy(p, u, sizeof(double) * (size_t)n);
    const double rho0 = sqrt(DOT(r, r));
    double gamma = DOT(r, u);
    if (o->history) o->history[0] = 1.0;
    if (!isfinite(rho0) || !isfinite(gamma)) { info->status = OR_NONFINITE; goto done; }
    if (rho0 == 0.0) { info->status = OR_SUCCESS; info->relres_rec = 0.0; goto done; }

    for (int32_t i = 0; i < o->maxit; ++i) {
        /* product with the search direction, then the step length from the first reduction */
        spmv(A, p, s);
        double delta = DOT(s, p);
        g_ctr.glred++; g_ctr.dots++; FLOPS(2);
        if (!isfinite(delta)) { info->status = OR_NONFINITE; goto done; }
        if (delta == 0.0) { info->status = OR_BREAKDOWN; goto done; }
        double alpha = gamma / delta;
        if (!isfinite(alpha)) { info->status = OR_NONFINITE; goto done; }
        /* iterate, residual and preconditioned residual updates */
        PAR for (int32_t j = 0; j < n; ++j) x[j] = x[j] + alpha * p[j];
        PAR for (int32_t j = 0; j < n; ++j) r[j] = r[j] - alpha * s[j];
        if (pc) { PAR for (int32_t j = 0; j < n; ++j) u[j] = dinv[j] * r[j]; g_ctr.pc++; }
        FLOPS(4); REC(2);
        info->iters = i + 1;
        if (o->scalars) o->scalars[3 * i] = alpha;
        /* reduction (r_{i+1}, u_{i+1}) with ||r_{i+1}||^2 */
        double gamma1 = DOT(r, u), nu = DOT(r, r);
        g_ctr.glred++; g_ctr.dots++; FLOPS(2);
        if (!isfinite(gamma1) || !isfinite(nu)) { info->status = OR_NONFINITE; goto done; }
        info->relres_rec = sqrt(nu) / rho0;
        if (o->history) o->history[i + 1] = info->relres_rec;
        if (info->relres_rec <= o->tol) { info->status = OR_SUCCESS; goto done; }
        /* second reduction: beta, then the next search direction */
        if (gamma == 0.0) { info->status = OR_BREAKDOWN; goto done; }
        double beta = gamma1 / gamma;
        if (!isfinite(beta)) { info->status = OR_NONFINITE; goto done; }
        if (o->scalars) o->scalars[3 * i + 2] = beta;
        PAR for (int32_t j = 0; j < n; ++j) p[j] = u[j] + beta * p[j];
        FLOPS(2); REC(1);
        gamma = gamma1;
    }
    info->status = OR_MAXIT;
done:
    finish(A, b, x, rho0, tmp, prod, info);
    free(r); free(p); free(s); free(tmp); free(prod);
    if (pc) free(u);
    return info->status;
oom:
    free(r); free(p); free(s); free(tmp); free(prod);
    if (pc) free(u);
    return OR_ERR_ALLOC;
}

/* alpha of Alg. 4 and Alg. 6 after the first iteration: (delta/gamma - beta/alpha_prev)^{-1}. */
static int cg_next_alpha(double gamma1, double gamma, double delta, double alpha_prev, double* beta,
                         double* alpha)
{
    if (gamma == 0.0 || gamma1 == 0.0 || alpha_prev == 0.0) return OR_BREAKDOWN;
    *beta = gamma1 / gamma;
    if (!isfinite(*beta)) return OR_NONFINITE;
    double den = delta / gamma1 - *beta / alpha_prev;
    if (den == 0.0) return OR_BREAKDOWN;
    *alpha = 1.0 / den;
    if (!isfinite(*alpha)) return OR_NONFINITE;
    return OR_SUCCESS;
}

static int cgcg(const csr_t* A, const double* dinv, const double* b, double* x, const or_opts* o, or_info* info)
{
    const int32_t n = A->n;
    const int pc = (dinv != NULL);
    double *r = 0, *u = 0, *w = 0, *p = 0, *s = 0, *tmp = 0, *prod = 0;
    NEWVEC(r); NEWVEC(w); NEWVEC(p); NEWVEC(s); NEWVEC(tmp);
    if (pc) NEWVEC(u); else u = r;
    prod = (double*)malloc(sizeof(double) * (size_t)pow2_at_least(n));
    if (!prod) goto oom;

    info->iters = 0; info->n_rr = 0; info->relres_rec = 1.0; info->relres_true = 0.0;
    /* initial residual, its preconditioned copy u, and w = A u */
    spmv(A, x, tmp);
    PAR for (int32_t j = 0; j < n; ++j) r[j] = b[j] - tmp[j];
    if (pc) { PAR for (int32_t j = 0; j < n; ++j) u[j] = dinv[j] * r[j]; }
    spmv(A, u, w);
    const double rho0 = sqrt(DOT(r, r));
    double gamma = DOT(r, u), delta = DOT(w, u);
    if (o->history) o->history[0] = 1.0;
    if (!isfinite(rho0) || !isfinite(gamma) || !isfinite(delta)) { info->status = OR_NONFINITE; goto done; }
    if (rho0 == 0.0) { info->status = OR_SUCCESS; info->relres_rec = 0.0; goto done; }
    /* first step length from the setup's inner products; beta and the previous directions start at 0 */
    if (delta == 0.0) { info->status = OR_BREAKDOWN; goto done; }
    double alpha = gamma / delta, beta = 0.0;
    if (!isfinite(alpha)) { info->status = OR_NONFINITE; goto done; }

    for (int32_t i = 0; i < o->maxit; ++i) {
        /* search direction p and its product s, both by recurrence */
        PAR for (int32_t j = 0; j < n; ++j) p[j] = u[j] + beta * p[j];
        PAR for (int32_t j = 0; j < n; ++j) s[j] = w[j] + beta * s[j];
        /* iterate and residual updates */
        PAR for (int32_t j = 0; j < n; ++j) x[j] = x[j] + alpha * p[j];
        PAR for (int32_t j = 0; j < n; ++j) r[j] = r[j] - alpha * s[j];
        FLOPS(8); REC(4);
        /* preconditioned residual, then its product with A */
        if (pc) { PAR for (int32_t j = 0; j < n; ++j) u[j] = dinv[j] * r[j]; g_ctr.pc++; }
        spmv(A, u, w);
        info->iters = i + 1;
        if (o->scalars) o->scalars[3 * i] = alpha;
        /* the single reduction phase of Algorithm 4: the two inner products and the residual norm */
        double gamma1 = DOT(r, u), nu = DOT(r, r);
        delta = DOT(w, u);
        g_ctr.glred++; g_ctr.dots += 2; FLOPS(4);
        if (!isfinite(gamma1) || !isfinite(delta) || !isfinite(nu)) { info->status = OR_NONFINITE; goto done; }
        info->relres_rec = sqrt(nu) / rho0;
        if (o->history) o->history[i + 1] = info->relres_rec;
        if (info->relres_rec <= o->tol) { info->status = OR_SUCCESS; goto done; }
        /* beta from consecutive preconditioned residual norms, then the next alpha from both */
        int st = cg_next_alpha(gamma1, gamma, delta, alpha, &beta, &alpha);
        if (st != OR_SUCCESS) { info->status = st; goto done; }
        if (o->scalars && i + 1 < o->maxit) o->scalars[3 * (i + 1) + 2] = beta;
        gamma = gamma1;
    }
    info->status = OR_MAXIT;
done:
    finish(A, b, x, rho0, tmp, prod, info);
    free(r); free(w); free(p); free(s); free(tmp); free(prod);
    if (pc) free(u);
    return info->status;
oom:
    free(r); free(w); free(p); free(s); free(tmp); free(prod);
    if (pc) free(u);
    return OR_ERR_ALLOC;
}

static int pipe_cg(const csr_t* A, const double* dinv, const double* b, double* x, const or_opts* o,
                   or_info* info)
{
    const int32_t n = A->n;
    const int pc = (dinv != NULL);
    double *r = 0, *u = 0, *w = 0, *m = 0, *nv = 0, *z = 0, *q = 0, *s = 0, *p = 0, *tmp = 0, *prod = 0;
    NEWVEC(r); NEWVEC(w); NEWVEC(nv); NEWVEC(z); NEWVEC(s); NEWVEC(p); NEWVEC(tmp);
    if (pc) { NEWVEC(u); NEWVEC(m); NEWVEC(q); } else { u = r; m = w; q = s; }
    prod = (double*)malloc(sizeof(double) * (size_t)pow2_at_least(n));
    if (!prod) goto oom;

    info->iters = 0; info->n_rr = 0; info->relres_rec = 1.0; info->relres_true = 0.0;
    /* initial residual, its preconditioned copy u, w = A u; all the auxiliary recurrences start at 0 */
    spmv(A, x, tmp);
    PAR for (int32_t j = 0; j < n; ++j) r[j] = b[j] - tmp[j];
    if (pc) { PAR for (int32_t j = 0; j < n; ++j) u[j] = dinv[j] * r[j]; }
    spmv(A, u, w);
    double rho0 = 0.0, alpha = 0.0, beta = 0.0, gamma = 0.0;
    if (o->history) o->history[0] = 1.0;

    for (int32_t i = 0;; ++i) {
        /* the reduction phase of Algorithm 6, on vectors the previous iteration finished */
        double gamma1 = DOT(r, u), delta = DOT(w, u), nu = DOT(r, r);
        if (i > 0) { g_ctr.glred++; g_ctr.dots += 2; FLOPS(4); }
        if (!isfinite(gamma1) || !isfinite(delta) || !isfinite(nu)) { info->status = OR_NONFINITE; goto done; }
        if (i == 0) {
            rho0 = sqrt(nu);
            if (rho0 == 0.0) { info->status = OR_SUCCESS; info->relres_rec = 0.0; goto done; }
        } else {
            info->relres_rec = sqrt(nu) / rho0;
            if (o->history) o->history[i] = info->relres_rec;
            if (info->relres_rec <= o->tol) { info->status = OR_SUCCESS; goto done; }
        }
        /* end reduction: beta_i, alpha_i (taken, like Alg. 4's, before the iteration budget is checked) */
        if (i == 0) {
            if (delta == 0.0) { info->status = OR_BREAKDOWN; goto done; }
            beta = 0.0;
            alpha = gamma1 / delta;
            if (!isfinite(alpha)) { info->status = OR_NONFINITE; goto done; }
        } else {
            int st = cg_next_alpha(gamma1, gamma, delta, alpha, &beta, &alpha);
            if (st != OR_SUCCESS) { info->status = st; goto done; }
        }
        gamma = gamma1;
        if (i == o->maxit) { info->status = OR_MAXIT; goto done; }
        if (o->scalars) { o->scalars[3 * i] = alpha; o->scalars[3 * i + 2] = beta; }
        /* the product the reduction overlaps in the paper (computed after it here; the order changes
           no value) */
        if (pc) { PAR for (int32_t j = 0; j < n; ++j) m[j] = dinv[j] * w[j]; g_ctr.pc++; }
        spmv(A, m, nv);
        /* the four auxiliary recurrences (z, q, s and the search direction p) with the new beta */
        PAR for (int32_t j = 0; j < n; ++j) z[j] = nv[j] + beta * z[j];
        if (pc) PAR for (int32_t j = 0; j < n; ++j) q[j] = m[j] + beta * q[j];
        PAR for (int32_t j = 0; j < n; ++j) s[j] = w[j] + beta * s[j];
        PAR for (int32_t j = 0; j < n; ++j) p[j] = u[j] + beta * p[j];
        /* iterate, residual and auxiliary updates with the new alpha */
        PAR for (int32_t j = 0; j < n; ++j) x[j] = x[j] + alpha * p[j];
        PAR for (int32_t j = 0; j < n; ++j) r[j] = r[j] - alpha * s[j];
        if (pc) PAR for (int32_t j = 0; j < n; ++j) u[j] = u[j] - alpha * q[j];
        PAR for (int32_t j = 0; j < n; ++j) w[j] = w[j] - alpha * z[j];
        FLOPS(pc ? 16 : 12); REC(pc ? 8 : 6);
        info->iters = i + 1;
    }
done:
    finish(A, b, x, rho0, tmp, prod, info);
    free(r); free(w); free(nv); free(z); free(s); free(p); free(tmp); free(prod);
    if (pc) { free(u); free(m); free(q); }
    return info->status;
oom:
    free(r); free(w); free(nv); free(z); free(s); free(p); free(tmp); free(prod);
    if (pc) { free(u); free(m); free(q); }
    return OR_ERR_ALLOC;
}

/* ------------------------------------------------------------------------ */
/* Precision form: p-BiCGStab (Alg. 9) with FP32 vectors, SpMV, recurrences */
/* and dot products, and FP64 residual replacement (Section 4.2), x update  */
/* and scalars alpha, beta, omega.                                           */
/*                                                                           */
/* f() is rounding to binary32.  The FP32 operator holds f(a_ij).  A dot    */
/* product is the pairwise sum of the binary32 products in binary32, + 0.0f, */
/* then widened.  Vector updates take the scalars rounded to binary32.  The  */
/* replacement steps run in binary64 on the binary64 operator and the       */
/* binary64 x, and round once when stored: r = f(b - A x), w = f(A (b - A x)),*/
/* s = f(A p), z = f(A (A p)).  The setup is such a replacement.             */
/* Convergence of the FP32 recursive residual is confirmed with the FP64    */
/* true residual ||b - A x|| / rho0; if that is still above tol, the        */
/* iteration is a replacement iteration and goes on.                        */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t n;
    const int32_t* rp;
    const int32_t* ci;
    const float* va;
} csr32_t;

/* Product with the binary32 operator in binary32, rows in stored order from 0.0f. */
static void spmv32(const csr32_t* A, const float* x, float* y)
{
    PAR for (int32_t i = 0; i < A->n; ++i) {
        float acc = 0.0f;
        for (int32_t k = A->rp[i]; k < A->rp[i + 1]; ++k) acc = acc + A->va[k] * x[A->ci[k]];
        y[i] = acc;
    }
    g_ctr.spmv++;
}

/* Product with the binary64 operator on a binary32 vector (widened exactly). */
static void spmv_wide(const csr_t* A, const float* x, double* y)
{
    PAR for (int32_t i = 0; i < A->n; ++i) {
        double acc = 0.0;
        for (int32_t k = A->rp[i]; k < A->rp[i + 1]; ++k) acc = acc + A->va[k] * (double)x[A->ci[k]];
        y[i] = acc;
    }
    g_ctr.spmv++;
}

static float pairwise32(const float* a, int64_t len)
{
    if (len == 1) return a[0];
    return pairwise32(a, len / 2) + pairwise32(a + len / 2, len / 2);
}

static float pairwise32_par(const float* a, int64_t len)
{
    if (len < (1 << 16)) return pairwise32(a, len);
    float part[64];
    const int64_t bl = len / 64;
    PAR for (int b = 0; b < 64; ++b) part[b] = pairwise32(a + b * bl, bl);
    return pairwise32(part, 64);
}

/* (x, y) in binary32, pairwise, widened to binary64. */
static double dot32_ws(int64_t n, const float* x, const float* y, float* prod)
{
    const int64_t len = pow2_at_least(n);
    PAR for (int64_t i = 0; i < len; ++i) prod[i] = (i < n) ? x[i] * y[i] : 0.0f;
    return (double)(pairwise32_par(prod, len) + 0.0f);
}

double or_dot32(int64_t n, const float* x, const float* y)
{
    if (n <= 0) return 0.0;
    float* prod = (float*)malloc(sizeof(float) * (size_t)pow2_at_least(n));
    if (!prod) return NAN;
    double s = dot32_ws(n, x, y, prod);
    free(prod);
    return s;
}

void or_spmv32(int32_t n, const int32_t* rp, const int32_t* ci, const float* va, const float* x, float* y)
{
    csr32_t A = {n, rp, ci, va};
    spmv32(&A, x, y);
}

/* periodic replacement in iteration i: (i+1) mod k == 0, at most rr_max of them */
static int rr_due_periodic(const or_opts* o, int32_t i)
{
    if (o->rr_period <= 0 || (i + 1) % o->rr_period != 0) return 0;
    return (o->rr_max < 0) || ((i + 1) / o->rr_period <= o->rr_max);
}

#define NEWV32(p) do { (p) = (float*)calloc((size_t)n, sizeof(float)); if (!(p)) goto oom; } while (0)
#define DOT32(a, b) dot32_ws(n, (a), (b), prod32)

static int pbicgstab_mp(const csr_t* A, const double* b, double* x, const or_opts* o, or_info* info)
{
    const int32_t n = A->n;
    float *va32 = 0, *r0 = 0, *r = 0, *w = 0, *t = 0, *p = 0, *s = 0, *z = 0, *v = 0, *q = 0, *y = 0;
    float* prod32 = 0;
    double *r64 = 0, *w64 = 0, *tmp = 0, *prod = 0;
    const int64_t nnz = A->rp[n];
    va32 = (float*)malloc(sizeof(float) * (size_t)(nnz > 0 ? nnz : 1));
    if (!va32) goto oom;
    for (int64_t k = 0; k < nnz; ++k) va32[k] = (float)A->va[k];
    csr32_t A32 = {n, A->rp, A->ci, va32};
    NEWV32(r0); NEWV32(r); NEWV32(w); NEWV32(t); NEWV32(p); NEWV32(s); NEWV32(z); NEWV32(v);
    NEWV32(q); NEWV32(y);
    NEWVEC(r64); NEWVEC(w64); NEWVEC(tmp);
    prod32 = (float*)malloc(sizeof(float) * (size_t)pow2_at_least(n));
    prod = (double*)malloc(sizeof(double) * (size_t)pow2_at_least(n));
    if (!prod32 || !prod) goto oom;

    info->iters = 0; info->n_rr = 0; info->relres_rec = 1.0; info->relres_true = 0.0;
    /* setup as a replacement: r_0 = f(b - A x_0), w_0 = f(A (b - A x_0)) */
    spmv(A, x, tmp);
    PAR for (int32_t j = 0; j < n; ++j) r64[j] = b[j] - tmp[j];
    PAR for (int32_t j = 0; j < n; ++j) { r0[j] = (float)r64[j]; r[j] = r0[j]; }
    double gamma = DOT32(r0, r0);
    const double rho0 = sqrt(gamma);
    if (o->history) o->history[0] = 1.0;
    if (!isfinite(rho0)) { info->status = OR_NONFINITE; goto done; }
    if (rho0 == 0.0) { info->status = OR_SUCCESS; info->relres_rec = 0.0; goto done; }
    spmv(A, r64, w64);
    PAR for (int32_t j = 0; j < n; ++j) w[j] = (float)w64[j];
    spmv32(&A32, w, t);
    double delta = DOT32(r0, w);
    if (!isfinite(delta)) { info->status = OR_NONFINITE; goto done; }
    if (delta == 0.0) { info->status = OR_BREAKDOWN; goto done; }
    double alpha = gamma / delta, beta = 0.0, omega = 0.0;
    if (!isfinite(alpha)) { info->status = OR_NONFINITE; goto done; }
    int rr_pending = 0;
    int32_t n_rr = 0;

    for (int32_t i = 0; i < o->maxit; ++i) {
        const float af = (float)alpha, bf = (float)beta, wf = (float)omega;
        /* search direction from the residual and the previous direction (binary32) */
        PAR for (int32_t j = 0; j < n; ++j) p[j] = r[j] + bf * (p[j] - wf * s[j]);
        if (rr_pending) {
            /* replacement, second half, in binary64: s = f(A p), z = f(A (A p)) */
            spmv_wide(A, p, r64);
            PAR for (int32_t j = 0; j < n; ++j) s[j] = (float)r64[j];
            spmv(A, r64, w64);
            PAR for (int32_t j = 0; j < n; ++j) z[j] = (float)w64[j];
            rr_pending = 0;
        } else {
            /* s_i, z_i from the old s, z, v */
            PAR for (int32_t j = 0; j < n; ++j) s[j] = w[j] + bf * (s[j] - wf * z[j]);
            PAR for (int32_t j = 0; j < n; ++j) z[j] = t[j] + bf * (z[j] - wf * v[j]);
        }
        /* intermediate residual q and y by recurrence (binary32) */
        PAR for (int32_t j = 0; j < n; ++j) { q[j] = r[j] - af * s[j]; y[j] = w[j] - af * z[j]; }
        double th1 = DOT32(q, y), th2 = DOT32(y, y);
        /* the product overlapped by the first reduction: v from z */
        spmv32(&A32, z, v);
        if (!isfinite(th1) || !isfinite(th2)) { info->status = OR_NONFINITE; goto done; }
        if (th2 == 0.0) {
            PAR for (int32_t j = 0; j < n; ++j) x[j] = x[j] + alpha * (double)p[j];
            info->iters = i + 1; info->relres_rec = 0.0; info->status = OR_SUCCESS;
            if (o->history) o->history[i + 1] = 0.0;
            goto done;
        }
        omega = th1 / th2;
        if (!isfinite(omega)) { info->status = OR_NONFINITE; goto done; }
        const float wn = (float)omega;
        /* the iterate is updated in binary64 from the binary32 directions */
        PAR for (int32_t j = 0; j < n; ++j) x[j] = x[j] + alpha * (double)p[j] + omega * (double)q[j];
        /* residual and w recurrences (binary32) */
        PAR for (int32_t j = 0; j < n; ++j) {
            r[j] = q[j] - wn * y[j];
            w[j] = y[j] - wn * (t[j] - af * v[j]);
        }
        info->iters = i + 1;
        int replaced = 0;
        for (;;) {
            if (!replaced && rr_due_periodic(o, i)) replaced = 1;
            if (replaced == 1 || replaced == 3) {
                /* replacement, first half, in binary64 */
                spmv(A, x, tmp);
                PAR for (int32_t j = 0; j < n; ++j) r64[j] = b[j] - tmp[j];
                PAR for (int32_t j = 0; j < n; ++j) r[j] = (float)r64[j];
                spmv(A, r64, w64);
                PAR for (int32_t j = 0; j < n; ++j) w[j] = (float)w64[j];
                rr_pending = 1;
                ++n_rr;
                info->n_rr = n_rr;
                replaced = (replaced == 3) ? 4 : 2;  /* 4: forced; no second stop test */
            }
            /* (r0,r), (r0,w), (r0,s), (r0,z) and ||r||^2 */
            double gamma1 = DOT32(r0, r), eta = DOT32(r0, w), sig_s = DOT32(r0, s), sig_z = DOT32(r0, z);
            double nu = DOT32(r, r);
            if (!isfinite(gamma1) || !isfinite(eta) || !isfinite(sig_s) || !isfinite(sig_z) || !isfinite(nu)) {
                info->status = OR_NONFINITE; goto done;
            }
            info->relres_rec = sqrt(nu) / rho0;
            if (o->history) o->history[i + 1] = info->relres_rec;
            if (o->scalars) { o->scalars[3 * i] = alpha; o->scalars[3 * i + 1] = omega; }
            if (info->relres_rec <= o->tol && replaced != 4) {
                /* confirm with the binary64 true residual */
                spmv(A, x, tmp);
                PAR for (int32_t j = 0; j < n; ++j) r64[j] = b[j] - tmp[j];
                const double tr = sqrt(DOT(r64, r64)) / rho0;
                if (tr <= o->tol) { info->status = OR_SUCCESS; goto done; }
                replaced = 3;  /* not converged: replace now and reduce again */
                continue;
            }
            /* the product overlapped by the second reduction: t from w */
            spmv32(&A32, w, t);
            /* beta_i ; alpha_{i+1} by eq. (3) */
            if (omega == 0.0 || gamma == 0.0) { info->status = OR_BREAKDOWN; goto done; }
            beta = (alpha / omega) * (gamma1 / gamma);
            if (!isfinite(beta)) { info->status = OR_NONFINITE; goto done; }
            if (o->scalars) o->scalars[3 * i + 2] = beta;
            if (g_alpha_form == 5) {
                if (gamma1 == 0.0) { info->status = OR_BREAKDOWN; goto done; }
                double den5 = (1.0 / omega + eta / gamma1) - (beta * omega) * (sig_z / gamma1);
                if (den5 == 0.0) { info->status = OR_BREAKDOWN; goto done; }
                alpha = 1.0 / den5;
            } else {
                double den = eta + beta * sig_s - beta * omega * sig_z;
                if (den == 0.0 || gamma1 == 0.0) { info->status = OR_BREAKDOWN; goto done; }
                alpha = gamma1 / den;
            }
            if (!isfinite(alpha)) { info->status = OR_NONFINITE; goto done; }
            gamma = gamma1;
            break;
        }
    }
    info->status = OR_MAXIT;
done:
    finish(A, b, x, rho0, tmp, prod, info);
    free(va32); free(r0); free(r); free(w); free(t); free(p); free(s); free(z); free(v); free(q); free(y);
    free(prod32); free(r64); free(w64); free(tmp); free(prod);
    return info->status;
oom:
    free(va32); free(r0); free(r); free(w); free(t); free(p); free(s); free(z); free(v); free(q); free(y);
    free(prod32); free(r64); free(w64); free(tmp); free(prod);
    return OR_ERR_ALLOC;
}

/* Entry point of the precision form (no preconditioner argument: a
 * preconditioned solve passes A M^{-1} formed).  Arguments as or_solve. */
int or_solve_mp(int32_t n, const int32_t* rp, const int32_t* ci, const double* va,
                const double* b, double* x, double tol, int32_t maxit, int32_t rr_period, int32_t rr_max,
                double* history, double* scalars, int32_t* ints_out, double* dbl_out)
{
    if (n <= 0 || !rp || !ci || !va || !b || !x || maxit < 0 || !(tol >= 0.0) || rr_period < 0)
        return OR_ERR_INVALID_ARG;
    csr_t A = {n, rp, ci, va};
    or_opts o = {tol, maxit, rr_period, rr_max, history, scalars};
    or_info info = {0, 0, 0, 0.0, 0.0};
    int st = pbicgstab_mp(&A, b, x, &o, &info);
    if (st < 0) return st;
    ints_out[0] = info.iters; ints_out[1] = info.n_rr; ints_out[2] = info.status;
    dbl_out[0] = info.relres_rec; dbl_out[1] = info.relres_true;
    return st;
}

/*
 * Entry point.  algo: 0 BiCGStab (Alg. 7 / 10), 1 p-BiCGStab (Alg. 9 / 11),
 * 2 p-BiCGStab with residual replacement, 3 CA-BiCGStab (Alg. 8; dinv must
 * be NULL), 4 CG (Alg. 2), 5 Chronopoulos & Gear CG (Alg. 4), 6 p-CG
 * (Alg. 6); the last three need a symmetric positive definite A.
 * dinv NULL = no preconditioner.
 * x holds x_0 on entry and the final iterate on return.
 * ints_out[3] = {iters, n_rr, status}; dbl_out[2] = {relres_rec, relres_true}.
 */
int or_solve(int32_t algo, int32_t n, const int32_t* rp, const int32_t* ci, const double* va,
             const double* dinv, const double* b, double* x,
             double tol, int32_t maxit, int32_t rr_period, int32_t rr_max,
             double* history, double* scalars, int32_t* ints_out, double* dbl_out)
{
    if (n <= 0 || !rp || !ci || !va || !b || !x || maxit < 0 || !(tol >= 0.0)) return OR_ERR_INVALID_ARG;
    csr_t A = {n, rp, ci, va};
    or_opts o = {tol, maxit, (algo == 2) ? rr_period : 0, rr_max, history, scalars};
    or_info info = {0, 0, 0, 0.0, 0.0};
    int st;
    if (algo == 0) st = bicgstab(&A, dinv, b, x, &o, &info);
    else if (algo == 1 || algo == 2) st = pbicgstab(&A, dinv, b, x, &o, &info);
    else if (algo == 3 && !dinv) st = ca_bicgstab(&A, b, x, &o, &info);
    else if (algo == 4) st = cg(&A, dinv, b, x, &o, &info);
    else if (algo == 5) st = cgcg(&A, dinv, b, x, &o, &info);
    else if (algo == 6) st = pipe_cg(&A, dinv, b, x, &o, &info);
    else return OR_ERR_INVALID_ARG;
    if (st < 0) return st;
    ints_out[0] = info.iters; ints_out[1] = info.n_rr; ints_out[2] = info.status;
    dbl_out[0] = info.relres_rec; dbl_out[1] = info.relres_true;
    return st;
}

/* Thread control for the OpenMP loops (results do not depend on it). */
#include <omp.h>
void or_set_threads(int32_t t) { if (t > 0) omp_set_num_threads(t); }
int32_t or_get_threads(void) { return (int32_t)omp_get_max_threads(); }
