/*
 * Plain-C user of the C ABI (include/pbcgs.h): assembles the 2-D 5-point
 * Poisson operator of an n x n grid on the host, copies it to the device with
 * the HIP runtime API, and solves A x = A 1 with p-BiCGStab and residual
 * replacement.  Exit status: 0 on a converged solve whose x is 1 to 1e-8,
 * 2 when no HIP device is available (the error path), 1 otherwise.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "pbcgs.h"

int main(int argc, char** argv) {
    const int n = argc > 1 ? atoi(argv[1]) : 64;
    const int N = n * n;
    int32_t* rp = malloc(sizeof(int32_t) * (N + 1));
    int32_t* ci = malloc(sizeof(int32_t) * 5 * N);
    double* va = malloc(sizeof(double) * 5 * N);
    double* ones = malloc(sizeof(double) * N);
    double* x = malloc(sizeof(double) * N);
    int64_t nnz = 0;
    rp[0] = 0;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            const int row = i + n * j;
            if (j > 0) { ci[nnz] = row - n; va[nnz++] = -1.0; }
            if (i > 0) { ci[nnz] = row - 1; va[nnz++] = -1.0; }
            ci[nnz] = row; va[nnz++] = 4.0;
            if (i < n - 1) { ci[nnz] = row + 1; va[nnz++] = -1.0; }
            if (j < n - 1) { ci[nnz] = row + n; va[nnz++] = -1.0; }
            rp[row + 1] = (int32_t)nnz;
            ones[row] = 1.0;
        }

    pbcgs_ctx_t ctx = NULL;
    int rc = pbcgs_ctx_create(0, NULL, &ctx);
    if (rc != PBCGS_SUCCESS) {
        printf("no context: %s (%s)\n", pbcgs_status_str(rc), pbcgs_last_error(NULL));
        return 2;
    }
    int32_t *d_rp, *d_ci;
    double *d_va, *d_b, *d_x, *d_one;
    if (hipMalloc((void**)&d_rp, sizeof(int32_t) * (N + 1)) != hipSuccess ||
        hipMalloc((void**)&d_ci, sizeof(int32_t) * nnz) != hipSuccess ||
        hipMalloc((void**)&d_va, sizeof(double) * nnz) != hipSuccess ||
        hipMalloc((void**)&d_b, sizeof(double) * N) != hipSuccess ||
        hipMalloc((void**)&d_x, sizeof(double) * N) != hipSuccess ||
        hipMalloc((void**)&d_one, sizeof(double) * N) != hipSuccess) {
        printf("device allocation failed\n");
        return 1;
    }
    hipMemcpy(d_rp, rp, sizeof(int32_t) * (N + 1), hipMemcpyHostToDevice);
    hipMemcpy(d_ci, ci, sizeof(int32_t) * nnz, hipMemcpyHostToDevice);
    hipMemcpy(d_va, va, sizeof(double) * nnz, hipMemcpyHostToDevice);
    hipMemcpy(d_one, ones, sizeof(double) * N, hipMemcpyHostToDevice);
    hipMemset(d_x, 0, sizeof(double) * N);

    pbcgs_op_t A = NULL;
    rc = pbcgs_op_csr(ctx, N, nnz, d_rp, d_ci, d_va, &A);
    if (rc == PBCGS_SUCCESS) rc = pbcgs_spmv(ctx, A, d_one, d_b); /* b = A 1 */
    pbcgs_opts o = {0};
    o.variant = PBCGS_PBICGSTAB_RR;
    o.precond = PBCGS_PRECOND_NONE;
    o.precision = PBCGS_FP64;
    o.maxit = 2000;
    o.tol = 1e-12;
    o.rr_period = 50;
    o.rr_max = -1;
    pbcgs_info info;
    if (rc == PBCGS_SUCCESS) rc = pbcgs_solve(ctx, A, d_b, d_x, NULL, &o, &info);
    if (rc < 0) {
        printf("error %s: %s\n", pbcgs_status_str(rc), pbcgs_last_error(ctx));
        return 1;
    }
    hipMemcpy(x, d_x, sizeof(double) * N, hipMemcpyDeviceToHost);
    double err = 0.0;
    for (int k = 0; k < N; ++k) err = fmax(err, fabs(x[k] - 1.0));
    printf("%s after %d iterations (%d replacements), true relative residual %.3e, max |x - 1| %.3e\n",
           pbcgs_status_str(info.status), info.iters, info.n_rr, info.relres_true, err);
    pbcgs_op_destroy(A);
    pbcgs_ctx_destroy(ctx);
    hipFree(d_rp); hipFree(d_ci); hipFree(d_va); hipFree(d_b); hipFree(d_x); hipFree(d_one);
    free(rp); free(ci); free(va); free(ones); free(x);
    return (info.status == PBCGS_SUCCESS && err < 1e-8) ? 0 : 1;
}
