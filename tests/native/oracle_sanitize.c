/*
 * Drives the oracle's C routines on small inputs under AddressSanitizer and
 * UndefinedBehaviorSanitizer (built by tests/test_oracle_sanitize.py with
 * gcc -fsanitize=address,undefined together with oracle/gcp_oracle.c): the
 * sorted index, stratified / semi-stratified / uniform sampling, the sampled
 * gradient and its rounding bound, the non-fused steps, Adam and the
 * parallel timing step.  Exits 0 and prints "ok" when every call returns and
 * the fused and non-fused gradients agree; any invalid access or undefined
 * operation aborts under the sanitizers.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct ora_tensor ora_tensor;
ora_tensor* ora_tensor_new(int d, const int64_t* dims, int64_t nnz, const int64_t* coords, const double* vals,
                           int* status);
void ora_tensor_free(ora_tensor* t);
int ora_sample_stratified(const ora_tensor* t, int64_t p, int64_t q, uint64_t seed, uint64_t step, uint64_t client,
                          int64_t max_attempts, int semi, int64_t* coords_out, double* x_out, double* w_out);
int ora_sample_uniform(int d, const int64_t* dims, const double* dense, int64_t s_count, uint64_t seed,
                       uint64_t step, uint64_t client, int64_t* coords_out, double* x_out, double* w_out);
void ora_loss_grad(int d, const int64_t* dims, int R, const double* A, int64_t n, const int64_t* coords,
                   const double* x, const double* w, int loss, int64_t n_semi, double* G, double* F);
void ora_loss_grad_bound(int d, const int64_t* dims, int R, const double* A, int64_t n, const int64_t* coords,
                         const double* x, const double* w, int loss, int64_t n_semi, double u, double* abssum,
                         double* yerr, int64_t* count);
void ora_sample_derivatives(int d, const int64_t* dims, int R, const double* A, int64_t n, const int64_t* coords,
                            const double* x, const double* w, int loss, int64_t n_semi, double* y);
void ora_mttkrp(int d, const int64_t* dims, int R, const double* A, int64_t n, const int64_t* coords,
                const double* y, double* G);
void ora_adam(int64_t n, double* A, const double* G, double* B, double* C, int64_t t, double lr, double beta1,
              double beta2, double eps, double lower);
int ora_omp_sgd_step(const ora_tensor* t, int R, double* A, double* B, double* C, int64_t adam_t, int loss,
                     int64_t p, int64_t q, uint64_t seed, uint64_t step, int64_t max_attempts, double lr,
                     double beta1, double beta2, double eps, double lower, int nthreads, int64_t* coords_ws,
                     double* x_ws, double* w_ws, double* G_priv, double* G, int* threads_used);

int main(void)
{
    const int d = 3, R = 4;
    const int64_t dims[3] = {7, 6, 5};
    const int64_t M = 7 * 6 * 5, nnz = 40, rows = 18;
    int64_t* coords = malloc(sizeof(int64_t) * nnz * d);
    double* vals = malloc(sizeof(double) * nnz);
    for (int64_t j = 0; j < nnz; ++j) {          /* every fifth cell, distinct */
        int64_t c = (j * 5 + 2) % M;
        coords[j * d + 0] = c / 30;
        coords[j * d + 1] = (c / 5) % 6;
        coords[j * d + 2] = c % 5;
        vals[j] = 1.0 + (double)(j % 3);
    }
    int st = 0;
    ora_tensor* t = ora_tensor_new(d, dims, nnz, coords, vals, &st);
    if (!t || st != 0) { printf("tensor %d\n", st); return 1; }
    const int64_t p = 50, q = 70, n = p + q;
    int64_t* sc = malloc(sizeof(int64_t) * n * d);
    double *sx = malloc(sizeof(double) * n), *sw = malloc(sizeof(double) * n), *y = malloc(sizeof(double) * n);
    double *A = malloc(sizeof(double) * rows * R), *G = malloc(sizeof(double) * rows * R);
    double *G2 = malloc(sizeof(double) * rows * R), *B = calloc(rows * R, sizeof(double));
    double *C = calloc(rows * R, sizeof(double)), *abssum = malloc(sizeof(double) * rows * R);
    double* yerr = malloc(sizeof(double) * rows * R);
    int64_t* count = malloc(sizeof(int64_t) * rows);
    for (int64_t i = 0; i < rows * R; ++i) A[i] = 0.3 + 0.01 * (double)(i % 17);
    for (int semi = 0; semi < 2; ++semi) {
        if (ora_sample_stratified(t, p, q, 9, 1, 0, 64, semi, sc, sx, sw) != 0) return 2;
        for (int loss = 0; loss < 3; ++loss) {
            double F = 0.0;
            ora_loss_grad(d, dims, R, A, n, sc, sx, sw, loss, semi ? p : 0, G, &F);
            ora_loss_grad_bound(d, dims, R, A, n, sc, sx, sw, loss, semi ? p : 0, 0x1p-24, abssum, yerr, count);
            ora_sample_derivatives(d, dims, R, A, n, sc, sx, sw, loss, semi ? p : 0, y);
            ora_mttkrp(d, dims, R, A, n, sc, y, G2);
            for (int64_t i = 0; i < rows * R; ++i)
                if (fabs(G[i] - G2[i]) > 1e-12 * (1.0 + fabs(G[i]))) return 3;
        }
    }
    double* dense = malloc(sizeof(double) * M);
    for (int64_t i = 0; i < M; ++i) dense[i] = sin((double)i);
    if (ora_sample_uniform(d, dims, dense, n, 3, 0, 0, sc, sx, sw) != 0) return 4;
    ora_adam(rows * R, A, G, B, C, 1, 1e-3, 0.9, 0.999, 1e-8, 0.0);
    double* Gp = malloc(sizeof(double) * 2 * rows * R);
    int used = 0;
    if (ora_omp_sgd_step(t, R, A, B, C, 2, 1, p, q, 9, 2, 64, 1e-3, 0.9, 0.999, 1e-8, 0.0, 2, sc, sx, sw, Gp, G,
                         &used) != 0)
        return 5;
    ora_tensor_free(t);
    free(coords); free(vals); free(sc); free(sx); free(sw); free(y); free(A); free(G); free(G2); free(B); free(C);
    free(abssum); free(yerr); free(count); free(dense); free(Gp);
    printf("ok\n");
    return 0;
}
