/*
 * gcp_oracle.c -- plain, slow, serial FP64 CPU oracle for the GCP sampled
 * stochastic gradient (Myers & Phipps, "Synchronous and Asynchronous
 * Parallelism Approaches for Generalized Canonical Polyadic Tensor
 * Decomposition with GenTen", arXiv 2605.20353).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table or helper with the HIP library: it has its own
 * Philox4x64-10, its own membership search (lexicographically sorted
 * coordinate tuples + binary search, the O(log N) search of Sec. 3.1.1) and
 * its own serial MTTKRP (the "serial" strategy of Sec. 3.1.2).  Everything is
 * computed in double precision.
 *
 * Conventions (0-based indices; the paper writes 1-based ranges):
 *   - A Kruskal model is ONE contiguous array of sum_k I_k rows of R values,
 *     row-major, mode 0's rows first (the single contiguous factor array of
 *     Sec. 3.1.3).  rowoff[k] = sum_{j<k} I_j.
 *   - Sample lists are (coords [n x d] int64 row-major, x [n], w [n]).
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------------ */
/* Counter-based RNG: Philox4x64 with 10 rounds, as defined by Salmon,      */
/* Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3"     */
/* (SC'11).  The paper leaves the RNG unspecified; this is the reading.     */
/* ------------------------------------------------------------------------ */

/* Round multipliers and Weyl key increments published with Philox4x64. */
#define ORA_PHILOX_M0 0xD2E7470EE14C6C93ULL
#define ORA_PHILOX_M1 0xCA5A826395121157ULL
#define ORA_PHILOX_W0 0x9E3779B97F4A7C15ULL
#define ORA_PHILOX_W1 0xBB67AE8584CAA73BULL

void ora_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {           /* key schedule: bump between rounds */
            k0 += ORA_PHILOX_W0;
            k1 += ORA_PHILOX_W1;
        }
        u128 p0 = (u128)ORA_PHILOX_M0 * (u128)x0;
        u128 p1 = (u128)ORA_PHILOX_M1 * (u128)x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t y0 = hi1 ^ x1 ^ k0;
        uint64_t y1 = lo1;
        uint64_t y2 = hi0 ^ x3 ^ k1;
        uint64_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Exact map of a 64-bit uniform word u onto [0, n): floor(u * n / 2^64). */
uint64_t ora_range(uint64_t u, uint64_t n)
{
    return (uint64_t)(((u128)u * (u128)n) >> 64);
}

/* Stream tags carried in the third counter word (low 8 bits); the rejection
 * attempt number sits above them. */
enum { ORA_STREAM_NONZERO = 0, ORA_STREAM_ZERO = 1, ORA_STREAM_UNIFORM = 2 };

/* Draw the d coordinates of one candidate cell for sample s, attempt t. */
static void ora_draw_cell(int d, const int64_t* dims, uint64_t seed, uint64_t client,
                          uint64_t s, uint64_t step, uint64_t stream, uint64_t attempt,
                          int64_t* idx)
{
    uint64_t key[2] = {seed, client};
    for (int blk = 0; blk * 4 < d; ++blk) {
        uint64_t ctr[4] = {s, step, stream | (attempt << 8), (uint64_t)blk};
        uint64_t out[4];
        ora_philox4x64_10(ctr, key, out);
        for (int j = 0; j < 4 && blk * 4 + j < d; ++j) {
            int k = blk * 4 + j;
            idx[k] = (int64_t)ora_range(out[j], (uint64_t)dims[k]);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Sparse tensor in coordinate (COO) format with a lexicographically sorted */
/* index for O(log N) membership search (Sec. 3.1.1).                       */
/* ------------------------------------------------------------------------ */

typedef struct {
    int d;
    int64_t dims[8];
    int64_t nnz;
    const int64_t* coords; /* borrowed, nnz x d */
    const double* vals;    /* borrowed, nnz */
    int64_t* order;        /* owned: positions sorted by coordinate tuple */
} ora_tensor;

static int ora_cmp_tuple(const int64_t* a, const int64_t* b, int d)
{
    for (int k = 0; k < d; ++k) {
        if (a[k] < b[k]) return -1;
        if (a[k] > b[k]) return 1;
    }
    return 0;
}

static int ora_cmp_positions(const void* pa, const void* pb, void* arg)
{
    const ora_tensor* t = (const ora_tensor*)arg;
    int64_t a = *(const int64_t*)pa, b = *(const int64_t*)pb;
    return ora_cmp_tuple(t->coords + a * t->d, t->coords + b * t->d, t->d);
}

/* Status codes shared by the oracle entry points. */
enum { ORA_OK = 0, ORA_ERR_ARG = -1, ORA_ERR_SAMPLING = -4 };

/* Builds the sorted index.  *status = ORA_ERR_ARG on a coordinate outside the
 * dims or on a repeated coordinate tuple (the nonzero list must be a set). */
ora_tensor* ora_tensor_new(int d, const int64_t* dims, int64_t nnz, const int64_t* coords,
                           const double* vals, int* status)
{
    *status = ORA_ERR_ARG;
    if (d < 1 || d > 8 || nnz < 0) return NULL;
    ora_tensor* t = (ora_tensor*)calloc(1, sizeof(ora_tensor));
    t->d = d;
    for (int k = 0; k < d; ++k) t->dims[k] = dims[k];
    t->nnz = nnz;
    t->coords = coords;
    t->vals = vals;
    t->order = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nnz > 0 ? nnz : 1));
    for (int64_t j = 0; j < nnz; ++j) {
        for (int k = 0; k < d; ++k) {
            int64_t c = coords[j * d + k];
            if (c < 0 || c >= dims[k]) { free(t->order); free(t); return NULL; }
        }
        t->order[j] = j;
    }
    qsort_r(t->order, (size_t)nnz, sizeof(int64_t), ora_cmp_positions, t);
    for (int64_t j = 1; j < nnz; ++j) {
        if (ora_cmp_tuple(coords + t->order[j - 1] * d, coords + t->order[j] * d, d) == 0) {
            free(t->order); free(t); return NULL;
        }
    }
    *status = ORA_OK;
    return t;
}

void ora_tensor_free(ora_tensor* t)
{
    if (!t) return;
    free(t->order);
    free(t);
}

/* Binary search: position of the nonzero with coordinates idx, or -1. */
int64_t ora_find(const ora_tensor* t, const int64_t* idx)
{
    int64_t lo = 0, hi = t->nnz; /* search in order[lo, hi) */
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        int c = ora_cmp_tuple(t->coords + t->order[mid] * t->d, idx, t->d);
        if (c == 0) return t->order[mid];
        if (c < 0) lo = mid + 1; else hi = mid;
    }
    return -1;
}

/* M = prod_k I_k, exact in unsigned 64-bit arithmetic (tensors of up to
 * 2^64 - 1 cells). */
static uint64_t ora_cell_count_u(int d, const int64_t* dims)
{
    uint64_t M = 1;
    for (int k = 0; k < d; ++k) M *= (uint64_t)dims[k];
    return M;
}

static double ora_cell_count(int d, const int64_t* dims)
{
    return (double)ora_cell_count_u(d, dims);
}

/* Stratified sampling (Sec. 3.1.1): p nonzeros drawn uniformly with
 * replacement from the N stored entries, weight N/p; then q zeros, each the
 * first candidate cell (uniform over all M cells) that is not a stored
 * nonzero, weight (M-N)/q.  With semi != 0 the search is skipped
 * (semi-stratified sampling): the first candidate is taken as is.
 * Output order: the p nonzero samples, then the q zero samples.
 * Returns ORA_ERR_SAMPLING if some zero sample exhausts max_attempts. */
int ora_sample_stratified(const ora_tensor* t, int64_t p, int64_t q, uint64_t seed, uint64_t step,
                          uint64_t client, int64_t max_attempts, int semi,
                          int64_t* coords_out, double* x_out, double* w_out)
{
    const int d = t->d;
    const int64_t N = t->nnz;
    const uint64_t M = ora_cell_count_u(d, t->dims);
    if (p < 0 || q < 0 || (p > 0 && N == 0) || (q > 0 && !semi && (uint64_t)N >= M)) return ORA_ERR_ARG;
    const double w_nz = p > 0 ? (double)N / (double)p : 0.0;
    const double w_z = q > 0 ? (double)(M - (uint64_t)N) / (double)q : 0.0;
    uint64_t key[2] = {seed, client};
    for (int64_t s = 0; s < p; ++s) {
        uint64_t ctr[4] = {(uint64_t)s, step, ORA_STREAM_NONZERO, 0};
        uint64_t out[4];
        ora_philox4x64_10(ctr, key, out);
        int64_t j = (int64_t)ora_range(out[0], (uint64_t)N);
        for (int k = 0; k < d; ++k) coords_out[s * d + k] = t->coords[j * d + k];
        x_out[s] = t->vals[j];
        w_out[s] = w_nz;
    }
    for (int64_t s = 0; s < q; ++s) {
        int64_t* idx = coords_out + (p + s) * d;
        int found_zero = 0;
        for (int64_t a = 0; a < max_attempts; ++a) {
            ora_draw_cell(d, t->dims, seed, client, (uint64_t)s, step, ORA_STREAM_ZERO, (uint64_t)a, idx);
            if (semi || ora_find(t, idx) < 0) { found_zero = 1; break; }
        }
        if (!found_zero) return ORA_ERR_SAMPLING;
        x_out[p + s] = 0.0;
        w_out[p + s] = w_z;
    }
    return ORA_OK;
}

/* Uniform sampling of a dense tensor (the "several sampling algorithms" of
 * Sec. 3.1.1; reading: s cells uniform over all M cells with replacement,
 * weight M/s, x read from the row-major dense array). */
int ora_sample_uniform(int d, const int64_t* dims, const double* dense, int64_t s_count,
                       uint64_t seed, uint64_t step, uint64_t client,
                       int64_t* coords_out, double* x_out, double* w_out)
{
    if (d < 1 || d > 8 || s_count < 0) return ORA_ERR_ARG;
    const double w = s_count > 0 ? ora_cell_count(d, dims) / (double)s_count : 0.0;
    for (int64_t s = 0; s < s_count; ++s) {
        int64_t* idx = coords_out + s * d;
        ora_draw_cell(d, dims, seed, client, (uint64_t)s, step, ORA_STREAM_UNIFORM, 0, idx);
        int64_t lin = 0;
        for (int k = 0; k < d; ++k) lin = lin * dims[k] + idx[k];
        x_out[s] = dense[lin];
        w_out[s] = w;
    }
    return ORA_OK;
}

/* ------------------------------------------------------------------------ */
/* Losses.  The paper names Poisson (count data) and Gaussian losses and     */
/* binary data but prints no formula; each loss below is the negative log-  */
/* likelihood of its distribution with terms depending on x alone dropped.  */
/*   0 Gaussian:         f = (m - x)^2 / 2,            f' = m - x            */
/*   1 Poisson (ident.): f = m - x log(m + 1e-10),     f' = 1 - x/(m + 1e-10)*/
/*   2 Bernoulli-logit:  f = log(1 + e^m) - x m,       f' = 1/(1+e^-m) - x   */
/* ------------------------------------------------------------------------ */

enum { ORA_LOSS_GAUSSIAN = 0, ORA_LOSS_POISSON = 1, ORA_LOSS_BERNOULLI_LOGIT = 2 };
#define ORA_POISSON_EPS 1e-10

double ora_f(int loss, double x, double m)
{
    switch (loss) {
    case ORA_LOSS_GAUSSIAN: return 0.5 * (m - x) * (m - x);
    case ORA_LOSS_POISSON: return m - x * log(m + ORA_POISSON_EPS);
    case ORA_LOSS_BERNOULLI_LOGIT: {
        /* log(1 + e^m) written without overflow */
        double softplus = (m > 0 ? m : 0.0) + log1p(exp(-fabs(m)));
        return softplus - x * m;
    }
    default: return NAN;
    }
}

double ora_df(int loss, double x, double m)
{
    switch (loss) {
    case ORA_LOSS_GAUSSIAN: return m - x;
    case ORA_LOSS_POISSON: return 1.0 - x / (m + ORA_POISSON_EPS);
    case ORA_LOSS_BERNOULLI_LOGIT: {
        double sig;
        if (m >= 0) sig = 1.0 / (1.0 + exp(-m));
        else { double e = exp(m); sig = e / (1.0 + e); }
        return sig - x;
    }
    default: return NAN;
    }
}

/* ------------------------------------------------------------------------ */
/* Kruskal model entry (eq. cp, elementwise): m = sum_r prod_k A_k[i_k, r]. */
/* ------------------------------------------------------------------------ */

static void ora_rowoff(int d, const int64_t* dims, int64_t* rowoff)
{
    rowoff[0] = 0;
    for (int k = 1; k <= d; ++k) rowoff[k] = rowoff[k - 1] + dims[k - 1];
}

double ora_model_value(int d, const int64_t* dims, int R, const double* A, const int64_t* idx)
{
    int64_t rowoff[9];
    ora_rowoff(d, dims, rowoff);
    double m = 0.0;
    for (int r = 0; r < R; ++r) {
        double prod = 1.0;
        for (int k = 0; k < d; ++k) prod *= A[(rowoff[k] + idx[k]) * R + r];
        m += prod;
    }
    return m;
}

/* Sampled loss and gradient (eq. gcp-gradient with Y replaced by the sampled
 * tensor, Sec. 3.1.1-3.1.2), serial MTTKRP over the sample list:
 *   y_s = w_s f'(x_s, m_s)
 *   G_k[i_k(s), r] += y_s prod_{n != k} A_n[i_n(s), r]   for every mode k
 *   F += w_s f(x_s, m_s)
 * Samples s < n_semi are the nonzero samples of semi-stratified sampling and
 * use f'(x,m) - f'(0,m) and f(x,m) - f(0,m) instead.  G (sum_k I_k x R) is
 * overwritten.  Repeated samples are simply summed as separate entries. */
void ora_loss_grad(int d, const int64_t* dims, int R, const double* A, int64_t n,
                   const int64_t* coords, const double* x, const double* w, int loss,
                   int64_t n_semi, double* G, double* F)
{
    int64_t rowoff[9];
    ora_rowoff(d, dims, rowoff);
    memset(G, 0, sizeof(double) * (size_t)(rowoff[d] * R));
    double Fsum = 0.0;
    for (int64_t s = 0; s < n; ++s) {
        const int64_t* idx = coords + s * d;
        double m = ora_model_value(d, dims, R, A, idx);
        double y, l;
        if (s < n_semi) {
            y = w[s] * (ora_df(loss, x[s], m) - ora_df(loss, 0.0, m));
            l = w[s] * (ora_f(loss, x[s], m) - ora_f(loss, 0.0, m));
        } else {
            y = w[s] * ora_df(loss, x[s], m);
            l = w[s] * ora_f(loss, x[s], m);
        }
        Fsum += l;
        for (int k = 0; k < d; ++k) {
            double* g = G + (rowoff[k] + idx[k]) * R;
            for (int r = 0; r < R; ++r) {
                double prod = y;
                for (int nn = 0; nn < d; ++nn)
                    if (nn != k) prod *= A[(rowoff[nn] + idx[nn]) * R + r];
                g[r] += prod;
            }
        }
    }
    if (F) *F = Fsum;
}

/* The two steps of the non-fused sampled gradient (Sec. 3.1.2), written out
 * on their own: the derivative values of the sampled tensor,
 *   y_s = w_s f'(x_s, m_s)   (s < n_semi: w_s (f'(x_s, m_s) - f'(0, m_s))),
 * and the sampled MTTKRP of a given sampled tensor (coords, y),
 *   G_k[i_k(s), r] += y_s prod_{j != k} A_j[i_j(s), r]   (G overwritten). */
void ora_sample_derivatives(int d, const int64_t* dims, int R, const double* A, int64_t n, const int64_t* coords,
                            const double* x, const double* w, int loss, int64_t n_semi, double* y)
{
    for (int64_t s = 0; s < n; ++s) {
        const double m = ora_model_value(d, dims, R, A, coords + s * d);
        y[s] = w[s] * ora_df(loss, x[s], m);
        if (s < n_semi) y[s] = w[s] * (ora_df(loss, x[s], m) - ora_df(loss, 0.0, m));
    }
}

void ora_mttkrp(int d, const int64_t* dims, int R, const double* A, int64_t n, const int64_t* coords,
                const double* y, double* G)
{
    int64_t rowoff[9];
    ora_rowoff(d, dims, rowoff);
    memset(G, 0, sizeof(double) * (size_t)(rowoff[d] * R));
    for (int64_t s = 0; s < n; ++s) {
        const int64_t* idx = coords + s * d;
        for (int k = 0; k < d; ++k) {
            double* g = G + (rowoff[k] + idx[k]) * R;
            for (int r = 0; r < R; ++r) {
                double prod = y[s];
                for (int j = 0; j < d; ++j)
                    if (j != k) prod *= A[(rowoff[j] + idx[j]) * R + r];
                g[r] += prod;
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Rounding-error bound of a sampled gradient computed in a floating-point   */
/* format with unit roundoff u (2^-24 for binary32, 2^-53 for binary64),     */
/* element by element, for ANY order of its sums (lane-parallel model        */
/* values, atomics, per-workgroup partial sums), against the exact gradient  */
/* of the same samples and factors.  It rests on the standard model          */
/* fl(a op b) = (a op b)(1 + t), |t| <= u, and gamma_n = n u / (1 - n u)      */
/* (Higham, "Accuracy and Stability of Numerical Algorithms", 2nd ed.,       */
/* Sec. 2.2 and 3.1): a product of n + 1 factors has relative error at most  */
/* gamma_n, and a sum of terms added in any tree of depth n has absolute     */
/* error at most gamma_n times the sum of their magnitudes.                  */
/*                                                                          */
/* Per sample s, with P_r = prod_k |A_k[i_k, r]| and mabs = sum_r P_r:        */
/*   |m^ - m| <= dm = gamma_{d+R} mabs            (d - 1 products, R terms)   */
/*   |f'^ - f'| <= e_f  from dm and the rounding of f' itself (per loss       */
/*                     below; exp is allowed 4u, a correctly rounded         */
/*                     division u),                                          */
/*   |y^ - y| <= e_y = |w| e_f + 3u |w| (|f'| + e_f)   (w rounded to the      */
/*                     format, one product, the device scale factor),        */
/* and for every mode k and column r, with Q = prod_{n != k} |A_n[i_n, r]|:   */
/*   yerr[k, i_k, r]   += e_y Q                                              */
/*   abssum[k, i_k, r] += |y| Q                                              */
/*   count[k, i_k]     += 1.                                                 */
/* The caller combines them as                                               */
/*   |G^ - G| <= yerr + (gamma_d + gamma_{count - 1}) abssum                 */
/* (d multiplications per contribution, count - 1 additions in any order).   */
/* Samples s < n_semi are semi-stratified nonzeros with y = w (f'(x, m) -    */
/* f'(0, m)).  A bound is +inf where a loss is not Lipschitz enough near m   */
/* for the estimate to hold (a Poisson m + eps within dm of zero).           */
/* ------------------------------------------------------------------------ */

static double ora_gamma(double n, double u)
{
    return n * u / (1.0 - n * u);
}

/* Bound on |f'^(x, m^) - f'(x, m)| given |m^ - m| <= dm. */
static double ora_df_err(int loss, double x, double m, double dm, double u)
{
    switch (loss) {
    case ORA_LOSS_GAUSSIAN: {             /* fl(m^ - x) */
        double df = m - x;
        return dm + u * (fabs(df) + dm);
    }
    case ORA_LOSS_POISSON: {              /* fl(1 - fl(x / fl(m^ + eps))) */
        double den = m + ORA_POISSON_EPS;
        double eden = dm + u * (fabs(den) + dm);
        if (eden >= 0.5 * fabs(den)) return INFINITY;
        double q = x / den;
        double eq = fabs(q) * eden / (fabs(den) - eden) + u * fabs(q) * fabs(den) / (fabs(den) - eden);
        return eq + u * (fabs(1.0 - q) + eq);
    }
    case ORA_LOSS_BERNOULLI_LOGIT: {      /* sigmoid(m^) - x, sigmoid via exp */
        double sig;
        if (m >= 0) sig = 1.0 / (1.0 + exp(-m));
        else { double e = exp(m); sig = e / (1.0 + e); }
        double es = 0.25 * dm + 6.0 * u * sig;
        return es + u * (fabs(sig - x) + es);
    }
    default: return INFINITY;
    }
}

void ora_loss_grad_bound(int d, const int64_t* dims, int R, const double* A, int64_t n,
                         const int64_t* coords, const double* x, const double* w, int loss,
                         int64_t n_semi, double u, double* abssum, double* yerr, int64_t* count)
{
    int64_t rowoff[9];
    ora_rowoff(d, dims, rowoff);
    memset(abssum, 0, sizeof(double) * (size_t)(rowoff[d] * R));
    memset(yerr, 0, sizeof(double) * (size_t)(rowoff[d] * R));
    memset(count, 0, sizeof(int64_t) * (size_t)rowoff[d]);
    for (int64_t s = 0; s < n; ++s) {
        const int64_t* idx = coords + s * d;
        double m = ora_model_value(d, dims, R, A, idx);
        double mabs = 0.0;
        for (int r = 0; r < R; ++r) {
            double prod = 1.0;
            for (int k = 0; k < d; ++k) prod *= fabs(A[(rowoff[k] + idx[k]) * R + r]);
            mabs += prod;
        }
        double dm = ora_gamma((double)(d + R), u) * mabs;
        double aw = fabs(w[s]);
        double y, ey;
        if (s < n_semi) {
            double d1 = ora_df(loss, x[s], m), d0 = ora_df(loss, 0.0, m);
            double e1 = ora_df_err(loss, x[s], m, dm, u), e0 = ora_df_err(loss, 0.0, m, dm, u);
            y = w[s] * (d1 - d0);
            ey = aw * (e1 + e0) + 3.0 * u * aw * (fabs(d1) + e1 + fabs(d0) + e0) + 2.0 * u * fabs(y);
        } else {
            double df = ora_df(loss, x[s], m);
            double ef = ora_df_err(loss, x[s], m, dm, u);
            y = w[s] * df;
            ey = aw * ef + 3.0 * u * aw * (fabs(df) + ef);
        }
        for (int k = 0; k < d; ++k) {
            const int64_t row = rowoff[k] + idx[k];
            count[row] += 1;
            for (int r = 0; r < R; ++r) {
                double q = 1.0;
                for (int nn = 0; nn < d; ++nn)
                    if (nn != k) q *= fabs(A[(rowoff[nn] + idx[nn]) * R + r]);
                abssum[row * R + r] += fabs(y) * q;
                yerr[row * R + r] += ey * q;
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Adam update (Alg. adam-update), over the one contiguous parameter vector  */
/* (Sec. 3.1.3).  t >= 1 counts the updates of this model; epsilon sits      */
/* inside the square root as the paper writes it; l is the lower bound.     */
/* ------------------------------------------------------------------------ */

void ora_adam(int64_t n, double* A, const double* G, double* B, double* C, int64_t t,
              double lr, double beta1, double beta2, double eps, double lower)
{
    double c1 = 1.0 - pow(beta1, (double)t);
    double c2 = 1.0 - pow(beta2, (double)t);
    for (int64_t i = 0; i < n; ++i) {
        B[i] = beta1 * B[i] + (1.0 - beta1) * G[i];
        C[i] = beta2 * C[i] + (1.0 - beta2) * G[i] * G[i];
        double bhat = B[i] / c1;
        double chat = C[i] / c2;
        A[i] = fmax(A[i] - lr * (bhat / sqrt(chat + eps)), lower);
    }
}

/* ------------------------------------------------------------------------ */
/* Timing-only parallel step, for the CPU baseline of the benchmark (not a   */
/* checker: the parity tests use the serial functions above).  One           */
/* synchronous GCP-SGD/Adam iteration -- stratified samples, sampled         */
/* gradient, Adam -- with the paper's CPU strategy for the MTTKRP (Sec.      */
/* 3.1.2, thread privatization): OpenMP threads split the samples, each      */
/* accumulates into its own copy of G, and the copies are summed.  Same      */
/* samples and arithmetic as the serial path; only the order of the          */
/* gradient's additions differs.                                             */
/*   coords_ws [(p+q) x d], x_ws, w_ws [p+q]: sample workspace;              */
/*   G_priv [nthreads x rows x R], G [rows x R]: gradient workspace.         */
/* Returns ORA_OK, ORA_ERR_ARG or ORA_ERR_SAMPLING; *threads_used gets the   */
/* size of the thread team.                                                  */
/* ------------------------------------------------------------------------ */
#ifdef _OPENMP
#include <omp.h>
#endif

int ora_omp_sgd_step(const ora_tensor* t, int R, double* A, double* B, double* C, int64_t adam_t,
                     int loss, int64_t p, int64_t q, uint64_t seed, uint64_t step, int64_t max_attempts,
                     double lr, double beta1, double beta2, double eps, double lower, int nthreads,
                     int64_t* coords_ws, double* x_ws, double* w_ws, double* G_priv, double* G,
                     int* threads_used)
{
    const int d = t->d;
    const int64_t N = t->nnz;
    const uint64_t M = ora_cell_count_u(d, t->dims);
    if (p < 0 || q < 0 || (p > 0 && N == 0) || (q > 0 && (uint64_t)N >= M) || nthreads < 1) return ORA_ERR_ARG;
    const double w_nz = p > 0 ? (double)N / (double)p : 0.0;
    const double w_z = q > 0 ? (double)(M - (uint64_t)N) / (double)q : 0.0;
    const int64_t n = p + q;
    int64_t rowoff[9];
    ora_rowoff(d, t->dims, rowoff);
    const int64_t elems = rowoff[d] * R;
    const double c1 = 1.0 - pow(beta1, (double)adam_t);
    const double c2 = 1.0 - pow(beta2, (double)adam_t);
    int status = ORA_OK;
    int team = 1;
    #pragma omp parallel num_threads(nthreads)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
        #pragma omp single
        team = omp_get_num_threads();
#endif
        const uint64_t key[2] = {seed, 0};
        #pragma omp for schedule(static)
        for (int64_t s = 0; s < p; ++s) {
            uint64_t ctr[4] = {(uint64_t)s, step, ORA_STREAM_NONZERO, 0};
            uint64_t out[4];
            ora_philox4x64_10(ctr, key, out);
            const int64_t j = (int64_t)ora_range(out[0], (uint64_t)N);
            for (int k = 0; k < d; ++k) coords_ws[s * d + k] = t->coords[j * d + k];
            x_ws[s] = t->vals[j];
            w_ws[s] = w_nz;
        }
        #pragma omp for schedule(dynamic, 1024)
        for (int64_t s = 0; s < q; ++s) {
            int64_t* idx = coords_ws + (p + s) * d;
            int found = 0;
            for (int64_t a = 0; a < max_attempts; ++a) {
                ora_draw_cell(d, t->dims, seed, 0, (uint64_t)s, step, ORA_STREAM_ZERO, (uint64_t)a, idx);
                if (ora_find(t, idx) < 0) { found = 1; break; }
            }
            if (!found) {
                #pragma omp atomic write
                status = ORA_ERR_SAMPLING;
            }
            x_ws[p + s] = 0.0;
            w_ws[p + s] = w_z;
        }
        double* Gt = G_priv + (int64_t)tid * elems;
        memset(Gt, 0, sizeof(double) * (size_t)elems);
        #pragma omp for schedule(static)
        for (int64_t s = 0; s < n; ++s) {
            const int64_t* idx = coords_ws + s * d;
            const double m = ora_model_value(d, t->dims, R, A, idx);
            const double y = w_ws[s] * ora_df(loss, x_ws[s], m);
            for (int k = 0; k < d; ++k) {
                double* g = Gt + (rowoff[k] + idx[k]) * R;
                for (int r = 0; r < R; ++r) {
                    double prod = y;
                    for (int nn = 0; nn < d; ++nn)
                        if (nn != k) prod *= A[(rowoff[nn] + idx[nn]) * R + r];
                    g[r] += prod;
                }
            }
        }
        #pragma omp for schedule(static)
        for (int64_t e = 0; e < elems; ++e) {
            double g = 0.0;
            for (int th = 0; th < team; ++th) g += G_priv[(int64_t)th * elems + e];
            G[e] = g;
            B[e] = beta1 * B[e] + (1.0 - beta1) * g;
            C[e] = beta2 * C[e] + (1.0 - beta2) * g * g;
            A[e] = fmax(A[e] - lr * ((B[e] / c1) / sqrt(C[e] / c2 + eps)), lower);
        }
    }
    *threads_used = team;
    return status;
}
