/*
 * CPU reference ("oracle") for the sparse CG path — TEST INFRASTRUCTURE ONLY.
 *
 * Plain, sequential, float64 code written to be checked by eye against its
 * definitions.  Only the test suite, the package smoke check and the CPU
 * baseline leg of the benchmark may load it; the GPU library never calls it
 * and shares no code with it.  Build with -ffp-contract=off so that every
 * `a*b + c` below is two roundings unless fma() is written out.
 *
 * What follows the paper and what is a stated reading of it:
 *  - CSR storage (Section 2.3): values row-wise in AA, their column numbers in
 *    JA, IA(i) the start of row i, row i spanning IA(i)..IA(i+1)-1.  The paper
 *    counts from 1; this code takes 0-based arrays.
 *  - SpMV, vector addition, element-wise product, dot product (Section 5.2,
 *    Tables "SpMV with CSR format", "Addition of vectors", "Element wise
 *    product", "Dot product"): their plain definitions.  The addition table is
 *    labelled as a daxpy, so both z = x + y and y = alpha*x + y (one fused
 *    rounding, fma) are provided.
 *  - Classical conjugate gradient without preconditioner (Section 5.3, which
 *    cites Saad's textbook for the method): the Hestenes-Stiefel recurrences,
 *    x0 given, stop when ||r_k||_2 <= rtol * ||b||_2 on the recursively
 *    updated residual.  The paper states neither tolerance nor x0.
 *  - Jacobi preconditioning (not used in the paper) and mixed-precision
 *    iterative refinement (the Anzt-Heuveline-Rocker reference cited beside
 *    CG in Section 5.3) extend the same recurrences.
 * Dots inside the solvers are compensated (Kahan) sums in index order.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Timing build only (gcc -fopenmp, used for the all-cores CPU baseline): the
 * row and element loops run in parallel, each row / element computed as
 * below; the compensated dot then sums per-thread partials.  The default
 * build (no -fopenmp) ignores these and is the sequential code as written. */
#ifdef _OPENMP
#include <omp.h>
#define ORC_PARALLEL_FOR _Pragma("omp parallel for schedule(static)")
#else
#define ORC_PARALLEL_FOR
#endif

/* Threads the timing build runs with (1 for the default build). */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

enum {
    ORC_OK = 0,
    ORC_EINVAL = -1,
    ORC_NOT_CONVERGED = -4,
    ORC_BREAKDOWN = -5,
    ORC_NONFINITE = -6,
};

/* ------------------------------------------------------------ CSR check -- */

/* Structural validity of a 0-based CSR matrix: row_ptr[0] = 0, row starts
 * non-decreasing, row_ptr[n] = nnz, columns in [0, n_cols), no column twice in
 * a row.  Returns 0 or the first offending row + 1 (negated for nnz/ptr
 * errors: -1). */
int64_t oracle_csr_check(int64_t n_rows, int64_t n_cols, int64_t nnz, const int32_t *row_ptr,
                         const int32_t *col_idx)
{
    if (n_rows < 0 || n_cols < 0 || nnz < 0) return -1;
    if (row_ptr[0] != 0 || (int64_t)row_ptr[n_rows] != nnz) return -1;
    unsigned char *seen = (unsigned char *)calloc((size_t)(n_cols > 0 ? n_cols : 1), 1);
    if (!seen) return -1;
    int64_t bad = 0;
    for (int64_t i = 0; i < n_rows && !bad; ++i) {
        if (row_ptr[i + 1] < row_ptr[i]) { bad = i + 1; break; }
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            int32_t c = col_idx[k];
            if (c < 0 || (int64_t)c >= n_cols || seen[c]) { bad = i + 1; break; }
            seen[c] = 1;
        }
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            int32_t c = col_idx[k];
            if (c >= 0 && (int64_t)c < n_cols) seen[c] = 0;
        }
    }
    free(seen);
    return bad;
}

/* ----------------------------------------------------- elementwise ops -- */

void oracle_add(int64_t n, const double *x, const double *y, double *z)
{
    ORC_PARALLEL_FOR
    for (int64_t i = 0; i < n; ++i) z[i] = x[i] + y[i];
}

void oracle_axpy(int64_t n, double alpha, const double *x, double *y)
{
    ORC_PARALLEL_FOR
    for (int64_t i = 0; i < n; ++i) y[i] = fma(alpha, x[i], y[i]);
}

void oracle_xmul(int64_t n, const double *x, const double *y, double *z)
{
    ORC_PARALLEL_FOR
    for (int64_t i = 0; i < n; ++i) z[i] = x[i] * y[i];
}

/* ------------------------------------------------------------------ dot -- */

/* Kahan-compensated sum of the rounded products x_i*y_i, in index order. */
static double kahan_dot(int64_t i0, int64_t i1, const double *x, const double *y)
{
    double s = 0.0, c = 0.0;
    for (int64_t i = i0; i < i1; ++i) {
        double t = x[i] * y[i] - c;
        double u = s + t;
        c = (u - s) - t;
        s = u;
    }
    return s;
}

double oracle_dot(int64_t n, const double *x, const double *y)
{
#ifdef _OPENMP
    /* timing build: a compensated sum per thread over contiguous index
     * ranges, the partials then added in thread order with compensation */
    enum { kMaxThreads = 1024 };
    double part[kMaxThreads];
    int nt = omp_get_max_threads();
    if (nt > kMaxThreads) nt = kMaxThreads;
#pragma omp parallel num_threads(nt)
    {
        const int t = omp_get_thread_num(), T = omp_get_num_threads();
        part[t] = kahan_dot(n * t / T, n * (t + 1) / T, x, y);
#pragma omp barrier
#pragma omp single
        nt = T;
    }
    double s = 0.0, c = 0.0;
    for (int t = 0; t < nt; ++t) {
        double v = part[t] - c;
        double u = s + v;
        c = (u - s) - v;
        s = u;
    }
    return s;
#else
    return kahan_dot(0, n, x, y);
#endif
}

/* The same compensated sum carried out entirely in binary32. */
float oracle_dot_f32(int64_t n, const float *x, const float *y)
{
    float s = 0.0f, c = 0.0f;
    for (int64_t i = 0; i < n; ++i) {
        float t = x[i] * y[i] - c;
        float u = s + t;
        c = (u - s) - t;
        s = u;
    }
    return s;
}

/* ----------------------------------------------------------------- SpMV -- */

/* y_i = sum over k in row i of val[k] * x[col_idx[k]], accumulated in k order
 * from +0.0; an empty row gives +0.0. */
void oracle_spmv(int64_t n_rows, const int32_t *row_ptr, const int32_t *col_idx, const double *val,
                 const double *x, double *y)
{
    ORC_PARALLEL_FOR
    for (int64_t i = 0; i < n_rows; ++i) {
        double s = 0.0;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) s = s + val[k] * x[col_idx[k]];
        y[i] = s;
    }
}

void oracle_spmv_f32(int64_t n_rows, const int32_t *row_ptr, const int32_t *col_idx,
                     const float *val, const float *x, float *y)
{
    for (int64_t i = 0; i < n_rows; ++i) {
        float s = 0.0f;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) s = s + val[k] * x[col_idx[k]];
        y[i] = s;
    }
}

/* ------------------------------------------------------------------- CG -- */

typedef struct {
    int32_t status;
    int32_t iters;       /* CG iterations (inner iterations summed for IR) */
    int32_t outer_iters; /* refinement steps (IR only) */
    int32_t pad;
    double relres;       /* ||r_k|| / ||b|| of the recursive residual at exit */
    double relres_true;  /* ||b - A x|| / ||b|| recomputed at exit */
} oracle_stats;

static double nrm2(int64_t n, const double *x) { return sqrt(oracle_dot(n, x, x)); }

static double true_relres(int64_t n, const int32_t *rp, const int32_t *ci, const double *val,
                          const double *b, const double *x, double bnorm)
{
    double *ax = (double *)malloc((size_t)n * sizeof(double));
    oracle_spmv(n, rp, ci, val, x, ax);
    for (int64_t i = 0; i < n; ++i) ax[i] = b[i] - ax[i];
    double r = nrm2(n, ax);
    free(ax);
    return bnorm > 0.0 ? r / bnorm : r;
}

/* Inverse diagonal for Jacobi preconditioning; returns the first row with a
 * missing or non-positive diagonal (+1), 0 if all are positive. */
int64_t oracle_inv_diag(int64_t n, const int32_t *rp, const int32_t *ci, const double *val,
                        double *dinv)
{
    for (int64_t i = 0; i < n; ++i) {
        double d = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
            if (ci[k] == i) d = val[k];
        if (!(d > 0.0)) return i + 1;
        dinv[i] = 1.0 / d;
    }
    return 0;
}

/* Conjugate gradient for A x = b, A symmetric positive definite (n x n CSR).
 *   r0 = b - A x0, z0 = M^-1 r0 (M = I, or diag(A) if jacobi), p0 = z0,
 *   rho0 = r0 . z0;
 *   for k = 0, 1, ...:
 *     q = A p_k,  alpha = rho_k / (p_k . q)
 *     x += alpha p_k,  r -= alpha q,  z = M^-1 r,  rho_{k+1} = r . z
 *     stop when ||r|| <= rtol ||b||
 *     beta = rho_{k+1} / rho_k,  p_{k+1} = z + beta p_k
 * b = 0 returns x = 0 after 0 iterations.  maxit <= 0 means n.
 * alpha_hist / beta_hist (length >= maxit, nullable) receive the coefficients
 * of every completed iteration (beta of the last one is not formed).
 * res_hist (length >= maxit + 1, nullable) receives ||r_k|| / ||b|| of the
 * recursively updated residual for k = 0 .. iters (output only: the values
 * the stopping test compares). */
int oracle_cg(int64_t n, const int32_t *rp, const int32_t *ci, const double *val,
              const double *b, double *x, double rtol, int32_t maxit, int32_t jacobi,
              oracle_stats *st, double *alpha_hist, double *beta_hist, double *res_hist)
{
    memset(st, 0, sizeof(*st));
    if (maxit <= 0) maxit = (int32_t)(n > 0x7fffffff ? 0x7fffffff : n);
    double bnorm = nrm2(n, b);
    if (!isfinite(bnorm)) { st->status = ORC_NONFINITE; return st->status; }
    if (bnorm == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        st->status = ORC_OK;
        return ORC_OK;
    }
    double *r = (double *)malloc((size_t)n * sizeof(double));
    double *p = (double *)malloc((size_t)n * sizeof(double));
    double *q = (double *)malloc((size_t)n * sizeof(double));
    double *z = jacobi ? (double *)malloc((size_t)n * sizeof(double)) : r;
    double *dinv = jacobi ? (double *)malloc((size_t)n * sizeof(double)) : NULL;
    int status = ORC_NOT_CONVERGED;
    int32_t k = 0;
    int have_r = 0;
    double rr;

    if (jacobi && oracle_inv_diag(n, rp, ci, val, dinv) != 0) { status = ORC_BREAKDOWN; goto done; }

    oracle_spmv(n, rp, ci, val, x, q);
    ORC_PARALLEL_FOR
    for (int64_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
    have_r = 1;
    if (jacobi) oracle_xmul(n, dinv, r, z);
    memcpy(p, z, (size_t)n * sizeof(double));
    double rho = oracle_dot(n, r, z);
    rr = jacobi ? oracle_dot(n, r, r) : rho;
    if (res_hist) res_hist[0] = sqrt(rr) / bnorm;
    if (!isfinite(rr)) { status = ORC_NONFINITE; goto done; }
    if (sqrt(rr) <= rtol * bnorm) { status = ORC_OK; goto done; }

    while (k < maxit) {
        oracle_spmv(n, rp, ci, val, p, q);
        double pq = oracle_dot(n, p, q);
        if (!isfinite(pq)) { status = ORC_NONFINITE; break; }
        if (!(pq > 0.0)) { status = ORC_BREAKDOWN; break; }
        double alpha = rho / pq;
        oracle_axpy(n, alpha, p, x);
        oracle_axpy(n, -alpha, q, r);
        if (jacobi) oracle_xmul(n, dinv, r, z);
        double rho_new = oracle_dot(n, r, z);
        rr = jacobi ? oracle_dot(n, r, r) : rho_new;
        if (alpha_hist) alpha_hist[k] = alpha;
        ++k;
        if (res_hist) res_hist[k] = sqrt(rr) / bnorm;
        if (!isfinite(rr) || !isfinite(rho_new)) { status = ORC_NONFINITE; break; }
        if (sqrt(rr) <= rtol * bnorm) { status = ORC_OK; break; }
        if (!(rho_new > 0.0)) { status = ORC_BREAKDOWN; break; }
        double beta = rho_new / rho;
        if (beta_hist) beta_hist[k - 1] = beta;
        rho = rho_new;
        ORC_PARALLEL_FOR
        for (int64_t i = 0; i < n; ++i) p[i] = fma(beta, p[i], z[i]);
    }

done:
    st->status = status;
    st->iters = k;
    st->relres = have_r ? nrm2(n, r) / bnorm : NAN;
    st->relres_true = true_relres(n, rp, ci, val, b, x, bnorm);
    free(r);
    free(p);
    free(q);
    if (jacobi) { free(z); free(dinv); }
    return status;
}

/* ------------------------------------------ mixed-precision refinement -- */

/* CG in binary32 for A32 d = c, d0 = 0, stopping when ||r_k|| <= tau ||c||;
 * with dinv32 (nullable) the residual is preconditioned by z = dinv32 .* r.
 * Every product, sum and dot is a float operation.  Returns the iteration
 * count; stops early (keeping the current d) when the recurrences break down
 * in binary32. */
static int32_t cg_f32(int64_t n, const int32_t *rp, const int32_t *ci, const float *val,
                      const float *dinv32, const float *c, float *d, float tau, int32_t maxit)
{
    float *r = (float *)malloc((size_t)n * sizeof(float));
    float *p = (float *)malloc((size_t)n * sizeof(float));
    float *q = (float *)malloc((size_t)n * sizeof(float));
    float *z = dinv32 ? (float *)malloc((size_t)n * sizeof(float)) : r;
    for (int64_t i = 0; i < n; ++i) {
        d[i] = 0.0f;
        r[i] = c[i];
        if (dinv32) z[i] = dinv32[i] * c[i];
        p[i] = z[i];
    }
    float rr = oracle_dot_f32(n, r, r);
    float rho = dinv32 ? oracle_dot_f32(n, r, z) : rr;
    const float stop = tau * sqrtf(rr);
    int32_t k = 0;
    while (k < maxit && sqrtf(rr) > stop) {
        oracle_spmv_f32(n, rp, ci, val, p, q);
        float pq = oracle_dot_f32(n, p, q);
        if (!(pq > 0.0f) || !isfinite(pq)) break;
        float alpha = rho / pq;
        for (int64_t i = 0; i < n; ++i) d[i] = fmaf(alpha, p[i], d[i]);
        for (int64_t i = 0; i < n; ++i) r[i] = fmaf(-alpha, q[i], r[i]);
        if (dinv32)
            for (int64_t i = 0; i < n; ++i) z[i] = dinv32[i] * r[i];
        float rho_new = dinv32 ? oracle_dot_f32(n, r, z) : oracle_dot_f32(n, r, r);
        rr = dinv32 ? oracle_dot_f32(n, r, r) : rho_new;
        ++k;
        if (!(rho_new > 0.0f) || !isfinite(rho_new)) break;
        float beta = rho_new / rho;
        rho = rho_new;
        for (int64_t i = 0; i < n; ++i) p[i] = fmaf(beta, p[i], z[i]);
    }
    free(r);
    free(p);
    free(q);
    if (dinv32) free(z);
    return k;
}

/* Iterative refinement with a binary32 inner CG:
 *   repeat: r = b - A64 x (float64); stop when ||r|| <= rtol ||b||;
 *           s = ||r||;  c = float(r / s);
 *           d = CG32(A32, c) to relative tolerance tau (d0 = 0);
 *           x += s * double(d).
 * val32 holds the values of A rounded to binary32 (same pattern as val).
 * jacobi: the inner CG is preconditioned by float(1 / a_ii). */
int oracle_mixed_ir(int64_t n, const int32_t *rp, const int32_t *ci, const double *val,
                    const float *val32, const double *b, double *x, double rtol, double tau,
                    int32_t inner_maxit, int32_t max_outer, int32_t jacobi, oracle_stats *st)
{
    memset(st, 0, sizeof(*st));
    if (inner_maxit <= 0) inner_maxit = (int32_t)(n > 0x7fffffff ? 0x7fffffff : n);
    double bnorm = nrm2(n, b);
    if (!isfinite(bnorm)) { st->status = ORC_NONFINITE; return st->status; }
    if (bnorm == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        return ORC_OK;
    }
    float *dinv32 = NULL;
    if (jacobi) {
        double *dinv = (double *)malloc((size_t)n * sizeof(double));
        if (oracle_inv_diag(n, rp, ci, val, dinv) != 0) {
            free(dinv);
            st->status = ORC_BREAKDOWN;
            return st->status;
        }
        dinv32 = (float *)malloc((size_t)n * sizeof(float));
        for (int64_t i = 0; i < n; ++i) dinv32[i] = (float)dinv[i];
        free(dinv);
    }
    double *r = (double *)malloc((size_t)n * sizeof(double));
    float *c = (float *)malloc((size_t)n * sizeof(float));
    float *d = (float *)malloc((size_t)n * sizeof(float));
    int status = ORC_NOT_CONVERGED;
    int32_t outer = 0, inner_total = 0;
    double relres = 0.0;
    for (;;) {
        oracle_spmv(n, rp, ci, val, x, r);
        for (int64_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
        double s = nrm2(n, r);
        relres = s / bnorm;
        if (!isfinite(relres)) { status = ORC_NONFINITE; break; }
        if (relres <= rtol) { status = ORC_OK; break; }
        if (outer >= max_outer) break;
        for (int64_t i = 0; i < n; ++i) c[i] = (float)(r[i] / s);
        inner_total += cg_f32(n, rp, ci, val32, dinv32, c, d, (float)tau, inner_maxit);
        for (int64_t i = 0; i < n; ++i) x[i] = fma(s, (double)d[i], x[i]);
        ++outer;
    }
    st->status = status;
    st->iters = inner_total;
    st->outer_iters = outer;
    st->relres = relres;
    st->relres_true = relres;
    free(r);
    free(c);
    free(d);
    free(dinv32);
    return status;
}

/* --------------------------- mixed precision with reliable updates -- */

/* oracle_mixed_ru: the method, iteration in binary32 (val_lp = val32). */
#define RU_T float
#define RU_NAME oracle_mixed_ru
#define RU_DOT oracle_dot_f32
#define RU_SPMV oracle_spmv_f32
#define RU_FMA fmaf
#define RU_SQRT sqrtf
#include "mixed_ru.inc"
#undef RU_T
#undef RU_NAME
#undef RU_DOT
#undef RU_SPMV
#undef RU_FMA
#undef RU_SQRT

/* oracle_mixed_ru_f64: the same steps with a float64 iteration (val_lp = val),
 * for the tests: in exact arithmetic the method is CG, so with float64
 * everywhere it must follow float64 CG. */
#define RU_T double
#define RU_NAME oracle_mixed_ru_f64
#define RU_DOT oracle_dot
#define RU_SPMV oracle_spmv
#define RU_FMA fma
#define RU_SQRT sqrt
#include "mixed_ru.inc"
#undef RU_T
#undef RU_NAME
#undef RU_DOT
#undef RU_SPMV
#undef RU_FMA
#undef RU_SQRT

/* oracle_mixed_ru_block (binary32 iteration) and oracle_mixed_ru_block_f64
 * (float64 iteration, for the tests): k right-hand sides of one matrix in
 * step, an update of one being taken by all (mixed_ru_block.inc). */
#define RU_T float
#define RUB_NAME oracle_mixed_ru_block
#define RU_DOT oracle_dot_f32
#define RU_SPMV oracle_spmv_f32
#define RU_FMA fmaf
#define RU_SQRT sqrtf
#include "mixed_ru_block.inc"
#undef RU_T
#undef RUB_NAME
#undef RU_DOT
#undef RU_SPMV
#undef RU_FMA
#undef RU_SQRT
#define RU_T double
#define RUB_NAME oracle_mixed_ru_block_f64
#define RU_DOT oracle_dot
#define RU_SPMV oracle_spmv
#define RU_FMA fma
#define RU_SQRT sqrt
#include "mixed_ru_block.inc"
#undef RU_T
#undef RUB_NAME
#undef RU_DOT
#undef RU_SPMV
#undef RU_FMA
#undef RU_SQRT
