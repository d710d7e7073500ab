/*
 * FP64 CPU oracle for P-Tucker's row-wise ALS (Oh, Park, Sael, Kang,
 * "Scalable Tucker Factorization for Sparse Tensors - Algorithms and
 * Discoveries", arXiv 1710.02261).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product calls, links or loads this
 * file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do. It shares no code, header, table or constant with the GPU
 * library: every quantity is computed from its definition with plain loops in
 * double precision, in the order the paper states it, with no blocking,
 * fusion or re-association.
 *
 * Conventions: indices are 0-based (the paper counts from 1); the core G is
 * stored in C order (last mode fastest); factor A^(n) is row-major I_n x J_n;
 * the observed set is structure-of-arrays idx[n*nnz + e] with values val[e].
 *
 * Threads: the rows of one mode are independent (Sec. 3.2), so the row
 * updates may run on several OpenMP threads, rows dealt dynamically as in
 * the paper's Sec. 3.4; each row is computed by one thread in the same order
 * whatever the thread count, so results do not depend on it. Per-entry
 * residuals are formed in parallel and summed in entry order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_MAX_ORDER 16
/* rows with at least this many entries form their deltas on all threads */
#define ORA_HEAVY_ROW 4096

/* Number of cells of the core, prod_n J_n. */
static int64_t ora_core_cells(int N, const int32_t *J)
{
    int64_t s = 1;
    for (int n = 0; n < N; ++n) s *= J[n];
    return s;
}

/* Threads for the row updates and residuals (1 without OpenMP). */
int ora_set_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
    return omp_get_max_threads();
#else
    (void)t;
    return 1;
#endif
}

/* Advance a core-cell multi-index in C order (last mode fastest). */
static void ora_next_cell(int N, const int32_t *J, int *beta)
{
    for (int k = N - 1; k >= 0; --k) {
        if (++beta[k] < J[k]) return;
        beta[k] = 0;
    }
}

/*
 * delta^(n)_alpha (Sec. 3.2, eq. "delta"): for every core cell beta whose
 * n-th index is j, add G_beta times the product over k != n of a^(k)_{i_k j_k}.
 * rows[k] points at row i_k of A^(k); rows[n] is not read. This is the
 * plain form of Alg. 3: N-1 multiplications per (entry, cell) pair.
 */
void ora_delta(int N, const int32_t *J, const double *G,
               const double *const *rows, int n, double *out)
{
    int beta[ORA_MAX_ORDER] = {0};
    int64_t S = ora_core_cells(N, J);
    for (int j = 0; j < J[n]; ++j) out[j] = 0.0;
    for (int64_t s = 0; s < S; ++s) {
        double p = G[s];
        for (int k = 0; k < N; ++k)
            if (k != n) p *= rows[k][beta[k]];
        out[beta[n]] += p;
        ora_next_cell(N, J, beta);
    }
}

/* Reconstruction of one entry (Sec. 2.2, eq. "recon2"). */
double ora_predict_one(int N, const int32_t *J, const double *G,
                       const double *const *rows)
{
    int beta[ORA_MAX_ORDER] = {0};
    int64_t S = ora_core_cells(N, J);
    double x = 0.0;
    for (int64_t s = 0; s < S; ++s) {
        double p = G[s];
        for (int k = 0; k < N; ++k) p *= rows[k][beta[k]];
        x += p;
        ora_next_cell(N, J, beta);
    }
    return x;
}

/* Gather the factor rows of entry e into rows[]. */
static void ora_rows_of(int N, const int32_t *J, const double *const *A,
                        const int32_t *idx, int64_t nnz, int64_t e,
                        const double **rows)
{
    for (int k = 0; k < N; ++k)
        rows[k] = A[k] + (int64_t)idx[(int64_t)k * nnz + e] * J[k];
}

/* Predictions for m cells (eq. "recon2"). */
void ora_predict(int N, const int32_t *J, const double *G,
                 const double *const *A, int64_t m, const int32_t *idx,
                 double *out)
{
    const double *rows[ORA_MAX_ORDER];
    for (int64_t e = 0; e < m; ++e) {
        ora_rows_of(N, J, A, idx, m, e, rows);
        out[e] = ora_predict_one(N, J, G, rows);
    }
}

/*
 * Sum of squared residuals over the observed set; the reconstruction error
 * of eq. "reconfull" is its square root.
 */
double ora_sse(int N, const int32_t *J, const double *G,
               const double *const *A, int64_t nnz, const int32_t *idx,
               const double *val)
{
    double *r2 = (double *)malloc(sizeof(double) * (nnz ? nnz : 1));
    if (!r2) return NAN;
    #pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < nnz; ++e) {
        const double *rows[ORA_MAX_ORDER];
        ora_rows_of(N, J, A, idx, nnz, e, rows);
        double r = val[e] - ora_predict_one(N, J, G, rows);
        r2[e] = r * r;
    }
    double sse = 0.0;
    for (int64_t e = 0; e < nnz; ++e) sse += r2[e];
    free(r2);
    return sse;
}

/* Loss of eq. "TF_PARTIAL": SSE + lambda * sum_n ||A^(n)||_F^2. */
double ora_loss(int N, const int64_t *I, const int32_t *J, const double *G,
                const double *const *A, int64_t nnz, const int32_t *idx,
                const double *val, double lambda)
{
    double reg = 0.0;
    for (int n = 0; n < N; ++n)
        for (int64_t t = 0; t < I[n] * J[n]; ++t) reg += A[n][t] * A[n][t];
    return ora_sse(N, J, G, A, nnz, idx, val) + lambda * reg;
}

/*
 * Solve (B + lambda I) a = c for symmetric B by Cholesky factorisation
 * (Golub & Van Loan, Alg. 4.2.1) and two triangular solves: eq. "rowupdate"
 * written as a linear solve instead of an explicit inverse, for a B that is
 * already formed. Returns 0, or -1 if B + lambda I is not positive definite
 * in floating point. The row updates below do not use it: they take the
 * least-squares form, which needs no formed B and cannot break down.
 */
int ora_solve(int Jn, const double *B, const double *c, double lambda,
              double *a)
{
    double *L = (double *)calloc((size_t)Jn * Jn, sizeof(double));
    double *y = (double *)calloc((size_t)Jn, sizeof(double));
    if (!L || !y) { free(L); free(y); return -2; }
    int rc = 0;
    for (int i = 0; i < Jn && rc == 0; ++i) {
        for (int j = 0; j <= i; ++j) {
            double s = B[i * Jn + j] + (i == j ? lambda : 0.0);
            for (int k = 0; k < j; ++k) s -= L[i * Jn + k] * L[j * Jn + k];
            if (i == j) {
                if (!(s > 0.0)) { rc = -1; break; }
                L[i * Jn + i] = sqrt(s);
            } else {
                L[i * Jn + j] = s / L[j * Jn + j];
            }
        }
    }
    if (rc == 0) {
        for (int i = 0; i < Jn; ++i) {          /* L y = c */
            double s = c[i];
            for (int k = 0; k < i; ++k) s -= L[i * Jn + k] * y[k];
            y[i] = s / L[i * Jn + i];
        }
        for (int i = Jn - 1; i >= 0; --i) {     /* L^T a = y */
            double s = y[i];
            for (int k = i + 1; k < Jn; ++k) s -= L[k * Jn + i] * a[k];
            a[i] = s / L[i * Jn + i];
        }
    }
    free(L);
    free(y);
    return rc;
}

/*
 * The row update as the regularised least-squares problem it solves.
 *
 * eq. "rowupdate" is the normal-equation form of
 *     min_a  sum_alpha (x_alpha - a^T delta_alpha)^2 + lambda ||a||^2
 * (the loss of eq. "TF_PARTIAL" restricted to one row, Theorem 1), whose
 * normal equations are (B + lambda I) a = c with B and c of eqs. "rowB",
 * "rowC". Forming B squares the conditioning: when ||B|| * eps exceeds lambda
 * the FP64 sum B + lambda I no longer holds lambda and its Cholesky factor
 * can fail or be wrong, although the minimiser is unique. The oracle
 * therefore solves the stacked problem
 *     || [ sqrt(lambda) I ; Delta ] a - [ 0 ; x ] ||  ->  min
 * by a QR factorisation built one entry at a time with Givens rotations
 * (Golub & Van Loan, Sec. 5.1.8 and 6.5, updating R by a row): R starts as
 * sqrt(lambda) I and z as 0; each entry's row [delta^T | x] is rotated into
 * [R | z]; finally R a = z by back substitution. In exact arithmetic this is
 * the solution of eq. "rowupdate". The diagonal of R never falls below
 * sqrt(lambda), so the solve exists for every lambda > 0 and every row (an
 * empty row gives a = 0 exactly).
 */
static void ora_ls_init(int Jn, double lambda, double *R, double *z)
{
    const double s = sqrt(lambda);
    for (int p = 0; p < Jn; ++p) {
        for (int q = 0; q < Jn; ++q) R[p * Jn + q] = (p == q) ? s : 0.0;
        z[p] = 0.0;
    }
}

/* Rotate the row [d | x] into [R | z]; d is overwritten. */
static void ora_ls_add(int Jn, double *R, double *z, double *d, double x)
{
    for (int j = 0; j < Jn; ++j) {
        if (d[j] == 0.0) continue;
        const double r = hypot(R[j * Jn + j], d[j]);
        const double cs = R[j * Jn + j] / r;
        const double sn = d[j] / r;
        R[j * Jn + j] = r;
        d[j] = 0.0;
        for (int q = j + 1; q < Jn; ++q) {
            const double t = R[j * Jn + q];
            R[j * Jn + q] = cs * t + sn * d[q];
            d[q] = cs * d[q] - sn * t;
        }
        const double t = z[j];
        z[j] = cs * t + sn * x;
        x = cs * x - sn * t;
    }
}

/* R a = z (R upper triangular). Returns 0, or -1 if a is not finite. */
static int ora_ls_finish(int Jn, const double *R, const double *z, double *a)
{
    int ok = 1;
    for (int j = Jn - 1; j >= 0; --j) {
        double s = z[j];
        for (int q = j + 1; q < Jn; ++q) s -= R[j * Jn + q] * a[q];
        a[j] = s / R[j * Jn + j];
        ok = ok && isfinite(a[j]);
    }
    return ok ? 0 : -1;
}

/* The row update of eq. "rowupdate" for the entries ents[0..cnt) of row i of
   mode n, by the least-squares form above. R (J_n x J_n), z and d (J_n) are
   work arrays. Returns 0, or -1 if the result is not finite. */
static int ora_row_update_list(int N, const int32_t *J, const double *G,
                               const double *const *A, int64_t nnz,
                               const int32_t *idx, const double *val, int n,
                               const int64_t *ents, int64_t cnt, double lambda,
                               double *R, double *z, double *d, double *a)
{
    const int Jn = J[n];
    const double *rows[ORA_MAX_ORDER];
    ora_ls_init(Jn, lambda, R, z);
    for (int64_t t = 0; t < cnt; ++t) {
        const int64_t e = ents[t];
        ora_rows_of(N, J, A, idx, nnz, e, rows);
        ora_delta(N, J, G, rows, n, d);
        ora_ls_add(Jn, R, z, d, val[e]);
    }
    return ora_ls_finish(Jn, R, z, a);
}

/* The same from the matrices of eq. "rowupdate" written as a stacked
   problem: solve for the rows of a given Delta (cnt x J_n, row-major) and x. */
int ora_ls_solve(int Jn, int64_t cnt, const double *Delta, const double *x,
                 double lambda, double *a)
{
    double *R = (double *)malloc(sizeof(double) * Jn * Jn);
    double *z = (double *)malloc(sizeof(double) * Jn);
    double *d = (double *)malloc(sizeof(double) * Jn);
    if (!R || !z || !d) { free(R); free(z); free(d); return -2; }
    ora_ls_init(Jn, lambda, R, z);
    for (int64_t t = 0; t < cnt; ++t) {
        memcpy(d, Delta + t * Jn, sizeof(double) * Jn);
        ora_ls_add(Jn, R, z, d, x[t]);
    }
    int rc = ora_ls_finish(Jn, R, z, a);
    free(R); free(z); free(d);
    return rc;
}

/*
 * B^(n)_i and c^(n)_i of eqs. "rowB" and "rowC" for row i of mode n, from
 * the list of entries ents[0..cnt) whose n-th index is i.
 */
static void ora_row_system_list(int N, const int32_t *J, const double *G,
                                const double *const *A, int64_t nnz,
                                const int32_t *idx, const double *val, int n,
                                const int64_t *ents, int64_t cnt, double *B,
                                double *c)
{
    const int Jn = J[n];
    const double *rows[ORA_MAX_ORDER];
    double delta[256];
    memset(B, 0, sizeof(double) * Jn * Jn);
    memset(c, 0, sizeof(double) * Jn);
    for (int64_t t = 0; t < cnt; ++t) {
        int64_t e = ents[t];
        ora_rows_of(N, J, A, idx, nnz, e, rows);
        ora_delta(N, J, G, rows, n, delta);
        for (int p = 0; p < Jn; ++p) {
            for (int q = 0; q < Jn; ++q) B[p * Jn + q] += delta[p] * delta[q];
            c[p] += val[e] * delta[p];
        }
    }
}

/* B and c for one row, found by scanning the whole observed set. */
int ora_row_system(int N, const int32_t *J, const double *G,
                   const double *const *A, int64_t nnz, const int32_t *idx,
                   const double *val, int n, int32_t row, double *B, double *c)
{
    if (J[n] > 256) return -3;
    int64_t cnt = 0;
    for (int64_t e = 0; e < nnz; ++e)
        if (idx[(int64_t)n * nnz + e] == row) ++cnt;
    int64_t *ents = (int64_t *)malloc(sizeof(int64_t) * (cnt ? cnt : 1));
    if (!ents) return -2;
    int64_t t = 0;
    for (int64_t e = 0; e < nnz; ++e)
        if (idx[(int64_t)n * nnz + e] == row) ents[t++] = e;
    ora_row_system_list(N, J, G, A, nnz, idx, val, n, ents, cnt, B, c);
    free(ents);
    return 0;
}

/*
 * One pass of Alg. 3 for mode n (the rows of A^(n) are independent, Sec. 3.2):
 * every requested row i gets a_i = c_i (B_i + lambda I)^{-1}, evaluated by
 * the least-squares form above; a row with no observed entry gets a_i = 0.
 *
 * rows_req: nreq row ids, or NULL for all I_n rows in order. Results go to
 * out (nreq x J_n, or I_n x J_n when rows_req is NULL); A is not modified.
 * Returns the number of rows whose result is not finite (none for finite
 * inputs and lambda > 0), or a negative code on allocation failure. Rows are
 * dealt to the threads dynamically.
 */
int64_t ora_update_rows(int N, const int64_t *I, const int32_t *J,
                        const double *G, const double *const *A, int64_t nnz,
                        const int32_t *idx, const double *val, int n,
                        double lambda, int64_t nreq, const int32_t *rows_req,
                        double *out)
{
    const int Jn = J[n];
    if (Jn > 256) return -3;
    const int64_t In = I[n];
    /* group the entries by their n-th index: counting sort, stable */
    int64_t *start = (int64_t *)calloc((size_t)In + 1, sizeof(int64_t));
    int64_t *ents = (int64_t *)malloc(sizeof(int64_t) * (nnz ? nnz : 1));
    int64_t *fill = (int64_t *)calloc((size_t)In + 1, sizeof(int64_t));
    if (!start || !ents || !fill) {
        free(start); free(ents); free(fill);
        return -2;
    }
    for (int64_t e = 0; e < nnz; ++e) start[idx[(int64_t)n * nnz + e] + 1]++;
    for (int64_t i = 0; i < In; ++i) start[i + 1] += start[i];
    for (int64_t e = 0; e < nnz; ++e) {
        int32_t i = idx[(int64_t)n * nnz + e];
        ents[start[i] + fill[i]++] = e;
    }
    free(fill);
    int64_t bad = 0;
    int nomem = 0;
    const int64_t count = rows_req ? nreq : In;
    /* rows with many entries one at a time, their deltas formed by all
       threads and rotated in by one, in entry order (the same arithmetic as
       the per-row loop below) */
    {
        double *R = (double *)malloc(sizeof(double) * Jn * Jn);
        double *z = (double *)malloc(sizeof(double) * Jn);
        double *dl = NULL;
        int64_t dl_cap = 0;
        if (!R || !z) nomem = 1;
        for (int64_t r = 0; r < count && !nomem; ++r) {
            const int64_t i = rows_req ? rows_req[r] : r;
            const int64_t cnt = start[i + 1] - start[i];
            if (cnt < ORA_HEAVY_ROW) continue;
            if (cnt > dl_cap) {
                free(dl);
                dl = (double *)malloc(sizeof(double) * Jn * cnt);
                dl_cap = dl ? cnt : 0;
                if (!dl) { nomem = 1; break; }
            }
            const int64_t *re = ents + start[i];
            #pragma omp parallel for schedule(static)
            for (int64_t t = 0; t < cnt; ++t) {
                const double *rows[ORA_MAX_ORDER];
                ora_rows_of(N, J, A, idx, nnz, re[t], rows);
                ora_delta(N, J, G, rows, n, dl + t * Jn);
            }
            ora_ls_init(Jn, lambda, R, z);
            for (int64_t t = 0; t < cnt; ++t)
                ora_ls_add(Jn, R, z, dl + t * Jn, val[re[t]]);
            if (ora_ls_finish(Jn, R, z, out + r * Jn) != 0) ++bad;
        }
        free(R); free(z); free(dl);
    }
    #pragma omp parallel reduction(+:bad) reduction(|:nomem)
    {
        double *R = (double *)malloc(sizeof(double) * Jn * Jn);
        double *z = (double *)malloc(sizeof(double) * Jn);
        double *d = (double *)malloc(sizeof(double) * Jn);
        if (!R || !z || !d) nomem = 1;
        #pragma omp for schedule(dynamic, 1)
        for (int64_t r = 0; r < count; ++r) {
            if (!R || !z || !d) continue;
            const int64_t i = rows_req ? rows_req[r] : r;
            if (start[i + 1] - start[i] >= ORA_HEAVY_ROW) continue;
            if (ora_row_update_list(N, J, G, A, nnz, idx, val, n, ents + start[i],
                                    start[i + 1] - start[i], lambda, R, z, d,
                                    out + r * Jn) != 0)
                ++bad;
        }
        free(R); free(z); free(d);
    }
    free(start); free(ents);
    return nomem ? -2 : bad;
}

/* Alg. 3 for mode n, writing the new rows into A[n]. */
int64_t ora_update_mode(int N, const int64_t *I, const int32_t *J,
                        const double *G, double *const *A, int64_t nnz,
                        const int32_t *idx, const double *val, int n,
                        double lambda)
{
    double *tmp = (double *)malloc(sizeof(double) * I[n] * J[n]);
    if (!tmp) return -2;
    int64_t bad = ora_update_rows(N, I, J, G, (const double *const *)A, nnz,
                                  idx, val, n, lambda, 0, NULL, tmp);
    if (bad >= 0) memcpy(A[n], tmp, sizeof(double) * I[n] * J[n]);
    free(tmp);
    return bad;
}

/*
 * Alg. 2 without the final orthogonalisation: iters times, update A^(1..N)
 * in order (Alg. 3) and measure the error. loss_after_mode[t*N+n] receives
 * the loss of eq. "TF_PARTIAL" after mode n of iteration t, sse[t] the sum of
 * squared residuals after iteration t (either may be NULL).
 */
int64_t ora_fit(int N, const int64_t *I, const int32_t *J, const double *G,
                double *const *A, int64_t nnz, const int32_t *idx,
                const double *val, double lambda, int iters,
                double *loss_after_mode, double *sse)
{
    int64_t bad = 0;
    for (int t = 0; t < iters; ++t) {
        for (int n = 0; n < N; ++n) {
            int64_t b = ora_update_mode(N, I, J, G, A, nnz, idx, val, n, lambda);
            if (b < 0) return b;
            bad += b;
            if (loss_after_mode)
                loss_after_mode[t * N + n] =
                    ora_loss(N, I, J, G, (const double *const *)A, nnz, idx,
                             val, lambda);
        }
        if (sse)
            sse[t] = ora_sse(N, J, G, (const double *const *)A, nnz, idx, val);
    }
    return bad;
}

/*
 * Thin QR of the Im x Jn row-major matrix A by Householder reflections
 * (Golub & Van Loan, Alg. 5.2.1), with the signs chosen so that diag(R) >= 0
 * (Sec. 3.1: A^(n) = Q^(n) R^(n), Q column-orthonormal, R upper triangular).
 * On return A holds Q and R (Jn x Jn, row-major) holds R. Requires Im >= Jn.
 */
int ora_qr(int64_t Im, int Jn, double *A, double *R)
{
    if (Im < Jn) return -1;
    double *W = (double *)malloc(sizeof(double) * Im * Jn);  /* reflectors */
    double *v = (double *)malloc(sizeof(double) * Im);
    double *Q = (double *)calloc((size_t)Im * Jn, sizeof(double));
    if (!W || !v || !Q) { free(W); free(v); free(Q); return -2; }
    memcpy(W, A, sizeof(double) * Im * Jn);
    double *vs = (double *)calloc((size_t)Im * Jn, sizeof(double));
    if (!vs) { free(W); free(v); free(Q); return -2; }
    for (int k = 0; k < Jn; ++k) {
        double nx = 0.0;
        for (int64_t i = k; i < Im; ++i) nx += W[i * Jn + k] * W[i * Jn + k];
        nx = sqrt(nx);
        for (int64_t i = 0; i < Im; ++i) v[i] = 0.0;
        for (int64_t i = k; i < Im; ++i) v[i] = W[i * Jn + k];
        double alpha = (W[(int64_t)k * Jn + k] >= 0.0) ? -nx : nx;
        v[k] -= alpha;
        double nv = 0.0;
        for (int64_t i = k; i < Im; ++i) nv += v[i] * v[i];
        if (nv > 0.0) {
            nv = sqrt(nv);
            for (int64_t i = k; i < Im; ++i) v[i] /= nv;
            /* W <- (I - 2 v v^T) W on columns k.. */
            for (int j = k; j < Jn; ++j) {
                double d = 0.0;
                for (int64_t i = k; i < Im; ++i) d += v[i] * W[i * Jn + j];
                for (int64_t i = k; i < Im; ++i) W[i * Jn + j] -= 2.0 * v[i] * d;
            }
        }
        for (int64_t i = 0; i < Im; ++i) vs[i * Jn + k] = v[i];
    }
    /* Q = H_0 H_1 ... H_{Jn-1} applied to the first Jn columns of I */
    for (int j = 0; j < Jn; ++j) Q[(int64_t)j * Jn + j] = 1.0;
    for (int k = Jn - 1; k >= 0; --k) {
        for (int j = 0; j < Jn; ++j) {
            double d = 0.0;
            for (int64_t i = k; i < Im; ++i) d += vs[i * Jn + k] * Q[i * Jn + j];
            for (int64_t i = k; i < Im; ++i) Q[i * Jn + j] -= 2.0 * vs[i * Jn + k] * d;
        }
    }
    for (int i = 0; i < Jn; ++i)
        for (int j = 0; j < Jn; ++j)
            R[i * Jn + j] = (j >= i) ? W[(int64_t)i * Jn + j] : 0.0;
    for (int i = 0; i < Jn; ++i) {
        if (R[i * Jn + i] < 0.0) {
            for (int j = 0; j < Jn; ++j) R[i * Jn + j] = -R[i * Jn + j];
            for (int64_t r = 0; r < Im; ++r) Q[r * Jn + i] = -Q[r * Jn + i];
        }
    }
    memcpy(A, Q, sizeof(double) * Im * Jn);
    free(W); free(v); free(Q); free(vs);
    return 0;
}

/*
 * G <- G x_n U for a square U (J_n x J_n), with the n-mode product of
 * Sec. 2.1: (G x_n U)[.., j, ..] = sum_k G[.., k, ..] U[j, k].
 */
int ora_core_update(int N, const int32_t *J, double *G, int n, const double *U)
{
    int64_t S = ora_core_cells(N, J);
    int64_t inner = 1;
    for (int k = n + 1; k < N; ++k) inner *= J[k];
    double *T = (double *)malloc(sizeof(double) * S);
    if (!T) return -2;
    int beta[ORA_MAX_ORDER] = {0};
    for (int64_t s = 0; s < S; ++s) {
        double acc = 0.0;
        int j = beta[n];
        int64_t base = s - (int64_t)j * inner;   /* same cell with beta_n = 0 */
        for (int k = 0; k < J[n]; ++k) acc += G[base + (int64_t)k * inner] * U[j * J[n] + k];
        T[s] = acc;
        ora_next_cell(N, J, beta);
    }
    memcpy(G, T, sizeof(double) * S);
    free(T);
    return 0;
}

/*
 * Final step of Alg. 2: for n = 1..N, A^(n) = Q R, A^(n) <- Q, G <- G x_n R.
 * R_out (optional) receives the N triangular factors, each J_n x J_n, packed.
 */
int ora_orthogonalize(int N, const int64_t *I, const int32_t *J, double *G,
                      double *const *A, double *R_out)
{
    int64_t off = 0;
    for (int n = 0; n < N; ++n) {
        double *R = (double *)malloc(sizeof(double) * J[n] * J[n]);
        if (!R) return -2;
        int rc = ora_qr(I[n], J[n], A[n], R);
        if (rc == 0) rc = ora_core_update(N, J, G, n, R);
        if (rc == 0 && R_out) memcpy(R_out + off, R, sizeof(double) * J[n] * J[n]);
        off += (int64_t)J[n] * J[n];
        free(R);
        if (rc) return rc;
    }
    return 0;
}

/*
 * Fold-in of a new row of mode n from k observations with the model held
 * fixed: the row update of eq. "rowupdate" over the given entries. idx is
 * [N][k]; the n-th index array is not read.
 */
int ora_fold_in(int N, const int32_t *J, const double *G,
                const double *const *A, int n, int64_t k, const int32_t *idx,
                const double *val, double lambda, double *out)
{
    const int Jn = J[n];
    if (Jn > 256) return -3;
    double *R = (double *)malloc(sizeof(double) * Jn * Jn);
    double *z = (double *)malloc(sizeof(double) * Jn);
    double *d = (double *)malloc(sizeof(double) * Jn);
    int64_t *ents = (int64_t *)malloc(sizeof(int64_t) * (k ? k : 1));
    int32_t *ix = (int32_t *)malloc(sizeof(int32_t) * N * (k ? k : 1));
    if (!R || !z || !d || !ents || !ix) {
        free(R); free(z); free(d); free(ents); free(ix);
        return -2;
    }
    for (int64_t e = 0; e < k; ++e) ents[e] = e;
    /* the n-th index of a fold-in entry does not exist; use row 0, which
       delta never reads */
    memcpy(ix, idx, sizeof(int32_t) * N * k);
    for (int64_t e = 0; e < k; ++e) ix[(int64_t)n * k + e] = 0;
    int rc = ora_row_update_list(N, J, G, A, k, ix, val, n, ents, k, lambda, R, z,
                                 d, out);
    free(R); free(z); free(d); free(ents); free(ix);
    return rc;
}

/*
 * The Cache variant of Alg. 3 (Sec. 3.3): a table Pres with one value per
 * (entry alpha, core cell beta), Pres[alpha][beta] = G_beta times the product
 * over ALL modes k of a^(k)_{i_k beta_k}. The delta of mode n then divides
 * the n-th factor back out, Pres / a^(n)_{i_n beta_n}, and after mode n is
 * updated every value is rescaled by new / old of that same factor element.
 * Where the factor element is exactly zero the division is impossible and
 * the plain product is formed instead (for delta: G_beta times the product
 * over k != n; for the rescale: the full product with the new row), as the
 * paper prescribes for that case. Meant for small cases: |Omega| * |G|
 * doubles.
 */
static double ora_cell_product(int N, const int32_t *J, const double *G,
                               const double *const *rows, const int *beta,
                               int64_t s, int skip)
{
    double p = G[s];
    for (int k = 0; k < N; ++k)
        if (k != skip) p *= rows[k][beta[k]];
    return p;
}

/* One mode of the Cache variant: new rows of A^(n) from Pres, then the
   rescale of Pres. Each row is solved by the least-squares form of the row
   update, its entries rotated in in entry order. Returns the number of rows
   whose result is not finite, or a negative code. */
static int64_t ora_update_mode_cached(int N, const int64_t *I, const int32_t *J,
                                      const double *G, double *const *A,
                                      int64_t nnz, const int32_t *idx,
                                      const double *val, int n, double lambda,
                                      double *Pres)
{
    const int Jn = J[n];
    const int64_t In = I[n];
    const int64_t S = ora_core_cells(N, J);
    double *anew = (double *)malloc(sizeof(double) * In * Jn);
    double *R = (double *)malloc(sizeof(double) * In * Jn * Jn);
    double *z = (double *)malloc(sizeof(double) * In * Jn);
    double delta[256];
    if (!anew || !R || !z || Jn > 256) {
        free(anew); free(R); free(z);
        return Jn > 256 ? -3 : -2;
    }
    for (int64_t i = 0; i < In; ++i) ora_ls_init(Jn, lambda, R + i * Jn * Jn, z + i * Jn);
    const double *rows[ORA_MAX_ORDER];
    /* every entry's delta from Pres, rotated into its row's problem */
    for (int64_t e = 0; e < nnz; ++e) {
        ora_rows_of(N, J, (const double *const *)A, idx, nnz, e, rows);
        const int64_t i = idx[(int64_t)n * nnz + e];
        int beta[ORA_MAX_ORDER] = {0};
        for (int j = 0; j < Jn; ++j) delta[j] = 0.0;
        for (int64_t s = 0; s < S; ++s) {
            const double an = rows[n][beta[n]];
            delta[beta[n]] += an != 0.0 ? Pres[e * S + s] / an
                                        : ora_cell_product(N, J, G, rows, beta, s, n);
            ora_next_cell(N, J, beta);
        }
        ora_ls_add(Jn, R + i * Jn * Jn, z + i * Jn, delta, val[e]);
    }
    int64_t bad = 0;
    for (int64_t i = 0; i < In; ++i)
        if (ora_ls_finish(Jn, R + i * Jn * Jn, z + i * Jn, anew + i * Jn) != 0) ++bad;
    /* rescale Pres: old -> new value of the n-th factor element */
    for (int64_t e = 0; e < nnz; ++e) {
        const int64_t i = idx[(int64_t)n * nnz + e];
        ora_rows_of(N, J, (const double *const *)A, idx, nnz, e, rows);
        const double *old_row = rows[n];
        rows[n] = anew + i * Jn;
        int beta[ORA_MAX_ORDER] = {0};
        for (int64_t s = 0; s < S; ++s) {
            const double ao = old_row[beta[n]];
            Pres[e * S + s] = ao != 0.0 ? Pres[e * S + s] / ao * rows[n][beta[n]]
                                        : ora_cell_product(N, J, G, rows, beta, s, -1);
            ora_next_cell(N, J, beta);
        }
    }
    memcpy(A[n], anew, sizeof(double) * In * Jn);
    free(anew); free(R); free(z);
    return bad;
}

/* Alg. 2 iterations with the Cache variant of Alg. 3: Pres is built once
   (Alg. 3, before the mode loop) and rescaled after every mode; sse[t] is
   the sum of squared residuals after iteration t (may be NULL). */
int64_t ora_fit_cached(int N, const int64_t *I, const int32_t *J, const double *G,
                       double *const *A, int64_t nnz, const int32_t *idx,
                       const double *val, double lambda, int iters, double *sse)
{
    const int64_t S = ora_core_cells(N, J);
    double *Pres = (double *)malloc(sizeof(double) * (nnz ? nnz : 1) * S);
    if (!Pres) return -2;
    const double *rows[ORA_MAX_ORDER];
    for (int64_t e = 0; e < nnz; ++e) {
        ora_rows_of(N, J, (const double *const *)A, idx, nnz, e, rows);
        int beta[ORA_MAX_ORDER] = {0};
        for (int64_t s = 0; s < S; ++s) {
            Pres[e * S + s] = ora_cell_product(N, J, G, rows, beta, s, -1);
            ora_next_cell(N, J, beta);
        }
    }
    int64_t bad = 0;
    for (int t = 0; t < iters; ++t) {
        for (int n = 0; n < N; ++n) {
            int64_t b = ora_update_mode_cached(N, I, J, G, A, nnz, idx, val, n,
                                               lambda, Pres);
            if (b < 0) { free(Pres); return b; }
            bad += b;
        }
        if (sse)
            sse[t] = ora_sse(N, J, G, (const double *const *)A, nnz, idx, val);
    }
    free(Pres);
    return bad;
}

/*
 * The Approx variant (Alg. 4, Sec. 3.3): the partial reconstruction error of
 * every core cell beta (eq. "recon_partial", first form): the sum over the
 * observed entries of the squared residual of the model minus the squared
 * residual of the model without the cell's term,
 *     R(beta) = sum_alpha (x - xhat)^2 - (x - (xhat - t))^2,
 *     t = G_beta prod_n a^(n)_{i_n beta_n}.
 * A high R(beta) means that removing the cell lowers the error.
 */
int ora_partial_error(int N, const int32_t *J, const double *G,
                      const double *const *A, int64_t nnz, const int32_t *idx,
                      const double *val, double *R)
{
    const int64_t S = ora_core_cells(N, J);
    double *xhat = (double *)malloc(sizeof(double) * (nnz ? nnz : 1));
    if (!xhat) return -2;
    const double *rows[ORA_MAX_ORDER];
    for (int64_t e = 0; e < nnz; ++e) {
        ora_rows_of(N, J, A, idx, nnz, e, rows);
        xhat[e] = ora_predict_one(N, J, G, rows);
    }
    int beta[ORA_MAX_ORDER] = {0};
    for (int64_t s = 0; s < S; ++s) {
        double r = 0.0;
        for (int64_t e = 0; e < nnz; ++e) {
            ora_rows_of(N, J, A, idx, nnz, e, rows);
            const double t = ora_cell_product(N, J, G, rows, beta, s, -1);
            const double with = val[e] - xhat[e];
            const double without = val[e] - (xhat[e] - t);
            r += with * with - without * without;
        }
        R[s] = r;
        ora_next_cell(N, J, beta);
    }
    free(xhat);
    return 0;
}

/*
 * Alg. 4's removal: among the cells of G that are not zero (the entries of
 * the core), the floor(p * count) cells with the largest R(beta) are set to
 * zero; equal R values are taken in increasing cell order. Returns the
 * number of cells removed.
 */
static const double *ora_sort_R;
static int ora_cmp_desc(const void *pa, const void *pb)
{
    const int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    if (ora_sort_R[a] > ora_sort_R[b]) return -1;
    if (ora_sort_R[a] < ora_sort_R[b]) return 1;
    return a < b ? -1 : (a > b ? 1 : 0);
}

int64_t ora_truncate(int N, const int32_t *J, double *G, const double *R, double p)
{
    const int64_t S = ora_core_cells(N, J);
    int64_t *cells = (int64_t *)malloc(sizeof(int64_t) * S);
    if (!cells) return -2;
    int64_t nz = 0;
    for (int64_t s = 0; s < S; ++s)
        if (G[s] != 0.0) cells[nz++] = s;
    const int64_t k = (int64_t)floor(p * (double)nz);
    ora_sort_R = R;
    qsort(cells, (size_t)nz, sizeof(int64_t), ora_cmp_desc);
    for (int64_t t = 0; t < k; ++t) G[cells[t]] = 0.0;
    free(cells);
    return k;
}

/* Alg. 2 with the Approx variant: each iteration updates the factors (Alg. 3),
   measures the error (sse[t], before the removal) and removes cells of G by
   Alg. 4 (core_nnz[t] = non-zero cells left). G is updated in place. */
int64_t ora_fit_approx(int N, const int64_t *I, const int32_t *J, double *G,
                       double *const *A, int64_t nnz, const int32_t *idx,
                       const double *val, double lambda, int iters, double p,
                       double *sse, int64_t *core_nnz)
{
    const int64_t S = ora_core_cells(N, J);
    double *R = (double *)malloc(sizeof(double) * S);
    if (!R) return -2;
    int64_t bad = 0;
    for (int t = 0; t < iters; ++t) {
        for (int n = 0; n < N; ++n) {
            int64_t b = ora_update_mode(N, I, J, G, A, nnz, idx, val, n, lambda);
            if (b < 0) { free(R); return b; }
            bad += b;
        }
        if (sse) sse[t] = ora_sse(N, J, G, (const double *const *)A, nnz, idx, val);
        int rc = ora_partial_error(N, J, G, (const double *const *)A, nnz, idx, val, R);
        if (rc) { free(R); return rc; }
        if (ora_truncate(N, J, G, R, p) < 0) { free(R); return -2; }
        if (core_nnz) {
            int64_t c = 0;
            for (int64_t s = 0; s < S; ++s) c += G[s] != 0.0;
            core_nnz[t] = c;
        }
    }
    free(R);
    return bad;
}
