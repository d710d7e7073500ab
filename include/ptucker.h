/*
 * ptucker.h -- C ABI of the MI355X (gfx950) row-wise sparse Tucker ALS library.
 *
 * The calls follow the problem statement of P-Tucker (Oh, Park, Sael, Kang,
 * arXiv 1710.02261): Def. "Sparse Tucker Factorization" (Sec. 2.2), the
 * inputs and outputs of Alg. 2 (Sec. 3.1) and Alg. 3 (Sec. 3.2). A user
 * hands over the observed entries as COO indices and values, the core G, the
 * factor matrices A^(n), the regularisation lambda and the ranks J_n.
 *
 * Conventions shared by every call
 *  - Indices are 0-based (the paper counts from 1).
 *  - Pointers are DEVICE pointers (memory of the device that was current when
 *    the context was created) unless the parameter name ends in "_host".
 *  - The observed set is structure-of-arrays: idx[n * nnz + e] is the mode-n
 *    index of entry e, val[e] its value (float32).
 *  - The core G is float32 in C order (J_1 x ... x J_N, last mode fastest).
 *    Factor A^(n) is float32 row-major I_n x J_n (row i is contiguous).
 *  - All device work is ordered on the HIP stream given to ptk_create. Calls
 *    that return host values synchronise that stream before returning.
 *  - Every call returns a ptk_status; no exception crosses the ABI. The text
 *    of the last failure is available from ptk_last_error(ctx).
 *  - A context is not thread-safe: one thread at a time may call into it.
 */
#ifndef PTUCKER_H
#define PTUCKER_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ptk_status {
    PTK_OK = 0,
    PTK_E_INVALID = 1,      /* bad argument or out-of-range input data      */
    PTK_E_NOMEM = 2,        /* device or host allocation failed             */
    PTK_E_UNSUPPORTED = 3,  /* shape outside what the library supports      */
    PTK_E_NOT_PD = 4,       /* a J x J system was not positive definite     */
    PTK_E_HIP = 5,          /* a HIP runtime call or kernel launch failed   */
    PTK_E_STATE = 6,        /* call order violated (e.g. no observed set)   */
    PTK_E_BUSY = 7,         /* queue full, or a wait timed out              */
    PTK_E_DIVERGED = 8      /* ptk_iterate: an error or loss not finite, or
                               the loss rose between iterations             */
} ptk_status;

typedef struct ptk_ctx ptk_ctx;

/* Arithmetic of the delta / Gram kernels (the solve and the QR are FP64). */
typedef enum ptk_precision {
    PTK_PREC_FP64_ACC = 0,  /* fp32 data, fp64 delta and Gram arithmetic    */
    PTK_PREC_FP32 = 1,      /* fp32 delta arithmetic, fp64 Gram sums        */
    PTK_PREC_BF16 = 2,      /* bf16 delta and Gram on the matrix cores with
                               fp32 accumulation; equal ranks only, (N, J) in
                               {(3,8),(3,10),(3,16),(4,8),(4,10)}           */
    PTK_PREC_BF16X3 = 3     /* as PTK_PREC_BF16 with every operand split into
                               two bf16 parts (hi + lo) and three products:
                               about 16 significant bits                    */
} ptk_precision;

typedef struct ptk_options {
    int32_t precision;      /* ptk_precision                                 */
    int32_t chunk_nnz;      /* entries per wavefront work range; 0 = auto    */
    int32_t fuse_error;     /* 1: error of ptk_iterate from the last mode's
                               row systems (sum x^2 - 2 a^T c + a^T B a per
                               row); 0: a separate pass over all entries     */
    int32_t profile;        /* 1: time every kernel launch with HIP events
                               (kernels are then launched one by one)        */
    int32_t use_graph;      /* 1: ptk_iterate replays one captured graph per
                               iteration (re-captured when lambda, options,
                               the observed set or the bound model change)   */
    int32_t pair_cache;     /* 1: per-entry partial-product cache inside
                               ptk_iterate (the Cache variant of Alg. 3 in a
                               reduced form). Modes are paired (0,1), (2,3),
                               ...: while mode 2k is updated, every entry
                               stores G contracted with all modes except 2k
                               and 2k+1 (J*J doubles), and mode 2k+1 then
                               forms its deltas from that table and the new
                               mode-2k row instead of from G. Same result up
                               to rounding. Needs equal ranks, PTK_PREC_FP64_ACC
                               or PTK_PREC_FP32, 3 <= N <= 10 and J in
                               {3,4,5,8,10,16} (else PTK_E_UNSUPPORTED),
                               and (nnz + 1) * R * 8 bytes of device
                               memory, R = J*J rounded up to even
                               (PTK_E_NOMEM from ptk_set_observed). Chosen
                               before ptk_set_observed. ptk_update_mode,
                               ptk_row_systems and fold-in never use it.      */
    double approx_rate;     /* p of the Approx variant (Alg. 4, Sec. 3.3),
                               0 <= p < 1; 0 turns it off. After the error of
                               every ptk_iterate iteration, the floor(p * nz)
                               non-zero cells of the core with the largest
                               partial reconstruction error (eq.
                               "recon_partial") are set to zero in the bound
                               core (nz = its non-zero cells; equal values in
                               increasing cell order). The error and loss
                               reported for the iteration are those before the
                               removal. Equal ranks and (N, J) in {3} x
                               {3,4,5,8,10,16}, {4} x {3,5,8,10} or {5} x
                               {3,5,8} (else PTK_E_UNSUPPORTED). Device
                               memory, allocated on first use: nnz + 64
                               doubles of residuals, the sums (per range,
                               2 * prod J_n doubles each) and R; J * nnz
                               doubles for the deltas the last mode's kernel
                               keeps when that mode has the fewest rows and
                               (N, J) is (4, 10) or (5, 8) in FP64 (only if
                               they fit in a quarter of the free memory);
                               plus the row-sum buffers of approx_form.      */
    int32_t delta_slices;   /* generic-kernel modes only (shapes without an
                               unrolled kernel): the delta sum of every entry
                               (Eq. 8) cut into this many slices of the core's
                               cells, one wavefront per 64 entries and slice,
                               partial sums added in slice order by a second
                               kernel. For observed sets too small to fill
                               the GPU otherwise (high orders, few entries).
                               0 = auto (sliced when nnz <= 64 * 16 * CUs),
                               1 = never, S > 1 = S slices (at most 65535;
                               a pair-cache writer rounds S up to a multiple
                               of its partner's rank, and no slice gets fewer
                               than one cell). Extra device memory: S * J_n *
                               nnz doubles. Chosen before ptk_set_observed.  */
    double tol;             /* early stop of ptk_iterate (Alg. 2's "until the
                               error converges"): after iteration t >= 2 it
                               stops when |e_t - e_{t-1}| <= tol * e_{t-1},
                               e = sqrt(SSE); 0 = run all iterations. With
                               tol > 0 every iteration waits for its error
                               (one small copy and synchronisation each).   */
    int32_t approx_form;    /* how the Approx variant forms its sums S1, S2
                               (ptk_iterate with approx_rate > 0,
                               ptk_partial_error, ptk_truncate); same values
                               up to rounding order. 0 = auto: row sums where
                               available, when the grouping mode's rows plus
                               the slices number at most nnz / 20 and the
                               buffers take at most a quarter of the free
                               device memory, else per-cell groups. 1 = per-cell groups: no memory
                               beyond the sums. 2 = row sums, orders 4 and 5
                               only (else PTK_E_UNSUPPORTED): every entry's
                               2J weights r a and a^2 of one mode, nnz * 2J
                               doubles, and one J^(N-1)-cell pair of sums per
                               row of the grouping mode (the one with the
                               fewest rows) and per slice of entries,
                               (rows + slices) * 2 * J^(N-1) doubles.         */
    double cond_limit;      /* accuracy limit of the Cholesky row solve (Sec.
                               3.2, eq. "rowupdate"): with M = B_i + lambda I
                               and S = diag(M)^-1/2 M diag(M)^-1/2, a row whose
                               factorisation breaks down or whose tr(S^-1)
                               exceeds cond_limit (cond(S) is within a factor
                               J_n of it) is solved instead as the regularised
                               least-squares problem whose normal equations
                               eq. "rowupdate" are: Householder QR of
                               [sqrt(lambda) I ; Delta] from the row's
                               entries, deltas recomputed in FP64. That form
                               needs no formed B_i and never breaks down for
                               lambda > 0. 0 = the default, 1e10; 1 sends
                               every non-empty row to the least-squares form.
                               Negative or not finite: PTK_E_INVALID.        */
    double sparse_limit;    /* Approx variant (approx_rate > 0) inside
                               ptk_iterate: at the start of every iteration
                               the non-zero cells of the bound core are listed
                               per mode (Sec. 3.3: after the removals most
                               cells are zero), and when their number is at
                               most sparse_limit * prod J_n the FP64 row
                               systems take delta (eq. "delta") as a sum over
                               the listed cells instead of the dense
                               contraction. Same result up to rounding order;
                               the switch is taken on the device, so it needs
                               no synchronisation. 0 = the default, 0.1;
                               negative = never; above 1 or not finite:
                               PTK_E_INVALID. Extra device memory with
                               approx_rate > 0: 16 * N * prod J_n bytes.      */
    int32_t shared_units;   /* row systems (eqs. "rowB", "rowC") from shared-
                               index units, FP64 arithmetic, equal ranks and
                               (N, J) in {(3,16), (4,10), (5,8)}: the entries
                               of every row are ordered by their index in the
                               last other mode s, and consecutive entries of
                               a row with the same i_s form units that share
                               the core contracted with that mode's row (its
                               J^N multiply-adds once per unit instead of once
                               per entry); deltas go through a J * nnz-double
                               buffer. Same result up to rounding order. 0 =
                               auto (per mode, when the units cut the
                               modelled work by a tenth or more); -1 = never
                               (rows keep the order of the input); 1 = always
                               where available, units of at most 2 entries;
                               2, 4 or 8 = always, with units of at most that
                               many entries. Runs of 64 entries or more of
                               one row and one i_s get a table of the core
                               contracted with that row (J^(N-1) doubles
                               each, at most 4 GiB per mode) instead. 16 =
                               index tables: G contracted with a row of
                               A^(s) (J^(N-1) doubles) serves every entry
                               with that i_s whatever its row; one table per
                               value of i_s with 64 entries or more (at most
                               16 GiB per mode, rebuilt at every mode
                               update), single-entry units for the entries
                               of the other values; auto takes them when the
                               model prefers them. Chosen
                               before ptk_set_observed; not used with
                               pair_cache, approx_rate > 0 or the FP32 and
                               BF16 forms. Other values: PTK_E_INVALID.      */
} ptk_options;

/*
 * Create a context for an N-order tensor of size dims_host[0..N) with core
 * ranks ranks_host[0..N), bound to the device that is current and to
 * hip_stream (a hipStream_t; NULL means the null stream).
 * Limits: 2 <= N <= 10, 1 <= J_n <= 32, 1 <= I_n < 2^31, prod J_n <= 2^20.
 * Returns PTK_E_INVALID for out-of-range arguments. *out owns all library
 * device memory of the context; release it with ptk_destroy.
 */
ptk_status ptk_create(ptk_ctx **out, int32_t N, const int64_t *dims_host,
                      const int32_t *ranks_host, void *hip_stream);

/* Release the context and all device memory it owns. NULL is accepted. */
ptk_status ptk_destroy(ptk_ctx *ctx);

/* Message of the last failed call on ctx (owned by ctx; never NULL). With
 * ctx = NULL: the message of the last failed context-free call (ptk_coo_*)
 * on the calling thread, or of a call that was given a NULL context. */
const char *ptk_last_error(const ptk_ctx *ctx);

/* Set options (see ptk_options). PTK_E_INVALID for unknown values,
 * PTK_E_UNSUPPORTED for the BF16 forms on a shape without a matrix-core
 * kernel or pair_cache where it is not available, PTK_E_STATE when chunk_nnz,
 * pair_cache or a change to or from a BF16 form comes after ptk_set_observed
 * (they shape what it builds). */
ptk_status ptk_set_options(ptk_ctx *ctx, const ptk_options *opt_host);

/*
 * Hand over the observed set Omega (Sec. 2.2): nnz entries, idx [N][nnz]
 * int32 and val [nnz] float32, both device memory that the library only
 * reads during this call. Builds, for every mode n, the grouping of entries
 * by their mode-n index (the sets Omega^(n)_i of Table 2) as a CSR copy in
 * library memory, and the per-wavefront work ranges. Synchronises the stream.
 * Errors: PTK_E_INVALID if any index is outside [0, I_n) or any value is not
 * finite (the message gives the count); PTK_E_NOMEM. nnz = 0 is valid.
 * Duplicate cells are accepted and act as separate observations.
 */
ptk_status ptk_set_observed(ptk_ctx *ctx, int64_t nnz, const int32_t *idx,
                            const float *val);

/*
 * Bind the model: core (device, float32, C order, prod J_n values) and the
 * N factor pointers in factors_host[0..N) (each device float32 I_n x J_n).
 * The caller keeps ownership and must keep the buffers alive while bound.
 * Later calls read them and update the factors in place; the core is only
 * written by ptk_orthogonalize. The core may be changed by the caller
 * between calls (the library re-reads it at the start of every call).
 */
ptk_status ptk_bind_model(ptk_ctx *ctx, float *core, float *const *factors_host);

/*
 * One pass of Alg. 3 for mode n (0-based): every row i of A^(n) becomes the
 * solution of (B_i + lambda I) a_i = c_i (eq. "rowupdate"), where B_i and
 * c_i sum delta delta^T and x delta (eqs. "rowB", "rowC", "delta") over the
 * entries of row i. A row with no entry becomes 0. Requires lambda > 0
 * (PTK_E_INVALID otherwise). Rows whose Cholesky solve would be inaccurate
 * are solved in the least-squares form (see ptk_options.cond_limit), so every
 * row gets the unique solution; PTK_E_NOT_PD only if a result is not finite
 * (non-finite or overflowing data; those rows are left unchanged).
 */
ptk_status ptk_update_mode(ptk_ctx *ctx, int32_t n, double lambda);

/*
 * iters iterations of Alg. 2: modes 0..N-1 in order, then the
 * reconstruction error. sse_host[t] / loss_host[t] (either may be NULL)
 * receive, after iteration t, sum over Omega of (x - x_hat)^2 (the square of
 * eq. "reconfull") and the loss of eq. "TF_PARTIAL". Every row is solved as
 * in ptk_update_mode. Status, after all iterations ran and the outputs are
 * filled: PTK_E_NOT_PD if some row result was not finite (count from
 * ptk_not_pd_count); else PTK_E_DIVERGED if some SSE or loss is not finite,
 * or a loss exceeds the previous iteration's of the same call by more than
 * 1e-6 relative (Theorem 2 makes the loss non-increasing in exact
 * arithmetic; the FP32 and BF16 forms can break this, the FP64 form only by
 * the rounding of the stored float32 factors; not checked with approx_rate >
 * 0, whose removal changes the model between iterations); else PTK_OK.
 */
ptk_status ptk_iterate(ptk_ctx *ctx, int32_t iters, double lambda,
                       double *sse_host, double *loss_host);

/* Iterations the last ptk_iterate ran (fewer than asked when options.tol
 * stopped it early; the sse/loss entries past them are NaN). */
ptk_status ptk_iterations_done(const ptk_ctx *ctx, int32_t *n_host);

/*
 * Number of rows left unsolved (result not finite, row unchanged) during the
 * last ptk_update_mode / ptk_iterate call, or of rank-deficient factors of the
 * last ptk_orthogonalize. Zero for finite data and lambda > 0. Synchronises
 * the stream.
 */
ptk_status ptk_not_pd_count(ptk_ctx *ctx, int64_t *count_host);

/*
 * Rows of the last ptk_update_mode / ptk_iterate call (summed over modes and
 * iterations) that the least-squares form solved (see
 * ptk_options.cond_limit), and the most entries any of them had.
 */
ptk_status ptk_solve_stats(ptk_ctx *ctx, int64_t *ls_rows_host,
                           int64_t *ls_max_entries_host);

/*
 * Sparse core of the Approx variant (ptk_options.sparse_limit) in the last
 * iteration of the last ptk_iterate: the non-zero cells of the bound core
 * that iteration started from, and a bit mask of the modes (bit n = mode n)
 * whose row systems summed delta over those cells only. Waits for the
 * context's stream. When that iteration listed no cells (approx_rate = 0,
 * sparse_limit < 0, a shape without the kernel, or no ptk_iterate yet):
 * -1 and 0.
 */
ptk_status ptk_approx_stats(ptk_ctx *ctx, int64_t *nonzero_cells_host,
                            int32_t *sparse_modes_host);

/*
 * Shared-index row systems of mode n (ptk_options.shared_units) as built by
 * the last ptk_set_observed; s is the last mode other than n. A run is a
 * maximal sequence of grouped entries of one row with the same i_s. A run of
 * 64 entries or more is long (it gets a table of the core contracted with
 * that row of A^(s), and its entries are processed in tasks of at most 128);
 * any other run of r entries gives floor(r / emax) units of emax entries,
 * then one unit for each set bit of r mod emax (emax is 2, or the option's
 * 4 or 8 where a kernel exists: 8 at orders 3 and 4 with J <= 10, else 4).
 * The index groups are the entries of one value of i_s whatever their row:
 * a value with 64 entries or more gets a table and its entries are processed
 * in tasks of at most 128; the entries of a value with fewer are single-entry
 * units instead. counts_host receives 9 values: the units of 1, 2, 4 and 8
 * entries, the long runs, their tasks, the index values with a table, their
 * tasks and the single-entry units of the other values (zero where a form
 * was not built). *on_host: the form mode n's row systems use: 0 the fused
 * kernels, 1 units, 2 index tables.
 * PTK_E_INVALID for n out of range, PTK_E_STATE before ptk_set_observed.
 */
ptk_status ptk_unit_stats(ptk_ctx *ctx, int32_t n, int64_t *counts_host, int32_t *on_host);

/*
 * ptk_fold_in without any allocation, for callers that cannot allocate:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * device allocation. Same arguments, result and errors as ptk_fold_in (same
 * kernels); the work buffers (row system, at most 128 work-range partial
 * systems, the merge and least-squares lists, least-squares triangles) live
 * in a fixed 2 MiB device array of the library, one per device, held until
 * the process ends; the call makes no hipMalloc / hipFree. Limit: k <= 2^24
 * entries (PTK_E_INVALID beyond it). Every call on a device shares that
 * device's array: calls that overlap on one device (other streams, other
 * threads, other contexts) race and must be serialised by the caller.
 */
ptk_status ptk_fold_in_noalloc(ptk_ctx *ctx, int32_t n, int64_t k, const int32_t *idx,
                               const float *val, double lambda, float *row_out);

/*
 * Autotuner of the batching form (the GPU counterpart of the dynamic row
 * schedule of Sec. 3.4). For every mode it times the row-system kernels
 * (delta, Gram, merge) of the bound model on the observed set for several
 * sizes of the per-wavefront work ranges (entries per range for the FP64 /
 * FP32 forms, 32-entry blocks per range for the BF16 forms) and, where both
 * are compiled (FP64 arithmetic at (N, J) = (4, 10) and (5, 8)), for tiles of
 * one and of two entries per lane, and keeps the fastest; the model is not
 * modified. Rows are cut at any entry between ranges (their pieces are merged
 * in range order), so there is no row-split threshold to choose. cache_path
 * (host string, may be NULL) names a text file of "key work" or "key work
 * two" lines keyed by order, ranks, precision, entry count, mode size and the
 * mode's row-length histogram: a hit is applied without timing, a new result
 * is appended. work_host (NULL or N entries) receives the chosen sizes.
 * Synchronises the stream.
 */
ptk_status ptk_autotune(ptk_ctx *ctx, const char *cache_path, int64_t *work_host);

/*
 * Reconstruction error of the bound model on Omega (eq. "reconfull"):
 * *sse_host = sum (x - x_hat)^2, *rmse_host = sqrt(sse / nnz),
 * *loss_host = sse + lambda * sum_n ||A^(n)||_F^2 (eq. "TF_PARTIAL").
 * Any output pointer may be NULL.
 */
ptk_status ptk_recon_error(ptk_ctx *ctx, double lambda, double *sse_host,
                           double *rmse_host, double *loss_host);

/*
 * Final step of Alg. 2 (Sec. 3.1): for n = 0..N-1, A^(n) = Q R (thin QR,
 * diag(R) > 0), A^(n) <- Q, G <- G x_n R. Writes the bound factors and core.
 * The QR is shifted CholeskyQR3 in FP64 (three Gram + Cholesky passes, the
 * first with a small diagonal shift), defined for factors with condition
 * numbers up to about 1e15. PTK_E_NOT_PD if some A^(n) does not have full
 * column rank in floating point.
 */
ptk_status ptk_orthogonalize(ptk_ctx *ctx);

/*
 * Predictions x_hat (eq. "recon2") for m cells: idx [N][m] int32 (device),
 * out [m] float32 (device, caller-owned). Stream-ordered; does not
 * synchronise. PTK_E_INVALID for m < 0. Indices are not range-checked here:
 * the caller guarantees 0 <= idx[n*m+e] < I_n.
 */
ptk_status ptk_predict(ptk_ctx *ctx, int64_t m, const int32_t *idx, float *out);

/*
 * Fold-in (eq. "rowupdate" for a row that is not in the model): the row of
 * mode n that best fits k observations with G and the other factors held
 * fixed. idx [N][k] int32 device (the mode-n array is not read), val [k]
 * float32 device, row_out [J_n] float32 device. k = 0 gives a zero row.
 * Stream-ordered; does not synchronise.
 */
ptk_status ptk_fold_in(ptk_ctx *ctx, int32_t n, int64_t k, const int32_t *idx,
                       const float *val, double lambda, float *row_out);

/*
 * Inspection of intermediate results (eqs. "delta", "rowB", "rowC").
 * ptk_delta: delta^(n) for m cells, idx [N][m] device, out [m][J_n] float32
 * device. ptk_row_systems: B_i and c_i of every row of mode n for the bound
 * model, written as float64 to B_out [I_n][J_n][J_n] and c_out [I_n][J_n]
 * (device; rows with no entry are zero). Both synchronise the stream.
 */
ptk_status ptk_delta(ptk_ctx *ctx, int32_t n, int64_t m, const int32_t *idx,
                     float *out);
ptk_status ptk_row_systems(ptk_ctx *ctx, int32_t n, double *B_out,
                           double *c_out);

/*
 * Approx variant (Alg. 4, Sec. 3.3) on the bound model, outside ptk_iterate.
 * ptk_partial_error: R(beta) of eq. "recon_partial" for every core cell,
 * R_out [J_1]...[J_N] float64 device (C order), 0 for cells that are zero in
 * the core. ptk_truncate: one removal with rate p (0 <= p < 1) as in
 * ptk_options.approx_rate, applied to the bound core; *removed_host receives
 * the number of cells set to zero. Both synchronise the stream. Errors:
 * PTK_E_INVALID, PTK_E_STATE (no observed set or model), PTK_E_UNSUPPORTED
 * (shape without the Approx kernels).
 */
ptk_status ptk_partial_error(ptk_ctx *ctx, double *R_out);
ptk_status ptk_truncate(ptk_ctx *ctx, double p, int32_t *removed_host);

/* ------------------------------------------------------------------------
 * Steps either side of the fit (Sec. 4.1, Sec. 4.5, Sec. 5).
 * --------------------------------------------------------------------- */

/*
 * COO text input: one observed entry per line, N indices starting at 1 (the
 * paper's convention, Sec. 2) and then the value, separated by blanks or
 * tabs; lines holding only blanks are skipped. Host code, no GPU, parsed by
 * up to 16 threads. ptk_coo_scan gives the entry count and, per mode, the
 * largest index (so dims_out[n] = max index; dims_out [N] host). ptk_coo_read
 * fills idx_host [N][nnz] int32 (0-based) and val_host [nnz] float32 (host
 * memory, caller-owned) in file order; nnz must be the scanned count.
 * Errors (text from ptk_last_error(NULL)): PTK_E_INVALID for an unreadable
 * file, N outside [1, 10], a line without exactly N integers >= 1 and a
 * finite value (the message gives the line number), an index above 2^31 - 1,
 * or an nnz that differs from the file's count.
 */
ptk_status ptk_coo_scan(const char *path, int32_t N, int64_t *nnz_out, int64_t *dims_out);
ptk_status ptk_coo_read(const char *path, int32_t N, int64_t nnz, int32_t *idx_host,
                        float *val_host);

/*
 * Min-max normalisation of the values to [0, 1] (Sec. 4.1): val [nnz] float32
 * device, in place, v <- (v - min) / (max - min) computed in FP64 (all 0 when
 * max = min). minmax_host [2] (may be NULL) receives min and max. Values must
 * be finite. Synchronises the stream.
 */
ptk_status ptk_normalize_values(ptk_ctx *ctx, int64_t nnz, float *val, double *minmax_host);

/*
 * Seeded train/test split of an entry list (Sec. 4.1 holds out 10 %). Entry e
 * is held out when u_e < test_fraction, where u_e is the top 53 bits, over
 * 2^53, of output e + 1 of the SplitMix64 generator (Steele, Lea and Flood,
 * 2014) seeded with `seed`: a pure function of (seed, e), so any subset can
 * be recomputed. ptk_split_count gives the held-out count. ptk_split_entries
 * writes both sides in their original order: idx_train [N][nnz - ntest],
 * val_train [nnz - ntest], idx_test [N][ntest], val_test [ntest] (device,
 * caller-owned) from idx [N][nnz], val [nnz] (device). ntest must be the
 * count ptk_split_count returns (else PTK_E_INVALID). test_fraction in
 * [0, 1]. Both synchronise the stream.
 */
ptk_status ptk_split_count(ptk_ctx *ctx, int64_t nnz, double test_fraction, uint64_t seed,
                           int64_t *ntest_host);
ptk_status ptk_split_entries(ptk_ctx *ctx, int32_t N, int64_t nnz, const int32_t *idx,
                             const float *val, double test_fraction, uint64_t seed,
                             int64_t ntest, int32_t *idx_train, float *val_train,
                             int32_t *idx_test, float *val_test);

/*
 * Error of the bound model over any entry list (the test RMSE of Sec. 4.5):
 * idx [N][m] int32, val [m] float32 (device), indices within the model's
 * dims (not range-checked here). *sse_host = sum (x - xhat)^2 (eq.
 * "reconfull" over the list), *rmse_host = sqrt(sse / m) (0 for m = 0).
 * Synchronises the stream.
 */
ptk_status ptk_entry_error(ptk_ctx *ctx, int64_t m, const int32_t *idx, const float *val,
                           double *sse_host, double *rmse_host);

/*
 * K-means over the rows of the bound factor A^(n) (concept discovery, Sec. 5):
 * Lloyd's iterations from the given centroids. centroids [K][J_n] float64
 * device, in/out: initial centroids on entry (the caller draws them), final
 * ones on return. Each of `iters` rounds assigns every row to its nearest
 * centroid (squared Euclidean distance in FP64, the lowest index among equal
 * distances) and moves each centroid to the mean of its rows (a centroid
 * without rows stays); a last assignment follows. assign [I_n] int32 device
 * receives it. result_host [2] (may be NULL): the inertia (sum of squared
 * distances of the last assignment) and the number of rows whose cluster
 * changed in it. K * (J_n + 1) * 8 <= 32768. Deterministic; synchronises.
 */
ptk_status ptk_kmeans(ptk_ctx *ctx, int32_t n, int32_t K, int32_t iters, double *centroids,
                      int32_t *assign, double *result_host);

/*
 * Per-kernel timing collected while options.profile = 1: for each kernel
 * family k < *count_host, names_host[k] (static strings), calls_host[k] and
 * ms_host[k] (summed HIP-event durations on the context's stream). *count_host
 * is in/out: capacity on entry, number of families on return.
 * ptk_reset_timers clears the totals.
 */
ptk_status ptk_kernel_times(ptk_ctx *ctx, int32_t *count_host,
                            const char **names_host, int64_t *calls_host,
                            double *ms_host);
ptk_status ptk_reset_timers(ptk_ctx *ctx);

/* ------------------------------------------------------------------------
 * Serving: a continuous-batching request loop on a bound model.
 *
 * Fold-in requests (the row update of eq. "rowupdate" for a new row of mode
 * n, with G and the factors fixed) and prediction requests (eq. "recon2" for
 * missing entries) are copied at submit, queued, and served by a library
 * thread in batches. Up to `slots` batches are in flight at once, each on its
 * own stream with its own part of the device-memory budget; requests are
 * admitted first-in first-out as a slot's memory frees up, so requests that
 * arrive while others run on the GPU start as soon as a slot is idle. Every
 * request's result is bitwise the same whether it is served alone or in a
 * mix. While a server runs on a context, the caller must not change the
 * bound model or call into the context.
 * ------------------------------------------------------------------------ */
typedef struct ptk_server ptk_server;

typedef struct ptk_server_opts {
    int64_t mem_budget_bytes;   /* device bytes for in-flight batches, split
                                   evenly over the slots; 0 = 512 MiB        */
    int32_t slots;              /* batches in flight; 0 = 2                  */
    int32_t max_batch_requests; /* requests per batch; 0 = 4096              */
    int32_t queue_capacity;     /* queued requests before PTK_E_BUSY; 0 = 2^20 */
    double lambda;              /* regularisation of the fold-in solves (> 0) */
} ptk_server_opts;

typedef struct ptk_server_stats {
    int64_t batches;            /* batches completed                        */
    int64_t requests;           /* requests completed                       */
    int64_t max_batch_requests; /* largest batch                            */
    int64_t max_in_flight;      /* most batches on the GPU at the same time  */
    int64_t queued;             /* requests waiting now                     */
} ptk_server_stats;

/* Start a server on ctx (which must have a bound model). *out owns the
 * thread, streams, device arenas and pinned staging memory.
 * PTK_E_INVALID for bad options (lambda <= 0, budget too small). */
ptk_status ptk_server_create(ptk_server **out, ptk_ctx *ctx,
                             const ptk_server_opts *opts_host);

/* Queue a fold-in of mode n from k observations: idx_host [N][k] (the mode-n
 * array is not read), val_host [k], both host memory copied before return.
 * *ticket identifies the request. PTK_E_INVALID for out-of-range indices or
 * non-finite values (nothing is queued), PTK_E_NOMEM if the request alone
 * exceeds a slot's memory, PTK_E_BUSY if the queue is full. */
ptk_status ptk_server_submit_foldin(ptk_server *srv, int32_t n, int64_t k,
                                    const int32_t *idx_host,
                                    const float *val_host, uint64_t *ticket);

/* Queue predictions of m cells: idx_host [N][m] host memory, copied. Errors
 * as for fold-in. */
ptk_status ptk_server_submit_predict(ptk_server *srv, int64_t m,
                                     const int32_t *idx_host, uint64_t *ticket);

/* Non-blocking: *done = 1 when the request has finished; then up to cap
 * floats of its result (J_n for a fold-in, m for predictions) are copied to
 * out_host, *req_status receives its own status (PTK_OK, PTK_E_NOT_PD for a
 * fold-in whose system was not positive definite in FP64, PTK_E_HIP), the
 * submit-to-completion time goes to *latency_ms (may be NULL) and the ticket
 * is released. */
ptk_status ptk_server_poll(ptk_server *srv, uint64_t ticket, float *out_host,
                           int64_t cap, int32_t *done, ptk_status *req_status,
                           double *latency_ms);

/* As ptk_server_poll, but blocks up to timeout_s seconds (PTK_E_BUSY on
 * timeout, the ticket stays valid). */
ptk_status ptk_server_wait(ptk_server *srv, uint64_t ticket, float *out_host,
                           int64_t cap, double timeout_s, ptk_status *req_status,
                           double *latency_ms);

ptk_status ptk_server_get_stats(ptk_server *srv, ptk_server_stats *out_host);
const char *ptk_server_last_error(const ptk_server *srv);

/* Finish every submitted request, stop the thread, free everything. */
ptk_status ptk_server_destroy(ptk_server *srv);

/* ------------------------------------------------------------------------
 * Measurement.
 * --------------------------------------------------------------------- */

/*
 * Sustained FP64 rates of the current device, the ceiling for the roofline
 * of the row-system kernels (one FP64 multiply-add per core cell and entry,
 * Alg. 3). Runs three kernels with no memory traffic, each over 2048 x 256
 * lanes for `iters` iterations (1..1e6), timed with HIP events on the null
 * stream after one warm-up launch. tflops_host[3] (host) receives TFLOP/s of:
 * [0] independent v_fma_f64 chains; [1] v_mfma_f64_16x16x4f64; [2] both
 * interleaved in every wavefront. Allocates and frees 4 MB of device memory.
 * Errors: PTK_E_INVALID, PTK_E_HIP.
 */
ptk_status ptk_fp64_rates(int32_t iters, double *tflops_host);

#ifdef __cplusplus
}
#endif

#endif /* PTUCKER_H */
