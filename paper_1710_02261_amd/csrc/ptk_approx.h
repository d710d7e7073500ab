// Approx variant of the ALS sweep (Alg. 4, Sec. 3.3): launchers.
#pragma once

#include "ptk_internal.h"

namespace ptk {

// Arguments of the partial-error kernel: the entries grouped by the rows of
// one mode g (the grouping of the row-system kernels for mode g).
struct ApproxArgs {
    const float *fac[kMaxN];          // factors of the modes other than g, in
    const int32_t *idx[kMaxN];        //   increasing mode order, and their indices
    const float *fac_g;               // factor of mode g
    const int32_t *rows;              // mode-g index per entry
    const double *resid;              // xhat - x per entry
    int32_t g;
    int64_t nnz;
    int64_t slice;                    // entries per slice
    int32_t nslices;
    double *part;                     // [nslices][2][cells]: sums S1, S2
};

// Arguments of the row-sum form (orders 4 and 5).
struct RowSumArgs {
    const float *fac[kMaxN];          // as ApproxArgs: modes other than g
    const int32_t *idx[kMaxN];
    const float *fac_g;
    const int32_t *rows;              // mode-g index per entry (grouped order)
    const int64_t *rowptr;            // CSR row pointers of mode g
    const double *resid;              // xhat - x per entry
    double *uw;                       // [nnz][2][J] per-entry weights (scratch)
    int32_t uw_ready;                 // 1: uw already written (with the residuals)
    double *tbuf;                     // [nslots][2][J^(N-1)] row-piece sums
    int32_t g;
    int64_t nrows;                    // rows of mode g
    int64_t nnz;
    int64_t slice;                    // entries per slice
    int64_t nslices;
    int64_t nslots;                   // nrows + nslices
    int64_t fold_per;                 // slots per fold range
    int32_t nfold;                    // fold ranges
    double *part;                     // [nfold][2][cells]: sums S1, S2
};

// Is the Approx variant compiled for this (N, J) with equal ranks?
bool approx_available(int N, int J);

// resid[e] = xhat_e - x_e over the entries of one mode's grouping (a.m of
// them; a.own / a.own_idx that mode's factor and indices); a.partial
// receives the residuals (FP64), a.gp is the FP64 core permuted for it.
hipError_t launch_residual(const EntryArgs &a, const Shape &s, int64_t nblocks,
                           hipStream_t st);

// The residuals of the same grouping from stored deltas ([J][nnz]) and the
// updated factor of that mode: resid = delta . a_new - x.
hipError_t launch_resid_from_delta(const double *delta, const float *fac, const int32_t *rows,
                                   const float *val, int64_t nnz, int J, double *resid,
                                   hipStream_t st);

// The same residuals into resid and, in the same pass, the row-sum form's
// weights into uw ([nnz][2][J]) from the rows of the third-last other mode
// (fac3, idx3); J in {3, 5, 8, 10}.
hipError_t launch_resid_uw_from_delta(const double *delta, const float *fac,
                                      const int32_t *rows, const float *val,
                                      const float *fac3, const int32_t *idx3, int64_t nnz,
                                      int J, double *resid, double *uw, hipStream_t st);

// Slices and part size (doubles) for nnz entries.
int32_t approx_slices(const Shape &s, int64_t nnz, int num_cu);
int64_t approx_part_doubles(const Shape &s, int32_t nslices);

// S1, S2 per slice, then R(beta) = 2 G S1 - G^2 S2 for every cell.
hipError_t launch_partial_error(const ApproxArgs &a, const Shape &s, hipStream_t st);
hipError_t launch_partial_reduce(const double *part, int32_t nslices, const float *G,
                                 int64_t cells, double *R, hipStream_t st);

// Row-sum form: available for orders 4 and 5; slices; slot buffer size
// (doubles); S1, S2 per fold range into a.part.
bool row_sums_available(int N, int J);
int64_t row_sums_slices(const Shape &s, int64_t nnz, int num_cu);
int64_t row_sums_tbuf_doubles(const Shape &s, int g, int64_t nslices);
hipError_t launch_row_sums(const RowSumArgs &a, const Shape &s, hipStream_t st);

// Alg. 4's removal: zero the floor(p * nz) non-zero cells of G with the
// largest R (ties: lower cell index first); *removed receives the count.
hipError_t launch_approx_select(const double *R, float *G, int64_t cells, double p,
                                int32_t *removed, hipStream_t st);

}  // namespace ptk
