// Core-sliced row systems for observed sets too small to fill the GPU with
// one wavefront per 64 entries (high orders, few entries: Sec. 4.2's order
// sweep). Launchers.
#pragma once

#include "ptk_internal.h"

namespace ptk {

// The delta of an entry (Eq. 8's vector: G contracted with the rows of every
// mode but n) is a sum over the J^(N-1) cells of the other modes. Here the
// cells are cut into S slices: one kernel gives every (64-entry tile, slice)
// pair its own wavefront and stores the slice's partial sum, the next one
// adds the S partials of each entry in slice order and sweeps the row
// systems as the unsliced kernels do.
//
// Pair-cache writer (writer = 1, other-mode slot 0 is the partner p and the
// permuted core leads with it): the slices never straddle two partner
// indices (S = J_p * sub, sub slices per index), the partner's weight is left
// out of the partials, and the second kernel stores the record T[m_p][:] (the
// sum of the sub partials of index m_p) before weighting it into delta.
struct SliceArgs {
    GramArgs g;
    double *dpart;     // [S][J_n][nnzp] partial sums (entry position fastest)
    int64_t nnzp;      // entry stride of dpart (nnz rounded up to 64)
    int32_t S;         // slices
    int32_t sub;       // slices per partner index (writer), else S
    int32_t writer;
};

// Slices for mode n on the generic path (1: do not slice): enough (tile,
// slice) wavefronts to keep every SIMD busy, at least 16 cells per slice.
// For a pair-cache writer (partner >= 0, the partner's slot leading) the
// result is a multiple of the partner's rank.
int32_t slice_count(const Shape &s, int n, int partner, int64_t nnz, int num_cu);
// A requested slice count made valid: at most one slice per cell, and for
// a pair-cache writer a multiple of the partner's rank (rounded up, at most
// one slice per cell of a partner index).
int32_t slice_fixed(const Shape &s, int n, int partner, int32_t want);
// Doubles of dpart for S slices.
int64_t slice_part_doubles(int J, int64_t nnz, int32_t S);

hipError_t launch_delta_slices(const SliceArgs &a, hipStream_t st);
hipError_t launch_gram_slices(const SliceArgs &a, int64_t nchunks, hipStream_t st);
int gram_slices_blocks_per_cu(int J);

}  // namespace ptk
