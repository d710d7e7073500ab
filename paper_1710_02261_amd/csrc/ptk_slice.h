// Core-sliced row systems for observed sets too small to fill the GPU with
// one wavefront per 64 entries (high orders, few entries: Sec. 4.2's order
// sweep). Launchers.
#pragma once

#include "ptk_internal.h"

namespace ptk {

// The delta of an entry (Eq. 8's vector: G contracted with the rows of every
// mode but n) is a sum over the J^(N-1) cells of the other modes. Here the
// cells are cut into S slices, one wavefront per (64-entry tile, slice). A
// workgroup holds W slices of one tile (W wavefronts sharing the tile's
// rows in LDS) and adds their sums in wavefront order, so S / W partial
// groups per entry reach memory; the second kernel adds those in group
// order and sweeps the row systems as the unsliced kernels do.
//
// Pair-cache writer (writer = 1, other-mode slot 0 is the partner p and the
// permuted core leads with it): S = J_p * sub with sub slices per partner
// index and W dividing sub, so no slice or group straddles two partner
// indices; the partner's weight is left out of the partials, and the second
// kernel stores the record T[m_p][:] (the sum of the sub / W groups of index
// m_p) before weighting it into delta.
struct SliceArgs {
    GramArgs g;
    double *dpart;     // [S / W][J_n][nnzp] partial sums (entry fastest)
    int64_t nnzp;      // entry stride of dpart (nnz rounded up to 64)
    int32_t S;         // slices
    int32_t sub;       // slices per partner index (writer), else S
    int32_t W;         // wavefronts (slices) per workgroup, a power of two <= 16
    int32_t writer;
};

struct SlicePlan {
    int32_t S = 1, sub = 1, W = 1;
};

// Slice plan of mode n on the generic path. want = 0: automatic (S = 1, no
// slicing, when the tiles alone fill the GPU; else enough (tile, slice)
// wavefronts to keep every SIMD busy with at least 16 cells per slice);
// want > 1: that many slices, at most one per cell. A pair-cache writer
// (partner >= 0) gets a multiple of the partner's rank (rounded up). W is
// the largest power of two <= 16 that divides S (writer: sub) and keeps the
// workgroup's LDS within 64 KiB.
SlicePlan slice_plan(const Shape &s, int n, int partner, int64_t nnz, int num_cu,
                     int32_t want);
// Doubles of dpart for a plan.
int64_t slice_part_doubles(int J, int64_t nnz, const SlicePlan &p);

hipError_t launch_delta_slices(const SliceArgs &a, hipStream_t st);
hipError_t launch_gram_slices(const SliceArgs &a, int64_t nchunks, hipStream_t st);
int gram_slices_blocks_per_cu(int J);

}  // namespace ptk
