// Row systems of the Approx variant from the non-zero cells of the core only
// (Alg. 4, Sec. 3.3): per-mode cell lists built on the device from the bound
// core, and the row-system kernel that forms delta from them.
#pragma once

#include "ptk_internal.h"

namespace ptk {

// Default of ptk_options.sparse_limit: the non-zero fraction of the core at
// or below which the sparse-core kernel is the faster one.
constexpr double kSparseLimitDefault = 0.1;

// Cell lists of all modes. For mode n: the non-zero cells sorted by
// j = beta_n, then by the other modes' indices in C order (last fastest);
// cstart[n][j] .. cstart[n][j + 1] are the records of j, and one empty record
// (value 0) follows the last, so reading one ahead stays in bounds. A record
// is four words: the value (FP64, two words); the register index of its last
// other-mode factor value, (N - 2) * J + beta; and, byte l for the leading
// other modes l < N - 2, l * J + beta_l, with the top byte holding the first
// slot whose index differs from the previous record of the same j (0 for
// the first record of a j).
struct SparseArgs {
    int32_t N, J;              // order and the (equal) rank (N <= 5)
    int64_t cells;             // J^N
    int64_t rec;               // cells + 1: records per mode
    int32_t *count;            // [N * J]   non-zero cells per (n, j)
    int32_t *cstart;           // [N * (J + 1)] first record per (n, j)
    uint32_t *recs;            // [N * rec * 4]
    int32_t *use;              // [N] 1: the sparse kernel forms mode n
    double limit;              // use when non-zero cells <= limit * cells
};

// One mode's lists, as the row-system kernel reads them.
struct SparseMode {
    const int32_t *use;        // &use[n]
    const int32_t *cstart;     // [J + 1]
    const uint32_t *recs;      // [rec * 4]
};

// (N, J) with a sparse-core row-system kernel.
bool sparse_available(int N, int J);

// Rebuild every mode's lists and switch from the core G (C order).
hipError_t launch_sparse_lists(const float *G, const SparseArgs &s, hipStream_t st);

// Row systems of one mode into bbuf / part, like launch_gram with the same
// chunks; returns at once on the device when *sm.use is 0.
hipError_t launch_gram_sparse(const GramArgs &a, int N, int J, const SparseMode &sm,
                              int64_t nchunks, hipStream_t st);

}  // namespace ptk
