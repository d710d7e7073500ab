// Context of the C ABI (shared by ptk_api.hip and ptk_server.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "ptk_internal.h"

namespace ptk {

constexpr int kRedBlocks = 1024;   // blocks of the error / norm reductions
constexpr int kSseBlocks = 8192;   // single-wave blocks of the direct error pass
constexpr int kCtrSlots = 4 + 4 * kMaxN;
constexpr int kFoldTasks = 1025;   // heavy-task capacity of one fold-in row

struct ModeData {
    int64_t *rowptr = nullptr;
    int32_t *rows = nullptr;
    int32_t *oidx = nullptr;     // [N-1][nnz]
    float *vals = nullptr;
    int32_t *cmap = nullptr;     // pair-cache reader: own position -> writer's
    int64_t chunk = 0, nchunks = 0;
    int32_t *split = nullptr;    // [nsplit][3]
    int32_t nsplit = 0;
    bool fast = false;
    bool two = true;             // the two-entries-per-lane kernel where compiled (tuned)
    // generic path on a small observed set: the delta sum cut into slices
    // of the core cells (1: unsliced), sub slices per partner index, W
    // slices per workgroup
    int32_t slices = 1, slice_sub = 1, slice_w = 1;
    // BF16 matrix-core form: blocks of <= 32 entries of one row
    bool bf16 = false;
    int split_bf16 = 1;          // 1: bf16 operands; 3: hi/lo split products
    int32_t *blk_row = nullptr, *blk_start = nullptr, *blk_cnt = nullptr;
    int64_t nblk = 0, blk_per_wave = 0, nwaves = 0;
    // shared-index units: start positions [sum ucount], classes of 2^c
    // entries at ubase[c]; on: the row systems of this mode use them
    int32_t *units = nullptr;
    int64_t ucount[4] = {0, 0, 0, 0}, ubase[4] = {0, 0, 0, 0};
    UnitLong lg;                 // long runs and their tasks (device arrays)
    bool units_on = false;
    // index tables: grouped positions in the order of i_s, the groups of one
    // i_s value and their tasks (task_run = the value); on: this mode uses them
    int32_t *spos = nullptr;
    UnitLong ix;
    bool ix_on = false;
    // host copies used to recompute the work split (autotuner)
    std::vector<int64_t> rp_host;
    std::vector<int32_t> first_blk, last_blk;
    int64_t part_elems = 0;
};

struct Timed {
    const char *name;
    hipEvent_t a, b;
};

}  // namespace ptk

struct ptk_ctx {
    using ModeData = ptk::ModeData;
    using Timed = ptk::Timed;
    using Shape = ptk::Shape;

    Shape s{};
    hipStream_t st = nullptr;
    int device = 0;
    int num_cu = 256;
    ptk_options opt{PTK_PREC_FP64_ACC, 0, 1, 0, 1, 0, 0.0, 0, 0.0, 0, 0.0, 0.0, 0};
    int64_t nnz = -1;
    ModeData md[ptk::kMaxN];
    float *core = nullptr;
    float *fac[ptk::kMaxN] = {};
    void *gp[ptk::kMaxN] = {};        // permuted cores of the row-system kernels
    void *frag[ptk::kMaxN] = {};      // bf16 core fragments of the matrix-core kernel
    double *gpe = nullptr;       // fp64 permuted core of the per-entry kernels
    int gpe_mode = -1;
    int64_t core_cells = 1;
    double *bbuf = nullptr;
    double *part = nullptr;
    double *pcache = nullptr;    // pair cache [nnz + 1][J][J]
    double *dpart = nullptr;     // slice partials of the sliced delta path
    double *dunits = nullptr;    // deltas [nnz][J] of the shared-index units
    double *gph = nullptr;       // pass-major copy of a permuted core (units)
    double *ltab = nullptr;      // tables of the long runs of one mode (units)
    double *itab = nullptr;      // index tables of one mode [I_s][J^(N-1)]
    // Approx variant: residuals [nnz], slice sums, R per cell, removed count
    double *ap_resid = nullptr, *ap_part = nullptr, *ap_R = nullptr;
    int32_t *ap_removed = nullptr;
    int32_t ap_slices = 0;
    // row-sum form of the partial errors: per-entry weights, row-piece sums
    double *ap_uw = nullptr, *ap_tbuf = nullptr;
    int32_t ap_form = 0;         // 0 none yet, 1 per-cell-group sums, 2 row sums
    int64_t ap_rs_slices = 0;
    int32_t ap_nfold = 0;
    // deltas of the last mode kept by its row-system kernel ([J][nnz]) for the
    // residuals; ap_store asks systems() to keep them, ap_stored says it did
    double *ap_delta = nullptr;
    bool ap_store = false, ap_stored = false;
    // sparse core of the Approx variant: per-mode lists of the non-zero
    // cells and the per-mode switch (ptk_sparse.h), rebuilt at the start of
    // every iteration; sp_live while such an iteration body is recorded
    int32_t *sp_count = nullptr, *sp_cstart = nullptr, *sp_use = nullptr;
    uint32_t *sp_recs = nullptr;
    bool sp_live = false;
    bool sp_lists = false;       // the iteration last recorded builds the lists
    int64_t part_cap = 0;
    double *red = nullptr;       // [kRedBlocks * (N + 1)] partials + scalars
    double *xsq = nullptr;       // sum of x^2 over Omega (device, 1 double)
    double *scal = nullptr;      // [2] error and factor norms of one iteration
    double *dres = nullptr;      // [2 * dres_cap] per-iteration results
    int64_t dres_cap = 0;
    int32_t *iter_ctr = nullptr; // device iteration counter for dres
    uint64_t epoch = 1;          // bumped whenever captured launch arguments change
    hipStream_t gstream = nullptr;
    hipGraphExec_t gexec = nullptr;
    uint64_t g_epoch = 0;
    double g_lambda = 0.0;
    int g_fuse = -1;
    // counters [kCtrSlots] int32: [0] rows left unsolved (or rank-deficient
    // factors of the final QR), [1] rows solved in least-squares form, [2] the
    // most entries of such a row, [3] spare, [4 + 4n .. 7 + 4n] the packed,
    // single and heavy rows and heavy tasks flagged in mode n (zeroed at the
    // start of every iteration)
    int32_t *ctr = nullptr;
    int32_t *bad = nullptr;      // ctr + 0
    // rows handed to the least-squares solve: the list (max I_n), a flag byte
    // per row, the rows' error terms (last mode of a fused-error iteration);
    // heavy rows, their first tasks and the tasks' triangles (sized at
    // ptk_set_observed, see SolveFlags)
    int32_t *lslist = nullptr;
    uint8_t *rflag = nullptr;
    double *rsse = nullptr;
    int64_t max_rows = 0;
    int32_t *ls_hrow = nullptr, *ls_hoff = nullptr;
    double *ls_tri = nullptr;
    int64_t ls_hcap = 0, ls_tcap = 0;
    int64_t last_not_pd = 0, last_ls_rows = 0, last_ls_max = 0;
    // deltas kept by the row-system kernels for the least-squares rows: the
    // plan of mode n at ls_kbase + kb_off[n] (one slot base per row, see
    // GramArgs::kbase), the kept deltas [ls_kcap][J_max], the plan's counter;
    // keep_live: the current mode update's row-system kernel kept them
    int64_t *ls_kbase = nullptr;
    int64_t kb_off[ptk::kMaxN] = {};
    double *ls_keep = nullptr;
    unsigned long long *ls_kused = nullptr;
    int64_t ls_kcap = 0;
    bool keep_live = false;
    // fold-in: counters [4], list [1], heavy row and first task [2], the
    // row's flag byte; its least-squares triangles go to fold_part
    int32_t *fold_ls = nullptr;
    void *noalloc = nullptr;     // this device's scratch of ptk_fold_in_noalloc
    int32_t last_iters = 0;      // iterations the last ptk_iterate ran
    double *host = nullptr;      // pinned results
    size_t host_cap = 0;
    void *qr_work = nullptr;
    size_t qr_cap = 0;
    double *fold_bbuf = nullptr, *fold_part = nullptr;
    int64_t *fold_rowptr = nullptr;
    int32_t *fold_split = nullptr;
    int64_t fold_part_chunks = 0;
    std::string err;
    std::vector<Timed> pending;
    std::vector<hipEvent_t> pool;
    std::map<std::string, std::pair<int64_t, double>> totals;
};

