// Internal declarations of the gfx950 sparse Tucker ALS library.
//
// Layout of the library's device data (per context):
//  * per mode n, a CSR copy of the observed set grouped by the mode-n index
//    (the sets Omega^(n)_i of Table 2): rowptr[I_n+1] (int64), rows[nnz]
//    (the mode-n index of every entry in grouped order, int32), oidx[N-1][nnz]
//    (the other modes' indices, int32, modes in increasing order) and
//    val[nnz] (float32);
//  * per mode n, the core permuted so that the mode-n index is fastest and
//    the other modes keep their order: gp[n][m_1..m_{N-1}][j_n], in the
//    arithmetic type of the delta kernels;
//  * a row-system buffer bbuf[I_n][E] (float64) with E = J(J+1)/2 + J: the
//    upper triangle of B_i row by row followed by c_i;
//  * per work range, two partial row systems (the range's first row when it
//    began in an earlier range, its last row when it continues past the end).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/ptucker.h"

namespace ptk {

constexpr int kMaxN = 10;
constexpr int kMaxJ = 32;
constexpr int kWave = 64;
constexpr int64_t kMaxCore = int64_t(1) << 20;

constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

// Entries of the packed row system for rank J: upper triangle + rhs.
__host__ __device__ constexpr inline int sys_entries(int J) {
    return J * (J + 1) / 2 + J;
}
// Position of B(p, q), p <= q, in the packed upper triangle (row by row).
__host__ __device__ inline int tri_pos(int p, int q, int J) {
    return p * J - (p * (p - 1)) / 2 + (q - p);
}

// Arguments of the delta / Gram kernels for one mode.
struct GramArgs {
    const void *gp;                   // permuted core of mode n (float or double)
    const float *fac[kMaxN];          // factors of the other modes, mode order
    const int32_t *oidx[kMaxN];       // other-mode index arrays, same order
    int32_t jk[kMaxN];                // ranks of the other modes
    int32_t aoff[kMaxN];              // prefix sums of jk (LDS row offsets)
    int32_t nother;                   // N - 1
    int32_t jn;                       // rank of mode n
    int32_t E;                        // sys_entries(jn)
    const int32_t *rows;              // mode-n index per entry, or null (all 0)
    int32_t skip_row;                 // row id whose sums are discarded (padding), or -1
    const float *val;                 // values in grouped order
    const int64_t *rowptr;            // CSR row pointers of mode n
    int64_t nnz;
    int64_t chunk;                    // entries per work range (multiple of 64)
    double *bbuf;                     // complete rows
    double *part;                     // [nchunks][2][E]
    // per-entry partial-product cache (pairs of modes n, p), records of
    // cache_record_doubles(J) doubles:
    // writer (mode n): cache[pos][m_p][j_n] = G contracted with all modes but
    //   n and p, the partner p being the first of the other modes;
    // reader (mode p): delta_p[m] = sum_j a^(n)_{i_n}[j] cache[cmap[pos]][m][j],
    //   a^(n) being other-mode slot cslot.
    double *cache;
    const int32_t *cmap;
    int32_t cslot;
    // optional (two-entry kernel): the delta of every entry, [jn][nnz] FP64 in
    // the grouped order, kept for the residuals of the Approx variant
    double *dstore;
    // optional: the kernel returns at once when *skip_if != 0 (the mode's
    // sparse-core kernel forms these row systems instead)
    const int32_t *skip_if;
    // optional: deltas kept for the least-squares solve; an entry at pos of
    // row i with kbase[i] != kNoKeep stores its delta at keep[(kbase[i] + pos)
    // * jn ..] (FP64, jn contiguous)
    const int64_t *kbase;
    double *keep;
};

// kbase value of a row whose deltas are not kept.
constexpr int64_t kNoKeep = INT64_MIN;

// Arguments of the per-entry kernels (predict, error, delta inspection).
struct EntryArgs {
    const void *gp;
    const float *fac[kMaxN];
    const int32_t *oidx[kMaxN];
    int32_t jk[kMaxN];
    int32_t aoff[kMaxN];
    int32_t nother;
    int32_t jn;
    const int32_t *own_idx;           // index of the entry in mode n
    const float *own;                 // factor A^(n)
    const float *val;                 // values (error mode)
    int64_t m;                        // number of entries
    float *out;                       // predictions [m] or deltas [m][jn]
    double *partial;                  // per-block partial sums (error mode)
};

enum EntryOut { kOutDelta = 0, kOutPredict = 1, kOutSSE = 2 };

// Arguments of the BF16 matrix-core row-system kernel (ptk_mfma.hip). The
// entries of mode n are cut into blocks of at most 32 entries that never span
// two rows; blk_* describe them in grouped order.
struct MfmaArgs {
    const void *frag;                 // bf16 core fragments [tiles][64][4]
    const float *fac[kMaxN];          // factors of the other modes, mode order
    const int32_t *oidx[kMaxN];       // other-mode index arrays, same order
    const float *val;
    const int64_t *rowptr;
    const int32_t *blk_row;
    const int32_t *blk_start;
    const int32_t *blk_cnt;
    int64_t nblk;
    int64_t blk_per_wave;
    int32_t E;
    double *bbuf;
    double *part;                     // [waves][2][E]
};

// ---------------------------------------------------------------------------
// kernel launchers (ptk_kernels.hip, ptk_sort.hip, ptk_solve.hip)
// ---------------------------------------------------------------------------
struct Shape {
    int N;
    int64_t dims[kMaxN];
    int32_t ranks[kMaxN];
};

// delta precision of the row-system kernels
enum Arith { kArithF64 = 0, kArithF32 = 1 };

// Is there a compiled fast kernel for this (N, J) with equal ranks?
bool fast_available(int N, int J, Arith ar);

// gp[others][j_n] <- G. The other modes are in ascending order, or, with
// lead >= 0, lead first and the rest ascending.
hipError_t launch_permute_core(const float *G, void *gp, const Shape &s, int n,
                               Arith ar, hipStream_t st, int lead = -1);
hipError_t launch_gram(const GramArgs &a, const Shape &s, int n, Arith ar,
                       int64_t nchunks, bool fast, hipStream_t st);
// cache_mode 1 = write the pair cache, 2 = read it (see GramArgs)
bool cache_available(int N, int J);
int cache_record_doubles(int J);    // doubles per entry record of the pair cache
hipError_t launch_gram_cache(const GramArgs &a, const Shape &s, int n, Arith ar,
                             int64_t nchunks, int cache_mode, hipStream_t st);
int gram_cache_blocks_per_cu(const Shape &s, int n, Arith ar, int cache_mode);
int gram_blocks_per_cu(const Shape &s, int n, Arith ar, bool fast);
// two entries per lane (ptk_gram2.hip), equal ranks
bool gram2_available(int N, int J, Arith ar);
int gram2_blocks_per_cu(int N, int J, Arith ar);
hipError_t launch_gram2(const GramArgs &a, int N, int J, Arith ar, int64_t nchunks,
                        hipStream_t st);
hipError_t launch_merge(const double *part, const int32_t *split, int32_t nsplit,
                        int E, double *bbuf, hipStream_t st);
// Rows the Cholesky solve hands to the least-squares solve (ptk_resolve.hip):
// those whose factorisation broke down or whose scaled condition estimate
// tr((D^-1/2 M D^-1/2)^-1), M = B_i + lambda I, D = diag(M), exceeds
// cond_limit. The solve kernel sets rflag[i] (one byte per row) to 1 for
// them and to 0 for the rest; k_ls_lists then sorts the flagged rows by
// length into three lists and rewrites their byte to kLsOwnError (packed and
// single rows, whose error term the least-squares kernel supplies) or
// kLsIdentity (heavy rows):
//  * packed: rows of at most kLsPack entries (with pack set), four per
//    wavefront; list[0, cnt[0]);
//  * single: other rows of at most 64 entries (and rows whose tasks find no
//    room), one wavefront each; list[cap - 1 - k], k < cnt[1];
//  * heavy: longer rows, cut into tasks of task_len entries (any wavefront
//    takes any task) whose triangles a second kernel merges. cnt[2], cnt[3]
//    form one 64-bit counter (tasks in the low word, rows in the high word)
//    that a row advances by (1 << 32) + its tasks in one atomic, so hoff[h],
//    the first task of heavy row h = hrow[h] (-1: no room, skipped), grows
//    with h and a task finds its row by binary search.
// Capacities: cap and hcap >= rows; tcap tasks (the triangles hold tcap).
constexpr int kLsPack = 16;
constexpr int32_t kLsTaskLen = 64;
constexpr size_t kLsTriBytes = size_t(256) << 20;
constexpr double kCondLimitDefault = 1e10;
constexpr size_t kKeepBytes = size_t(512) << 20;   // kept deltas, at most
constexpr uint8_t kLsOwnError = 2;
constexpr uint8_t kLsIdentity = 3;
struct SolveFlags {
    uint8_t *rflag;
    int32_t *cnt;                     // [4], 8-byte aligned
    int32_t *list;
    int64_t cap;
    int32_t *hrow, *hoff;
    int64_t hcap, tcap;
    int32_t task_len;
    int32_t pack;
    double cond_limit;
};
hipError_t launch_solve(const double *bbuf, const int64_t *rowptr, int64_t I,
                        int J, double lambda, float *A, const SolveFlags &f,
                        hipStream_t st);
// the lists of the flagged rows (after launch_solve)
hipError_t launch_ls_lists(const int64_t *rowptr, int64_t I, const SolveFlags &f,
                           hipStream_t st);

// Arguments of the least-squares row solve of the flagged rows (the entries
// of mode n in grouped order, as for the row-system kernels).
struct LsArgs {
    const void *gp;                   // FP64 permuted core of mode n
    const float *fac[kMaxN];
    const int32_t *oidx[kMaxN];
    int32_t jk[kMaxN];
    int32_t aoff[kMaxN];
    int32_t nother;
    int32_t jn;
    const float *val;
    const int64_t *rowptr;
    SolveFlags f;                     // the lists the solve kernel filled
    double *tri;                      // [tcap][jn][jn + 1] triangles of heavy tasks
    double lambda;
    float *A;                         // A^(n): the flagged rows are written
    double *rsse;                     // optional: for packed and single rows i,
                                      // sum over the entries of p (p - 2x),
                                      // p = a_i^T delta (a_i as stored)
    int32_t *stats;                   // [0] rows left unsolved (result not
                                      // finite), [1] rows solved here,
                                      // [2] most entries of such a row
    // optional: the deltas the row-system kernel of this mode update kept
    // (GramArgs::kbase / keep); a row with kbase[i] != kNoKeep reads them
    // instead of recomputing
    const int64_t *kbase;
    const double *keep;
};

// Plan of the kept deltas for the next update of a mode: every row that the
// least-squares form solved in this one (rflag != 0) gets a run of slots,
// one per entry, when all of them fit in kcap entries; else, and for the
// other rows, kNoKeep. With rflag null every row gets kNoKeep. used: a
// device counter of the library (zeroed here).
hipError_t launch_keep_plan(const uint8_t *rflag, const int64_t *rowptr, int64_t I,
                            int64_t kcap, int64_t *kbase, unsigned long long *used,
                            hipStream_t st);
// equal_fast: the (N, J) of an unrolled delta kernel with all ranks J
hipError_t launch_ls(const LsArgs &a, int N, bool equal_fast, int num_cu,
                     hipStream_t st);
// rflag / rsse (optional): rows marked kLsOwnError in rflag add rsse[i]
// instead of the identity of their row system.
hipError_t launch_row_sse(const double *bbuf, const int64_t *rowptr, const float *A,
                          int64_t I, int J, const uint8_t *rflag, const double *rsse,
                          double *partial, int nblocks, hipStream_t st);
hipError_t launch_entries(const EntryArgs &a, const Shape &s, int n, int kind,
                          bool fast, int64_t nblocks, hipStream_t st);
hipError_t launch_sumsq(const float *x, int64_t n, double *partial, int nblocks,
                        hipStream_t st);
hipError_t launch_reduce(const double *partial, int n, double *out,
                         hipStream_t st);
hipError_t launch_expand_systems(const double *bbuf, const int64_t *rowptr,
                                 int64_t I, int J, double *B, double *c,
                                 hipStream_t st);
hipError_t launch_validate(const int32_t *idx, const float *val, int64_t nnz,
                           const Shape &s, unsigned long long *bad,
                           hipStream_t st);

// BF16 matrix-core form (ptk_mfma.hip)
bool mfma_available(int N, int J);
int64_t mfma_tiles(int N, int J);
int mfma_waves_per_cu(int N, int J, int split);
hipError_t launch_mfma_frags(const float *G, void *frag, const Shape &s, int n,
                             hipStream_t st);
hipError_t launch_gram_mfma(const MfmaArgs &a, int N, int J, int split, int64_t nwaves,
                            hipStream_t st);

// sort / CSR build (ptk_sort.hip)
size_t sort_workspace_bytes(int64_t nnz);
hipError_t build_mode_csr(const int32_t *idx, const float *val, int64_t nnz,
                          const Shape &s, int n, void *work, int64_t *rowptr,
                          int32_t *rows, int32_t *oidx, float *vals,
                          hipStream_t st, int32_t *perm_out = nullptr, int sub = -1);
// Unit lists of the shared-index row systems (ptk_sort.hip). A run is a
// maximal sequence of consecutive grouped entries with the same row (unless
// rows is null) and the same index sidx (an other mode's). A run of at least lmin entries (lmin >
// 0) is long: it is listed in lg (its first position, and tasks of at most
// tlen consecutive entries, each naming its long run). Every other run is cut
// into units of emax entries and then at most one unit each of emax/2, ...,
// 2, 1 entries (the binary digits of the rest). units receives the units'
// first positions, classes in the order emax, ..., 1, each in increasing
// position; count[c] is the number of units of class c (2^c entries), c =
// 0..3. A long run below wmin entries (wmin > 0) is not listed as a run:
// its entries are listed one by one (ntask_pos) instead. The workspace holds
// units_workspace_ints int32 values; lg's arrays hold cap_long, cap_tasks and
// cap_ntasks values (hipErrorInvalidValue beyond).
struct UnitLong {
    int32_t *run_pos = nullptr;       // [n_long] first position of each long run
    int32_t *task_pos = nullptr;      // [n_tasks] first position of each task
    int32_t *task_len = nullptr;      // [n_tasks] its entries (<= tlen)
    int32_t *task_run = nullptr;      // [n_tasks] its long run
    int32_t *ntask_pos = nullptr;     // [n_ntasks] the entries of runs below wmin entries
    int64_t n_long = 0, n_tasks = 0, n_ntasks = 0;
    int64_t cap_long = 0, cap_tasks = 0, cap_ntasks = 0;
};
// Stable sort of keys (values below extent) with their positions: keys_out
// sorted, pos_out[k] = the position of keys_out[k]. work: sort_workspace_bytes.
hipError_t sort_by_key(const int32_t *keys, int64_t nnz, int64_t extent, void *work,
                       int32_t *keys_out, int32_t *pos_out, hipStream_t st);
// For runs of equal keys (build_units with rows null): run_pos[r] <- the key
// value of run r.
hipError_t launch_run_keys(const int32_t *keys, const UnitLong &lg, hipStream_t st);
// list[i] <- perm[list[i]] for i < n.
hipError_t launch_permute_list(const int32_t *perm, int32_t *list, int64_t n, hipStream_t st);
int64_t units_workspace_ints(int64_t nnz);
hipError_t build_units(const int32_t *rows, const int32_t *sidx, int64_t nnz, int emax,
                       int32_t lmin, int32_t tlen, int32_t wmin, int32_t *work, int32_t *units,
                       int64_t *count, UnitLong *lg, hipStream_t st);
// inv[perm[i]] = i
hipError_t launch_invert_perm(const int32_t *perm, int64_t nnz, int32_t *inv,
                              hipStream_t st);
// out[i] = inv[perm[i]]
hipError_t launch_compose_perm(const int32_t *inv, const int32_t *perm, int64_t nnz,
                               int32_t *out, hipStream_t st);

// message of the last failed context-free call on this thread (ptk_data.hip)
const char *global_error();

// finalisation (ptk_finalize.hip)
size_t qr_workspace_bytes(int64_t I, int J);
// thin QR by shifted CholeskyQR3: A (I x J, float) <- Q, R (J x J, row-major,
// device) <- R; *bad counts factorisations that failed (rank-deficient A)
hipError_t launch_thin_qr(float *A, int64_t I, int J, void *work, double *R,
                          int32_t *bad, hipStream_t st);
hipError_t launch_core_mode_product(const float *G, float *Gout, const Shape &s,
                                    int n, const double *R, hipStream_t st);

}  // namespace ptk
