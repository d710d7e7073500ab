// Row systems from shared-index units (Alg. 3 with the contraction of eq.
// "delta" reordered): the entries of a row are grouped by their index in the
// last other mode s, and the core contracted with that mode's row,
// t = G x_s a^(s)_{i_s}, is formed once per unit of entries that share i_s
// instead of once per entry. Deltas go to a buffer; a second kernel sweeps
// them into the packed row systems in grouped order, like the other
// row-system kernels.
#pragma once

#include "ptk_internal.h"

namespace ptk {

// Largest unit (entries sharing one t) with a kernel: 8 at orders 3 and 4
// up to J = 10, else 4 (register and LDS footprint).
constexpr int units_emax(int N, int J) { return (J <= 10 && N <= 4) ? 8 : 4; }
// Largest unit by default: the kernels of 4 and 8 entries keep too few
// wavefronts resident to hide the scalar loads of the core, and measured
// slower per entry than pairs on the order-4 and order-5 workloads; long
// runs take most of what they would save.
constexpr int kUnitsDefault = 2;

// Arguments of the unit delta kernel for one class of units.
struct UnitArgs {
    const void *gp;                   // FP64 permuted core of mode n
    const void *gph;                  // the same in pass-major order (launch_core_passes)
    const float *fac[kMaxN];          // factors of the other modes, mode order
    const int32_t *oidx[kMaxN];       // other-mode index arrays, same order
    const int32_t *units;             // first grouped position of each unit
    int64_t count;                    // units in this class
    double *dout;                     // deltas [nnz][J] in grouped order
};

// Long runs: a run of at least kLongRun entries gets its own table
// T[o][j] = sum_m gp[o][m][j] a^(s)[m] (J^(N-1) doubles), formed once, and
// its entries, in tasks of at most kLongTask, read T through the scalar
// cache instead of forming t per unit.
constexpr int32_t kLongRun = 64;
constexpr int32_t kLongTask = 128;
// Tables of one mode beyond this many bytes: no long runs (units only).
constexpr int64_t kLongTableBytes = int64_t(4) << 30;

struct LongArgs {
    const void *gp;                   // FP64 permuted core of mode n
    const float *fac[kMaxN];          // factors of the other modes, mode order
    const int32_t *oidx[kMaxN];       // other-mode index arrays, same order
    UnitLong lg;                      // long runs and their tasks
    double *tab;                      // tables [n_long][J^(N-2)][J]
    double *dout;                     // deltas [nnz][J] in grouped order
    // index tables: table r is that of the index value run_pos[r] of mode s,
    // a task's entries are at grouped positions perm[task_pos ..], and
    // task_run names its table
    int32_t index_tables;
    const int32_t *perm;
};

// Tables of every long run (or index value), then the deltas of every task's
// entries, P entries per lane (tasks of at most P * 64 entries); the two
// steps are also available apart.
hipError_t launch_long_runs(const LongArgs &a, int N, int J, int P, hipStream_t st);
hipError_t launch_run_tables(const LongArgs &a, int N, int J, hipStream_t st);
hipError_t launch_long_tasks(const LongArgs &a, int N, int J, int P, hipStream_t st);

// Index tables: a table per index value of mode s with kIndexTask / 2
// entries or more, T_v = G x_s a^(s)_v, serves every entry of mode n with
// i_s = v, whatever its row. Entries are taken in the order of i_s, in tasks
// of at most kIndexTask of one value (two entries per lane); the entries of
// the other values are single-entry units.
constexpr int32_t kIndexTask = 128;
// Tables of one mode beyond this many bytes: not used.
constexpr int64_t kIndexTableBytes = int64_t(16) << 30;

// (N, J) with equal ranks and unit kernels (FP64 arithmetic).
bool units_available(int N, int J);

// Passes over delta's components of the largest unit class at (N, J) (the
// pass-major core layout that class reads; 1 = none needed).
int units_passes(int N, int J);

// gph <- gp in pass-major order ([pass][outer][m][J / passes]); nothing when
// units_passes(N, J) is 1. gph holds J^N doubles.
hipError_t launch_core_passes(const double *gp, double *gph, int N, int J, hipStream_t st);

// Deltas of every unit of class c (2^c entries) into a.dout.
hipError_t launch_delta_units(const UnitArgs &a, int N, int J, int c, hipStream_t st);

// Row systems of mode n from the stored deltas din ([nnz][J]), over the
// work ranges of a (same chunks, partial slots and merge as launch_gram);
// keeps the deltas of planned least-squares rows when a.kbase is set.
hipError_t launch_gram_stored(const GramArgs &a, int J, const double *din, int64_t nchunks,
                              hipStream_t st);
// Resident single-wave workgroups of the stored-delta sweep per CU.
int gram_stored_blocks_per_cu(int J);

// Multiply-adds per entry of the plain contraction and of one unit of e
// entries (the model that decides whether a mode uses units).
double plain_fma_per_entry(int N, int J);
double unit_fma(int N, int J, int e);
// Multiply-adds of the long-run form: one table per run, then J^(N-1) + J^(N-2)
// per entry.
double long_fma(int N, int J, double runs, double entries);
// The stored-delta sweep of one entry (8 J + 8 bytes read) in multiply-add
// equivalents: 15 FP64 multiply-adds per byte, the ratio of the rates
// measured for the delta kernels (27 T multiply-adds/s) and the sweep
// (1.8 TB/s) on the order-4 workload.
double stored_delta_fma(int J);

}  // namespace ptk
