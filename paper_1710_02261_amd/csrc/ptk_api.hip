// C ABI of the row-wise sparse Tucker ALS library (include/ptucker.h).
//
// Host orchestration only: argument checks, device buffers, the per-mode CSR
// build, the work-range split, and the launch order of Alg. 2 / Alg. 3.
// Every arithmetic step runs in the HIP kernels of this directory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "ptk_approx.h"
#include "ptk_sparse.h"
#include "ptk_context.h"
#include "ptk_internal.h"
#include "ptk_slice.h"
#include "ptk_units.h"

using namespace ptk;

// device address of the scratch of ptk_fold_in_noalloc (defined with it)
hipError_t noalloc_scratch(int device, void **out);

namespace {

ptk_status fail(ptk_ctx *c, ptk_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return s;
}

#define HIPCHK(ctx, x)                                                          \
    do {                                                                        \
        hipError_t e_ = (x);                                                    \
        if (e_ != hipSuccess)                                                   \
            return fail(ctx, PTK_E_HIP, "%s failed: %s", #x,                    \
                        hipGetErrorString(e_));                                 \
    } while (0)

template <typename T>
hipError_t dalloc(T **p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    return hipMalloc((void **)p, count * sizeof(T));
}

void dfree(void *p) {
    if (p) (void)hipFree(p);
}

hipEvent_t get_event(ptk_ctx *c) {
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

// Launch through fn, bracketed by events when profiling.
template <typename F>
hipError_t timed(ptk_ctx *c, const char *name, F fn) {
    if (!c->opt.profile) return fn();
    Timed t{name, get_event(c), get_event(c)};
    (void)hipEventRecord(t.a, c->st);
    hipError_t e = fn();
    (void)hipEventRecord(t.b, c->st);
    c->pending.push_back(t);
    return e;
}

void collect_timers(ptk_ctx *c) {
    if (c->pending.empty()) return;
    (void)hipStreamSynchronize(c->st);
    for (auto &t : c->pending) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, t.a, t.b);
        auto &tot = c->totals[t.name];
        tot.first += 1;
        tot.second += ms;
        c->pool.push_back(t.a);
        c->pool.push_back(t.b);
    }
    c->pending.clear();
}

void free_approx(ptk_ctx *c) {
    dfree(c->ap_resid);
    dfree(c->ap_part);
    dfree(c->ap_R);
    dfree(c->ap_removed);
    dfree(c->ap_uw);
    dfree(c->ap_tbuf);
    dfree(c->ap_delta);
    dfree(c->sp_count);
    dfree(c->sp_cstart);
    dfree(c->sp_use);
    dfree(c->sp_recs);
    c->sp_count = c->sp_cstart = c->sp_use = nullptr;
    c->sp_recs = nullptr;
    c->ap_resid = c->ap_part = c->ap_R = c->ap_uw = c->ap_tbuf = c->ap_delta = nullptr;
    c->ap_removed = nullptr;
    c->ap_slices = 0;
    c->ap_form = 0;
    c->ap_rs_slices = 0;
    c->ap_nfold = 0;
}

void free_modes(ptk_ctx *c) {
    for (int n = 0; n < kMaxN; ++n) {
        ModeData &m = c->md[n];
        dfree(m.rowptr);
        dfree(m.rows);
        dfree(m.oidx);
        dfree(m.vals);
        dfree(m.cmap);
        dfree(m.split);
        dfree(m.blk_row);
        dfree(m.blk_start);
        dfree(m.blk_cnt);
        dfree(m.units);
        dfree(m.lg.run_pos);
        dfree(m.lg.task_pos);
        dfree(m.lg.task_len);
        dfree(m.lg.task_run);
        dfree(m.spos);
        dfree(m.ix.run_pos);
        dfree(m.ix.task_pos);
        dfree(m.ix.task_len);
        dfree(m.ix.task_run);
        dfree(m.ix.ntask_pos);
        m = ModeData();
    }
    dfree(c->bbuf);
    dfree(c->part);
    dfree(c->pcache);
    c->pcache = nullptr;
    dfree(c->dpart);
    c->dpart = nullptr;
    dfree(c->dunits);
    c->dunits = nullptr;
    dfree(c->gph);
    c->gph = nullptr;
    dfree(c->ltab);
    c->ltab = nullptr;
    dfree(c->itab);
    c->itab = nullptr;
    free_approx(c);
    c->bbuf = c->part = nullptr;
    c->part_cap = 0;
    dfree(c->ls_hrow);
    dfree(c->ls_hoff);
    dfree(c->ls_tri);
    c->ls_hrow = c->ls_hoff = nullptr;
    c->ls_tri = nullptr;
    c->ls_hcap = c->ls_tcap = 0;
    dfree(c->ls_kbase);
    dfree(c->ls_keep);
    dfree(c->ls_kused);
    c->ls_kbase = nullptr;
    c->ls_keep = nullptr;
    c->ls_kused = nullptr;
    c->ls_kcap = 0;
    c->keep_live = false;
    c->nnz = -1;
}

Arith arith_of(const ptk_ctx *c, int n) {
    if (!c->md[n].fast) return kArithF64;
    return c->opt.precision == PTK_PREC_FP32 ? kArithF32 : kArithF64;
}

bool equal_ranks(const Shape &s) {
    for (int k = 1; k < s.N; ++k)
        if (s.ranks[k] != s.ranks[0]) return false;
    return true;
}

// The other mode whose index orders the entries inside the rows of mode n
// (the last other mode, the second-fastest index of the permuted core) when
// mode n may use shared-index units, else -1.
int units_sub(const ptk_ctx *c, int n) {
    const Shape &s = c->s;
    if (c->opt.shared_units < 0 || c->opt.pair_cache || !equal_ranks(s) ||
        c->opt.precision == PTK_PREC_BF16 || c->opt.precision == PTK_PREC_BF16X3 ||
        !units_available(s.N, s.ranks[0]))
        return -1;
    return n == s.N - 1 ? s.N - 2 : s.N - 1;
}

// Role of mode n in the pair cache of a full sweep: 1 writes it (modes 2k
// with a partner 2k+1), 2 reads it (modes 2k+1), 0 neither.
int cache_role(const ptk_ctx *c, int n) {
    if (!c->opt.pair_cache) return 0;
    if (n % 2 == 1) return 2;
    return n + 1 < c->s.N ? 1 : 0;
}

ptk_status need_model(ptk_ctx *c) {
    if (c->nnz < 0) return fail(c, PTK_E_STATE, "no observed set (ptk_set_observed)");
    if (!c->core) return fail(c, PTK_E_STATE, "no model bound (ptk_bind_model)");
    return PTK_OK;
}

// A pair-cache writer (role 1) needs its partner as the leading other mode.
hipError_t permute(ptk_ctx *c, int n, int role = 0) {
    if (c->md[n].bf16)
        return timed(c, "permute_core", [&] {
            return launch_mfma_frags(c->core, c->frag[n], c->s, n, c->st);
        });
    return timed(c, "permute_core", [&] {
        return launch_permute_core(c->core, c->gp[n], c->s, n, arith_of(c, n), c->st,
                                   role == 1 ? n + 1 : -1);
    });
}

// The per-entry kernels (error, predict, delta) always read an fp64 core.
hipError_t permute_entries(ptk_ctx *c, int n) {
    return timed(c, "permute_core", [&] {
        return launch_permute_core(c->core, c->gpe, c->s, n, kArithF64, c->st);
    });
}

// Arguments of the delta kernels for mode n over an entry list whose
// other-mode index arrays are other[t] (t over the modes k != n in order).
template <typename Args>
void fill_common(const ptk_ctx *c, int n, Args &a, const int32_t *const *other) {
    a.gp = c->gp[n];
    int t = 0, off = 0;
    for (int k = 0; k < c->s.N; ++k) {
        if (k == n) continue;
        a.fac[t] = c->fac[k];
        a.oidx[t] = other[t];
        a.jk[t] = c->s.ranks[k];
        a.aoff[t] = off;
        off += c->s.ranks[k];
        ++t;
    }
    a.nother = c->s.N - 1;
    a.jn = c->s.ranks[n];
}

GramArgs gram_args(const ptk_ctx *c, int n) {
    const ModeData &m = c->md[n];
    GramArgs a{};
    const int32_t *other[kMaxN];
    for (int t = 0; t < c->s.N - 1; ++t) other[t] = m.oidx + (int64_t)t * c->nnz;
    fill_common(c, n, a, other);
    a.skip_row = -1;
    a.E = sys_entries(c->s.ranks[n]);
    a.rows = m.rows;
    a.val = m.vals;
    a.rowptr = m.rowptr;
    a.nnz = c->nnz;
    a.chunk = m.chunk;
    a.bbuf = c->bbuf;
    a.part = c->part;
    return a;
}

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Pair-cache arguments. Writer n: other-mode slots reordered so that the
// partner n+1 (slot n of the ascending list) leads, as in its permuted core.
// Reader n: the partner n-1 is slot n-1 of the ascending list.
GramArgs cache_args(const ptk_ctx *c, int n, int role) {
    GramArgs a = gram_args(c, n);
    a.cache = c->pcache;
    if (role == 1) {
        const float *f = a.fac[n];
        const int32_t *o = a.oidx[n];
        for (int t = n; t > 0; --t) {
            a.fac[t] = a.fac[t - 1];
            a.oidx[t] = a.oidx[t - 1];
        }
        a.fac[0] = f;
        a.oidx[0] = o;
    } else {
        a.cmap = c->md[n].cmap;
        a.cslot = n - 1;
    }
    return a;
}

MfmaArgs mfma_args(const ptk_ctx *c, int n) {
    const ModeData &m = c->md[n];
    MfmaArgs a{};
    a.frag = c->frag[n];
    int t = 0;
    for (int k = 0; k < c->s.N; ++k) {
        if (k == n) continue;
        a.fac[t] = c->fac[k];
        a.oidx[t] = m.oidx + (int64_t)t * c->nnz;
        ++t;
    }
    a.val = m.vals;
    a.rowptr = m.rowptr;
    a.blk_row = m.blk_row;
    a.blk_start = m.blk_start;
    a.blk_cnt = m.blk_cnt;
    a.nblk = m.nblk;
    a.blk_per_wave = m.blk_per_wave;
    a.E = sys_entries(c->s.ranks[n]);
    a.bbuf = c->bbuf;
    a.part = c->part;
    return a;
}

// Cell lists of the sparse core (Approx variant).
SparseArgs sparse_args(const ptk_ctx *c) {
    SparseArgs sa{};
    sa.N = c->s.N;
    sa.J = c->s.ranks[0];
    sa.cells = c->core_cells;
    sa.rec = c->core_cells + 1;
    sa.count = c->sp_count;
    sa.cstart = c->sp_cstart;
    sa.recs = c->sp_recs;
    sa.use = c->sp_use;
    sa.limit = c->opt.sparse_limit > 0.0 ? c->opt.sparse_limit : kSparseLimitDefault;
    return sa;
}

SparseMode sparse_mode(const ptk_ctx *c, int n) {
    SparseMode sm{};
    const int J = c->s.ranks[0];
    sm.use = c->sp_use + n;
    sm.cstart = c->sp_cstart + (int64_t)n * (J + 1);
    sm.recs = c->sp_recs + (int64_t)n * (c->core_cells + 1) * 4;
    return sm;
}

// Mode n forms its row systems from shared-index units: FP64 arithmetic, no
// pair cache, no Approx variant (whose kernels keep their own deltas).
bool units_live(const ptk_ctx *c, int n) {
    const ModeData &m = c->md[n];
    return (m.units_on || m.ix_on) && c->dunits && m.fast && !m.bf16 && m.slices <= 1 &&
           arith_of(c, n) == kArithF64 && cache_role(c, n) == 0 &&
           !(c->opt.approx_rate > 0.0);
}

// ... and from the index tables of the last other mode (units_live and ix_on).
bool index_live(const ptk_ctx *c, int n) { return units_live(c, n) && c->md[n].ix_on; }

// B_i, c_i for every row of mode n into bbuf (delta + Gram kernel, merge).
ptk_status systems(ptk_ctx *c, int n, int role = 0) {
    const ModeData &m = c->md[n];
    c->keep_live = false;
    if (m.bf16) {
        MfmaArgs a = mfma_args(c, n);
        HIPCHK(c, timed(c, "gram_mfma", [&] {
            return launch_gram_mfma(a, c->s.N, c->s.ranks[n], m.split_bf16, m.nwaves,
                                    c->st);
        }));
        HIPCHK(c, timed(c, "merge", [&] {
            return launch_merge(c->part, m.split, m.nsplit, a.E, c->bbuf, c->st);
        }));
        return PTK_OK;
    }
    if (m.slices > 1 && role != 2) {
        SliceArgs sa{};
        sa.g = role == 1 ? cache_args(c, n, role) : gram_args(c, n);
        sa.dpart = c->dpart;
        sa.nnzp = round_up(c->nnz, kWave);
        sa.S = m.slices;
        sa.sub = role == 1 ? m.slice_sub : m.slices;
        sa.W = m.slice_w;
        sa.writer = role == 1;
        HIPCHK(c, timed(c, "delta_slices", [&] { return launch_delta_slices(sa, c->st); }));
        HIPCHK(c, timed(c, role == 1 ? "gram_cache_write" : "gram", [&] {
            return launch_gram_slices(sa, m.nchunks, c->st);
        }));
        HIPCHK(c, timed(c, "merge", [&] {
            return launch_merge(c->part, m.split, m.nsplit, sa.g.E, c->bbuf, c->st);
        }));
        return PTK_OK;
    }
    if (role) {
        GramArgs a = cache_args(c, n, role);
        HIPCHK(c, timed(c, role == 1 ? "gram_cache_write" : "gram_cache_read", [&] {
            return launch_gram_cache(a, c->s, n, arith_of(c, n), m.nchunks, role, c->st);
        }));
        HIPCHK(c, timed(c, "merge", [&] {
            return launch_merge(c->part, m.split, m.nsplit, a.E, c->bbuf, c->st);
        }));
        return PTK_OK;
    }
    GramArgs a = gram_args(c, n);
    if (units_live(c, n)) {
        UnitArgs ua{};
        ua.gp = a.gp;
        for (int t = 0; t < c->s.N - 1; ++t) {
            ua.fac[t] = a.fac[t];
            ua.oidx[t] = a.oidx[t];
        }
        ua.dout = c->dunits;
        ua.gph = c->gph;
        if (units_passes(c->s.N, c->s.ranks[n]) > 1)
            HIPCHK(c, timed(c, "core_passes", [&] {
                return launch_core_passes((const double *)a.gp, c->gph, c->s.N,
                                          c->s.ranks[n], c->st);
            }));
        static const char *const names[4] = {"delta_units1", "delta_units2", "delta_units4",
                                             "delta_units8"};
        if (m.ix_on) {
            LongArgs la{};
            la.gp = a.gp;
            for (int t = 0; t < c->s.N - 1; ++t) {
                la.fac[t] = a.fac[t];
                la.oidx[t] = a.oidx[t];
            }
            la.lg = m.ix;                  // a table per value with tasks
            la.tab = c->itab;
            la.dout = c->dunits;
            la.index_tables = 1;
            la.perm = m.spos;
            la.lg.n_ntasks = 0;
            HIPCHK(c, timed(c, "index_tables", [&] {
                return launch_run_tables(la, c->s.N, c->s.ranks[n], c->st);
            }));
            HIPCHK(c, timed(c, "delta_index", [&] {
                return launch_long_tasks(la, c->s.N, c->s.ranks[n], kIndexTask / kWave, c->st);
            }));
            if (m.ix.n_ntasks > 0) {
                // the entries of values with fewer than kIndexTask / 2 entries
                UnitArgs ub = ua;
                ub.units = m.ix.ntask_pos;
                ub.count = m.ix.n_ntasks;
                HIPCHK(c, timed(c, "delta_units1", [&] {
                    return launch_delta_units(ub, c->s.N, c->s.ranks[n], 0, c->st);
                }));
            }
        } else if (m.lg.n_long > 0) {
            LongArgs la{};
            la.gp = a.gp;
            for (int t = 0; t < c->s.N - 1; ++t) {
                la.fac[t] = a.fac[t];
                la.oidx[t] = a.oidx[t];
            }
            la.lg = m.lg;
            la.tab = c->ltab;
            la.dout = c->dunits;
            HIPCHK(c, timed(c, "delta_long", [&] {
                return launch_long_runs(la, c->s.N, c->s.ranks[n], 2, c->st);
            }));
        }
        for (int cl = 3; cl >= 0 && !m.ix_on; --cl) {
            if (m.ucount[cl] == 0) continue;
            ua.units = m.units + m.ubase[cl];
            ua.count = m.ucount[cl];
            HIPCHK(c, timed(c, names[cl], [&] {
                return launch_delta_units(ua, c->s.N, c->s.ranks[n], cl, c->st);
            }));
        }
        c->keep_live = c->ls_keep != nullptr;
        if (c->keep_live) {
            a.kbase = c->ls_kbase + c->kb_off[n];
            a.keep = c->ls_keep;
        }
        HIPCHK(c, timed(c, "gram_stored", [&] {
            return launch_gram_stored(a, c->s.ranks[n], c->dunits, m.nchunks, c->st);
        }));
        HIPCHK(c, timed(c, "merge", [&] {
            return launch_merge(c->part, m.split, m.nsplit, a.E, c->bbuf, c->st);
        }));
        return PTK_OK;
    }
    const bool two = m.fast && m.two && gram2_available(c->s.N, c->s.ranks[n], arith_of(c, n));
    if (two && c->ap_store && c->ap_delta) {
        a.dstore = c->ap_delta;
        c->ap_stored = true;
    }
    // Approx variant on a sparse core: both kernels are launched and the
    // device-side switch of the mode lets one of them run
    const bool sparse = c->sp_live && arith_of(c, n) == kArithF64;
    if (sparse) a.skip_if = c->sp_use + n;
    // the FP64 unrolled kernels (and the sparse one) keep the deltas of the
    // rows the plan names for the least-squares solve
    c->keep_live = c->ls_keep && arith_of(c, n) == kArithF64 && (two || m.fast);
    if (c->keep_live) {
        a.kbase = c->ls_kbase + c->kb_off[n];
        a.keep = c->ls_keep;
    }
    HIPCHK(c, timed(c, "gram", [&] {
        if (two)
            return launch_gram2(a, c->s.N, c->s.ranks[n], arith_of(c, n), m.nchunks, c->st);
        return launch_gram(a, c->s, n, arith_of(c, n), m.nchunks, m.fast, c->st);
    }));
    if (sparse)
        HIPCHK(c, timed(c, "gram_sparse", [&] {
            return launch_gram_sparse(a, c->s.N, c->s.ranks[n], sparse_mode(c, n), m.nchunks,
                                      c->st);
        }));
    HIPCHK(c, timed(c, "merge", [&] {
        return launch_merge(c->part, m.split, m.nsplit, a.E, c->bbuf, c->st);
    }));
    return PTK_OK;
}

// The FP64 permuted core of mode n in the default order (the other modes
// ascending, j_n fastest) for the least-squares solve: the row-system core
// itself when it has that form, else the per-entry kernels' copy.
hipError_t ls_core(ptk_ctx *c, int n, int role, const void **gp) {
    if (!c->md[n].bf16 && arith_of(c, n) == kArithF64 && role != 1) {
        *gp = c->gp[n];
        return hipSuccess;
    }
    *gp = c->gpe;
    return permute_entries(c, n);
}

// Cholesky solve of every row of mode n; the rows it flags (breakdown or a
// large condition estimate) are then solved in least-squares form from their
// entries. want_rsse: keep those rows' error terms for the fused error.
ptk_status update_mode_impl(ptk_ctx *c, int n, double lambda, int role = 0,
                            bool want_rsse = false) {
    ptk_status s = systems(c, n, role);
    if (s != PTK_OK) return s;
    const ModeData &m = c->md[n];
    SolveFlags f{};
    f.rflag = c->rflag;
    f.cnt = c->ctr + 4 + 4 * n;
    f.list = c->lslist;
    f.cap = c->max_rows;
    f.hrow = c->ls_hrow;
    f.hoff = c->ls_hoff;
    f.hcap = c->ls_hcap;
    f.tcap = c->ls_tcap;
    f.task_len = kLsTaskLen;
    f.pack = c->s.ranks[n] < kLsPack;
    f.cond_limit = c->opt.cond_limit > 0.0 ? c->opt.cond_limit : kCondLimitDefault;
    HIPCHK(c, timed(c, "solve", [&] {
        return launch_solve(c->bbuf, m.rowptr, c->s.dims[n], c->s.ranks[n], lambda,
                            c->fac[n], f, c->st);
    }));
    HIPCHK(c, timed(c, "solve_ls", [&] {
        return launch_ls_lists(m.rowptr, c->s.dims[n], f, c->st);
    }));
    LsArgs r{};
    HIPCHK(c, ls_core(c, n, role, &r.gp));
    int t = 0, off = 0;
    for (int k = 0; k < c->s.N; ++k) {
        if (k == n) continue;
        r.fac[t] = c->fac[k];
        r.oidx[t] = m.oidx + (int64_t)t * c->nnz;
        r.jk[t] = c->s.ranks[k];
        r.aoff[t] = off;
        off += c->s.ranks[k];
        ++t;
    }
    r.nother = c->s.N - 1;
    r.jn = c->s.ranks[n];
    r.val = m.vals;
    r.rowptr = m.rowptr;
    r.f = f;
    r.tri = c->ls_tri;
    r.lambda = lambda;
    r.A = c->fac[n];
    r.rsse = want_rsse ? c->rsse : nullptr;
    r.stats = c->ctr;
    if (c->keep_live) {
        r.kbase = c->ls_kbase + c->kb_off[n];
        r.keep = c->ls_keep;
    }
    const bool fast = equal_ranks(c->s) && fast_available(c->s.N, c->s.ranks[n], kArithF64);
    HIPCHK(c, timed(c, "solve_ls", [&] {
        return launch_ls(r, c->s.N, fast, c->num_cu, c->st);
    }));
    // the rows solved in least-squares form now keep their deltas in the
    // next update of this mode
    if (c->ls_keep)
        HIPCHK(c, timed(c, "solve_ls", [&] {
            return launch_keep_plan(c->rflag, m.rowptr, c->s.dims[n], c->ls_kcap,
                                    c->ls_kbase + c->kb_off[n], c->ls_kused, c->st);
        }));
    return PTK_OK;
}

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_f64(double *p, double v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// dres[2k .. 2k+1] = scal[0..1] with k = (*ctr)++ (one thread; stream-ordered)
__global__ void k_store_iter(const double *scal, double *dres, int32_t *ctr) {
    if (threadIdx.x == 0) {
        const int k = *ctr;
        dres[2 * k] = scal[0];
        dres[2 * k + 1] = scal[1];
        *ctr = k + 1;
    }
}

// partial[n] = *x (appends one term to a list of partial sums)
__global__ void k_add_scalar(double *partial, int n, const double *x) {
    if (threadIdx.x == 0) partial[n] = *x;
}

// All counters (call start) / the per-mode list counters (iteration start).
hipError_t zero_bad(ptk_ctx *c) {
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, c->st, c->ctr, 0,
                       (int64_t)kCtrSlots);
    return hipGetLastError();
}

hipError_t zero_lists(ptk_ctx *c) {
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, c->st, c->ctr + 4, 0,
                       (int64_t)4 * c->s.N);
    return hipGetLastError();
}

ptk_status ensure_host(ptk_ctx *c, size_t doubles) {
    if (doubles <= c->host_cap) return PTK_OK;
    if (c->host) (void)hipHostFree(c->host);
    c->host = nullptr;
    c->host_cap = 0;
    HIPCHK(c, hipHostMalloc((void **)&c->host, doubles * sizeof(double)));
    c->host_cap = doubles;
    return PTK_OK;
}

__global__ void k_fill_f64(double *p, double v, int64_t n);

// sum over n of ||A^(n)||_F^2 into *out (device).
hipError_t factor_norms(ptk_ctx *c, double *partial, double *out) {
    for (int n = 0; n < c->s.N; ++n) {
        hipError_t e = launch_sumsq(c->fac[n], c->s.dims[n] * c->s.ranks[n],
                                    partial + (int64_t)n * kRedBlocks, kRedBlocks,
                                    c->st);
        if (e != hipSuccess) return e;
    }
    return launch_reduce(partial, c->s.N * kRedBlocks, out, c->st);
}

// SSE of the bound model over Omega via the per-entry kernel on mode 0.
hipError_t sse_direct(ptk_ctx *c, double *partial, double *out) {
    const ModeData &m = c->md[0];
    EntryArgs a{};
    const int32_t *other[kMaxN];
    for (int t = 0; t < c->s.N - 1; ++t) other[t] = m.oidx + (int64_t)t * c->nnz;
    fill_common(c, 0, a, other);
    a.gp = c->gpe;
    a.own_idx = m.rows;
    a.own = c->fac[0];
    a.val = m.vals;
    a.m = c->nnz;
    a.partial = partial;
    hipError_t e = permute_entries(c, 0);
    if (e != hipSuccess) return e;
    const int64_t nb = std::max<int64_t>(
        1, std::min<int64_t>(kSseBlocks, (c->nnz + kWave - 1) / kWave));
    if (c->nnz == 0) {
        hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, c->st, partial, 0.0,
                           (int64_t)1);
        e = hipGetLastError();
    } else {
        e = launch_entries(a, c->s, 0, kOutSSE, m.fast, nb, c->st);
    }
    if (e != hipSuccess) return e;
    return launch_reduce(partial, (int)nb, out, c->st);
}

ptk_status check_bad(ptk_ctx *c, const char *what) {
    int32_t v[3] = {0, 0, 0};
    HIPCHK(c, hipMemcpyAsync(v, c->ctr, sizeof v, hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    c->last_not_pd = v[0];
    c->last_ls_rows = v[1];
    c->last_ls_max = v[2];
    if (v[0] > 0)
        return fail(c, PTK_E_NOT_PD, "%s: %d row(s) or factor(s) could not be solved", what,
                    v[0]);
    return PTK_OK;
}

// Default work per wavefront: one round of resident wavefronts covers the mode.
int64_t default_work(const ptk_ctx *c, int n) {
    const ModeData &m = c->md[n];
    if (m.bf16) {
        const int64_t waves = (int64_t)c->num_cu *
                              mfma_waves_per_cu(c->s.N, c->s.ranks[n], m.split_bf16);
        return std::max<int64_t>(1, (m.nblk + waves - 1) / std::max<int64_t>(waves, 1));
    }
    const int role = cache_role(c, n);
    const int bpc = units_live(c, n) ? gram_stored_blocks_per_cu(c->s.ranks[n])
                    : (m.slices > 1 && role != 2)
                        ? gram_slices_blocks_per_cu(c->s.ranks[n])
                    : role ? gram_cache_blocks_per_cu(c->s, n, arith_of(c, n), role)
                    : (m.fast && m.two && gram2_available(c->s.N, c->s.ranks[n], arith_of(c, n)))
                        ? gram2_blocks_per_cu(c->s.N, c->s.ranks[n], arith_of(c, n))
                        : gram_blocks_per_cu(c->s, n, arith_of(c, n), m.fast);
    const int64_t waves = (int64_t)c->num_cu * std::max(1, bpc);
    int64_t chunk = round_up((c->nnz + waves - 1) / std::max<int64_t>(waves, 1), kWave);
    return std::max<int64_t>(chunk, kWave);
}

// Shared-index units of every mode whose rows are ordered for them, the
// decision per mode (shared_units: 0 = by the work model, else always) and
// the delta buffer. Called by ptk_set_observed after the grouping.
ptk_status build_unit_lists(ptk_ctx *c) {
    const Shape &s = c->s;
    const int64_t nnz = c->nnz;
    if (nnz <= 0 || units_sub(c, 0) < 0) return PTK_OK;
    const int J = s.ranks[0];
    const int su = c->opt.shared_units;
    const int emax = (su >= 2 && su <= 8) ? std::min(su, units_emax(s.N, J)) : kUnitsDefault;
    int64_t inner = 1;                          // J^(N-1): one long run's table
    for (int n = 1; n < s.N; ++n) inner *= s.ranks[n];
    int32_t *work = nullptr;
    HIPCHK(c, dalloc(&work, (size_t)units_workspace_ints(nnz)));
    bool any = false;
    int64_t tab_need = 0, itab_need = 0;
    for (int n = 0; n < s.N; ++n) {
        ModeData &m = c->md[n];
        UnitLong &lg = m.lg;
        lg.cap_long = nnz / kLongRun + 1;
        lg.cap_tasks = nnz / kLongTask + lg.cap_long + 1;
        hipError_t e = dalloc(&m.units, nnz + 64);
        if (e == hipSuccess) e = dalloc(&lg.run_pos, (size_t)lg.cap_long);
        if (e == hipSuccess) e = dalloc(&lg.task_pos, (size_t)lg.cap_tasks);
        if (e == hipSuccess) e = dalloc(&lg.task_len, (size_t)lg.cap_tasks);
        if (e == hipSuccess) e = dalloc(&lg.task_run, (size_t)lg.cap_tasks);
        const int32_t *sidx = m.oidx + (int64_t)(s.N - 2) * nnz;
        if (e == hipSuccess)
            e = build_units(m.rows, sidx, nnz, emax, kLongRun, kLongTask, 0, work, m.units,
                            m.ucount, &lg, c->st);
        // tables beyond their budget: units only
        if (e == hipSuccess && lg.n_long * inner * 8 > kLongTableBytes)
            e = build_units(m.rows, sidx, nnz, emax, 0, kLongTask, 0, work, m.units, m.ucount,
                            &lg, c->st);
        if (e != hipSuccess) {
            dfree(work);
            free_modes(c);
            return fail(c, e == hipErrorOutOfMemory ? PTK_E_NOMEM : PTK_E_HIP,
                        "unit lists of mode %d: %s", n, hipGetErrorString(e));
        }
        int64_t at = 0, in_units = 0;
        double f_units = 0.0;
        for (int cl = 3; cl >= 0; --cl) {
            m.ubase[cl] = at;
            at += m.ucount[cl];
            in_units += m.ucount[cl] << cl;
            f_units += (double)m.ucount[cl] * unit_fma(s.N, J, 1 << cl);
        }
        f_units += long_fma(s.N, J, (double)lg.n_long, (double)(nnz - in_units));
        f_units += (double)nnz * stored_delta_fma(J);
        const double f_plain = (double)nnz * plain_fma_per_entry(s.N, J);
        // index tables: entries in the order of i_s, groups of one value
        const int sub = units_sub(c, n);
        const int64_t Is = s.dims[sub];
        // tables only for the values with kIndexTask / 2 entries or more
        const int64_t wide_max = std::min<int64_t>(Is, nnz / (kIndexTask / 2));
        const bool ix_fits = wide_max * inner * 8 <= kIndexTableBytes;
        double f_index = 1e300;
        if (ix_fits && su != 1 && !(su >= 2 && su <= 8)) {
            UnitLong &ix = m.ix;
            ix.cap_long = std::min<int64_t>(nnz, Is) + 1;
            ix.cap_tasks = nnz / kIndexTask + ix.cap_long + 1;
            ix.cap_ntasks = nnz;                  // the entries of the small values
            int32_t *skeys = nullptr;
            void *swork = nullptr;
            e = dalloc(&m.spos, nnz + 64);
            if (e == hipSuccess) e = dalloc(&skeys, nnz + 64);
            if (e == hipSuccess) e = hipMalloc(&swork, sort_workspace_bytes(nnz));
            if (e == hipSuccess) e = dalloc(&ix.run_pos, (size_t)ix.cap_long);
            if (e == hipSuccess) e = dalloc(&ix.task_pos, (size_t)ix.cap_tasks);
            if (e == hipSuccess) e = dalloc(&ix.task_len, (size_t)ix.cap_tasks);
            if (e == hipSuccess) e = dalloc(&ix.task_run, (size_t)ix.cap_tasks);
            if (e == hipSuccess) e = dalloc(&ix.ntask_pos, (size_t)ix.cap_ntasks);
            if (e == hipSuccess) e = sort_by_key(sidx, nnz, Is, swork, skeys, m.spos, c->st);
            int64_t none[4];
            if (e == hipSuccess)
                e = build_units(nullptr, skeys, nnz, 1, 1, kIndexTask, kIndexTask / 2, work,
                                m.units, none,
                                &ix, c->st);
            // tables for the values with tasks only: run r names its value
            if (e == hipSuccess) e = launch_run_keys(skeys, ix, c->st);
            // entries of values with few entries: grouped positions, for the
            // single-entry unit kernel
            if (e == hipSuccess) e = launch_permute_list(m.spos, ix.ntask_pos, ix.n_ntasks, c->st);
            if (e == hipSuccess) e = hipStreamSynchronize(c->st);
            dfree(skeys);
            if (swork) (void)hipFree(swork);
            if (e != hipSuccess) {
                dfree(work);
                free_modes(c);
                return fail(c, e == hipErrorOutOfMemory ? PTK_E_NOMEM : PTK_E_HIP,
                            "index groups of mode %d: %s", n, hipGetErrorString(e));
            }
            f_index = (double)ix.n_long * (double)inner * J +
                      (double)(ix.n_tasks * kIndexTask) * (double)(inner + inner / J) +
                      (double)ix.n_ntasks * unit_fma(s.N, J, 1) +
                      (double)nnz * stored_delta_fma(J);
        }
        m.ix_on = ix_fits && (su == 16 || (su == 0 && f_index <= 0.9 * f_plain &&
                                           f_index <= f_units));
        m.units_on = !m.ix_on && (su != 0 || f_units <= 0.9 * f_plain);
        any = any || m.units_on || m.ix_on;
        if (m.units_on) tab_need = std::max(tab_need, lg.n_long * inner);
        if (m.ix_on) itab_need = std::max(itab_need, m.ix.n_long * inner);
    }
    dfree(work);
    int64_t cells = 1;
    for (int n = 0; n < s.N; ++n) cells *= s.ranks[n];
    if (any && (dalloc(&c->dunits, (size_t)nnz * J) != hipSuccess ||
                dalloc(&c->gph, (size_t)cells) != hipSuccess ||
                (tab_need > 0 && dalloc(&c->ltab, (size_t)tab_need) != hipSuccess) ||
                (itab_need > 0 && dalloc(&c->itab, (size_t)itab_need) != hipSuccess))) {
        dfree(c->dunits);
        dfree(c->gph);
        dfree(c->ltab);
        c->dunits = nullptr;
        c->gph = nullptr;
        c->ltab = nullptr;
        c->itab = nullptr;
        if (su != 0) {
            free_modes(c);
            return fail(c, PTK_E_NOMEM, "shared-index deltas: %.2f GB of device memory",
                        (nnz * J + tab_need) * 8e-9);
        }
        for (int n = 0; n < s.N; ++n) c->md[n].units_on = c->md[n].ix_on = false;
    }
    return PTK_OK;
}

// Cut mode n into wavefront work ranges of `work` entries (FP64/FP32 path,
// a multiple of 64) or `work` blocks (BF16 path); 0 picks the default. Lists
// the rows that cross ranges for the merge and grows the partial buffer.
ptk_status configure_ranges(ptk_ctx *c, int n, int64_t work) {
    ModeData &m = c->md[n];
    const int E = sys_entries(c->s.ranks[n]);
    if (work <= 0) work = default_work(c, n);
    const std::vector<int64_t> &rp = m.rp_host;
    std::vector<int32_t> split;
    int64_t ranges;
    if (m.bf16) {
        m.blk_per_wave = work;
        m.nwaves = (m.nblk + work - 1) / work;
        ranges = m.nwaves;
        for (int64_t r = 0; r < c->s.dims[n]; ++r) {
            if (m.first_blk[r] < 0) continue;
            const int64_t w0 = m.first_blk[r] / work, w1 = m.last_blk[r] / work;
            if (w0 != w1) {
                split.push_back((int32_t)r);
                split.push_back((int32_t)w0);
                split.push_back((int32_t)w1);
            }
        }
    } else {
        work = round_up(work, kWave);
        m.chunk = work;
        m.nchunks = (c->nnz + work - 1) / work;
        ranges = m.nchunks;
        for (int64_t r = 0; r < c->s.dims[n]; ++r) {
            if (rp[r] == rp[r + 1]) continue;
            const int64_t c0 = rp[r] / work, c1 = (rp[r + 1] - 1) / work;
            if (c0 != c1) {
                split.push_back((int32_t)r);
                split.push_back((int32_t)c0);
                split.push_back((int32_t)c1);
            }
        }
    }
    dfree(m.split);
    m.split = nullptr;
    m.nsplit = (int32_t)(split.size() / 3);
    if (m.nsplit > 0) {
        HIPCHK(c, dalloc(&m.split, split.size()));
        HIPCHK(c, hipMemcpy(m.split, split.data(), split.size() * 4, hipMemcpyHostToDevice));
    }
    const int64_t need = ranges * 2 * E;
    if (need > c->part_cap) {
        dfree(c->part);
        c->part = nullptr;
        c->part_cap = 0;
        HIPCHK(c, dalloc(&c->part, need));
        c->part_cap = need;
    }
    c->epoch++;
    return PTK_OK;
}

// Buffers of the Approx variant, sized for the observed set (not inside a
// graph capture).
// The mode whose rows group the entries of the partial errors: the one with
// the fewest rows (fewest folds); among equals the last one, whose row-system
// kernel runs last in an iteration and can keep its deltas.
int approx_mode(const ptk_ctx *c) {
    int g = c->s.N - 1;
    for (int n = c->s.N - 2; n >= 0; --n)
        if (c->s.dims[n] < c->s.dims[g]) g = n;
    return g;
}

ptk_status ensure_approx(ptk_ctx *c) {
    const int N = c->s.N, J = c->s.ranks[0];
    if (!(equal_ranks(c->s) && approx_available(N, J)))
        return fail(c, PTK_E_UNSUPPORTED, "no Approx kernels for this shape");
    // form: row sums where compiled, when the row pieces average at least
    // 20 entries and the buffers take at most a quarter of the free device
    // memory (or when asked for), else per-cell groups. Each slot costs
    // 2 J^(N-1) doubles written and read again, which the row sums' faster
    // per-entry loop (19 against 4.5 TFLOP/s) repays from about 20 entries on.
    int form = 1;
    int64_t rs_slices = 0, tdoubles = 0, udoubles = 0;
    if (c->opt.approx_form != 1 && row_sums_available(N, J)) {
        rs_slices = row_sums_slices(c->s, c->nnz, c->num_cu);
        const int64_t slots = c->s.dims[approx_mode(c)] + rs_slices;
        tdoubles = row_sums_tbuf_doubles(c->s, approx_mode(c), rs_slices);
        udoubles = std::max<int64_t>(c->nnz, 1) * 2 * J;
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = 0;
        const double need = 8.0 * (double)(tdoubles + udoubles);
        if (c->opt.approx_form == 2 ||
            (need <= 0.25 * (double)free_b && 20.0 * (double)slots <= (double)c->nnz))
            form = 2;
    } else if (c->opt.approx_form == 2) {
        return fail(c, PTK_E_UNSUPPORTED, "no row-sum form of the partial errors for this shape");
    }
    if (c->ap_R && c->ap_form == form) return PTK_OK;
    if (c->ap_R) free_approx(c);
    c->ap_slices = approx_slices(c->s, c->nnz, c->num_cu);
    int64_t ranges = c->ap_slices;
    if (form == 2) {
        c->ap_rs_slices = rs_slices;
        c->ap_nfold = (int32_t)std::min<int64_t>(256, c->s.dims[approx_mode(c)] + rs_slices);
        ranges = std::max<int64_t>(ranges, c->ap_nfold);
        HIPCHK(c, dalloc(&c->ap_uw, (size_t)udoubles));
        HIPCHK(c, dalloc(&c->ap_tbuf, (size_t)tdoubles));
    }
    if (approx_mode(c) == N - 1 && gram2_available(N, J, kArithF64)) {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = 0;
        const double need = 8.0 * (double)J * (double)std::max<int64_t>(c->nnz, 1);
        if (need <= 0.25 * (double)free_b)
            HIPCHK(c, dalloc(&c->ap_delta, (size_t)J * std::max<int64_t>(c->nnz, 1)));
    }
    if (sparse_available(N, J)) {
        HIPCHK(c, dalloc(&c->sp_count, (size_t)N * J));
        HIPCHK(c, dalloc(&c->sp_cstart, (size_t)N * (J + 1)));
        HIPCHK(c, dalloc(&c->sp_use, (size_t)N));
        HIPCHK(c, hipMemsetAsync(c->sp_use, 0, (size_t)N * sizeof(int32_t), c->st));
        HIPCHK(c, dalloc(&c->sp_recs, (size_t)N * (c->core_cells + 1) * 4));
    }
    HIPCHK(c, dalloc(&c->ap_resid, (size_t)c->nnz + 64));
    HIPCHK(c, dalloc(&c->ap_part, (size_t)approx_part_doubles(c->s, (int32_t)ranges)));
    HIPCHK(c, dalloc(&c->ap_R, (size_t)c->core_cells));
    HIPCHK(c, dalloc(&c->ap_removed, 1));
    c->ap_form = form;
    c->epoch++;
    return PTK_OK;
}

// Alg. 4 on the bound model: residuals over the grouping of mode g
// (approx_mode), from the deltas the last mode's kernel kept in this
// iteration when deltas_kept and g is that mode, else by a full contraction;
// R(beta) of every cell into ap_R; with remove, the removal of the top cells
// from the bound core followed by fresh permuted cores. Kernels only
// (capturable).
ptk_status approx_step(ptk_ctx *c, double p, bool remove, bool deltas_kept = false) {
    const int N = c->s.N;
    const int g = approx_mode(c);
    const ModeData &m = c->md[g];
    EntryArgs ea{};
    const int32_t *other[kMaxN];
    for (int t = 0; t < N - 1; ++t) other[t] = m.oidx + (int64_t)t * c->nnz;
    fill_common(c, g, ea, other);
    ea.gp = c->gpe;
    ea.own_idx = m.rows;
    ea.own = c->fac[g];
    ea.val = m.vals;
    ea.m = c->nnz;
    ea.partial = c->ap_resid;
    HIPCHK(c, permute_entries(c, g));
    const int64_t nb = std::max<int64_t>(
        1, std::min<int64_t>(kSseBlocks, (c->nnz + kWave - 1) / kWave));
    const bool kept = deltas_kept && g == N - 1;
    // with the row sums, the kept-delta pass also writes their weights
    const bool fused = kept && c->ap_form == 2;
    HIPCHK(c, timed(c, kept ? "approx_resid_kept" : "approx_resid", [&] {
        // g is the last mode and its kernel kept the deltas of this iteration
        if (fused)
            return launch_resid_uw_from_delta(c->ap_delta, c->fac[g], m.rows, m.vals,
                                              c->fac[N - 4 < g ? N - 4 : N - 3],
                                              other[N - 4], c->nnz, c->s.ranks[g],
                                              c->ap_resid, c->ap_uw, c->st);
        if (kept)
            return launch_resid_from_delta(c->ap_delta, c->fac[g], m.rows, m.vals, c->nnz,
                                           c->s.ranks[g], c->ap_resid, c->st);
        return launch_residual(ea, c->s, nb, c->st);
    }));
    if (c->ap_form == 2) {
        RowSumArgs ra{};
        for (int t = 0; t < N - 1; ++t) {
            ra.fac[t] = c->fac[t < g ? t : t + 1];
            ra.idx[t] = other[t];
        }
        ra.fac_g = c->fac[g];
        ra.rows = m.rows;
        ra.rowptr = m.rowptr;
        ra.resid = c->ap_resid;
        ra.uw = c->ap_uw;
        ra.uw_ready = fused ? 1 : 0;
        ra.tbuf = c->ap_tbuf;
        ra.g = g;
        ra.nrows = c->s.dims[g];
        ra.nnz = c->nnz;
        ra.nslices = c->ap_rs_slices;
        ra.slice = std::max<int64_t>(1, (c->nnz + ra.nslices - 1) / ra.nslices);
        ra.nslots = ra.nrows + ra.nslices;
        ra.nfold = c->ap_nfold;
        ra.fold_per = (ra.nslots + ra.nfold - 1) / ra.nfold;
        ra.part = c->ap_part;
        HIPCHK(c, timed(c, "approx_partial", [&] { return launch_row_sums(ra, c->s, c->st); }));
        HIPCHK(c, timed(c, "approx_reduce", [&] {
            return launch_partial_reduce(c->ap_part, ra.nfold, c->core, c->core_cells,
                                         c->ap_R, c->st);
        }));
    } else {
        ApproxArgs aa{};
        for (int t = 0; t < N - 1; ++t) {
            aa.fac[t] = c->fac[t < g ? t : t + 1];
            aa.idx[t] = other[t];
        }
        aa.fac_g = c->fac[g];
        aa.rows = m.rows;
        aa.g = g;
        aa.resid = c->ap_resid;
        aa.nnz = c->nnz;
        aa.nslices = c->ap_slices;
        aa.slice = std::max<int64_t>(1, (c->nnz + c->ap_slices - 1) / c->ap_slices);
        aa.part = c->ap_part;
        HIPCHK(c, timed(c, "approx_partial",
                        [&] { return launch_partial_error(aa, c->s, c->st); }));
        HIPCHK(c, timed(c, "approx_reduce", [&] {
            return launch_partial_reduce(c->ap_part, c->ap_slices, c->core, c->core_cells,
                                         c->ap_R, c->st);
        }));
    }
    if (remove) {
        HIPCHK(c, timed(c, "approx_select", [&] {
            return launch_approx_select(c->ap_R, c->core, c->core_cells, p,
                                        c->ap_removed, c->st);
        }));
        for (int n = 0; n < N; ++n) HIPCHK(c, permute(c, n, cache_role(c, n)));
    }
    return PTK_OK;
}

// One iteration of Alg. 2 as stream-ordered kernels only: the
// N mode updates, the error and the factor norms, stored to dres through the
// device counter. Contains no memset, copy or synchronisation, so it can be
// captured into a graph and replayed.
ptk_status iteration_body(ptk_ctx *c, double lambda) {
    const int N = c->s.N;
    double *partial = c->red;
    double *scal = c->scal;
    // Approx variant: the last mode's kernel may keep its deltas for the
    // residuals (when the partial errors group by that mode)
    c->ap_stored = false;
    HIPCHK(c, zero_lists(c));
    // Approx variant: lists of the core's non-zero cells as it stands after
    // the last removal, and the switch to the sparse-core kernels
    c->sp_live = false;
    if (c->opt.approx_rate > 0.0 && c->sp_recs && c->opt.sparse_limit >= 0.0) {
        const SparseArgs sa = sparse_args(c);
        HIPCHK(c, timed(c, "sparse_lists", [&] { return launch_sparse_lists(c->core, sa, c->st); }));
        c->sp_live = true;
    }
    c->sp_lists = c->sp_live;
    for (int n = 0; n < N; ++n) {
        c->ap_store = c->opt.approx_rate > 0.0 && n == N - 1;
        ptk_status s = update_mode_impl(c, n, lambda, cache_role(c, n),
                                        n == N - 1 && c->opt.fuse_error);
        c->ap_store = false;
        if (s != PTK_OK) {
            c->sp_live = false;
            return s;
        }
    }
    c->sp_live = false;
    HIPCHK(c, timed(c, "error", [&]() -> hipError_t {
        if (c->opt.fuse_error) {
            // from the last mode's row systems, still in bbuf
            const ModeData &m = c->md[N - 1];
            hipError_t e = launch_row_sse(c->bbuf, m.rowptr, c->fac[N - 1],
                                          c->s.dims[N - 1], c->s.ranks[N - 1], c->rflag,
                                          c->rsse, partial, kRedBlocks, c->st);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(k_add_scalar, dim3(1), dim3(64), 0, c->st, partial,
                               kRedBlocks, c->xsq);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            return launch_reduce(partial, kRedBlocks + 1, scal, c->st);
        }
        return sse_direct(c, partial, scal);
    }));
    HIPCHK(c, timed(c, "norms", [&] { return factor_norms(c, partial, scal + 1); }));
    hipLaunchKernelGGL(k_store_iter, dim3(1), dim3(64), 0, c->st, scal, c->dres,
                       c->iter_ctr);
    HIPCHK(c, hipGetLastError());
    // Approx variant: remove cells of G after the error (Alg. 2, Alg. 4)
    if (c->opt.approx_rate > 0.0)
        return approx_step(c, c->opt.approx_rate, true, c->ap_stored);
    return PTK_OK;
}

// Capture iteration_body into a graph on a private stream (capture needs a
// stream other than the null stream); replayed on the context's stream.
ptk_status ensure_iteration_graph(ptk_ctx *c, double lambda) {
    const int fuse = c->opt.fuse_error ? 1 : 0;
    if (c->gexec && c->g_epoch == c->epoch && c->g_lambda == lambda && c->g_fuse == fuse)
        return PTK_OK;
    if (c->gexec) {
        (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
    }
    if (!c->gstream) HIPCHK(c, hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking));
    hipStream_t user = c->st;
    c->st = c->gstream;
    hipError_t e = hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal);
    ptk_status s = PTK_OK;
    if (e == hipSuccess) s = iteration_body(c, lambda);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(c->gstream, &g);
    c->st = user;
    if (e != hipSuccess) return fail(c, PTK_E_HIP, "graph capture: %s", hipGetErrorString(e));
    if (s != PTK_OK) {
        if (g) (void)hipGraphDestroy(g);
        return s;
    }
    if (e2 != hipSuccess) return fail(c, PTK_E_HIP, "graph capture: %s", hipGetErrorString(e2));
    e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        c->gexec = nullptr;
        return fail(c, PTK_E_HIP, "graph instantiate: %s", hipGetErrorString(e));
    }
    c->g_epoch = c->epoch;
    c->g_lambda = lambda;
    c->g_fuse = fuse;
    return PTK_OK;
}

}  // namespace

extern "C" {

ptk_status ptk_create(ptk_ctx **out, int32_t N, const int64_t *dims_host,
                      const int32_t *ranks_host, void *hip_stream) {
    if (!out) return PTK_E_INVALID;
    *out = nullptr;
    if (N < 2 || N > kMaxN || !dims_host || !ranks_host) return PTK_E_INVALID;
    int64_t cells = 1;
    for (int n = 0; n < N; ++n) {
        if (dims_host[n] < 1 || dims_host[n] >= (int64_t(1) << 31)) return PTK_E_INVALID;
        if (ranks_host[n] < 1 || ranks_host[n] > kMaxJ) return PTK_E_INVALID;
        cells *= ranks_host[n];
        if (cells > kMaxCore) return PTK_E_INVALID;
    }
    ptk_ctx *c = new (std::nothrow) ptk_ctx();
    if (!c) return PTK_E_NOMEM;
    c->s.N = N;
    for (int n = 0; n < N; ++n) {
        c->s.dims[n] = dims_host[n];
        c->s.ranks[n] = ranks_host[n];
    }
    c->core_cells = cells;
    c->st = (hipStream_t)hip_stream;
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount,
                                  c->device);
    // generic kernels keep the other factor rows in LDS: bound their size
    for (int n = 0; n < N && e == hipSuccess; ++n) {
        int sumj = 0;
        for (int k = 0; k < N; ++k)
            if (k != n) sumj += ranks_host[k];
        const size_t lds = (size_t)sumj * kWave * 4 + (ranks_host[n] + 1) * 65 * 8;
        if (lds > 64 * 1024) {
            delete c;
            return PTK_E_UNSUPPORTED;
        }
    }
    for (int n = 0; n < N && e == hipSuccess; ++n)
        e = hipMalloc(&c->gp[n], (size_t)(cells + 64) * sizeof(double));
    if (e == hipSuccess) e = dalloc(&c->gpe, (size_t)(cells + 64));
    if (e == hipSuccess)
        e = dalloc(&c->red, std::max<size_t>((size_t)kRedBlocks * (N + 1), kSseBlocks + 2) + 64);
    int64_t max_rows = 1;
    for (int n = 0; n < N; ++n) max_rows = std::max<int64_t>(max_rows, dims_host[n]);
    c->max_rows = max_rows;
    if (e == hipSuccess) e = dalloc(&c->ctr, kCtrSlots);
    if (e == hipSuccess) e = hipMemset(c->ctr, 0, kCtrSlots * sizeof(int32_t));
    c->bad = c->ctr;
    if (e == hipSuccess) e = dalloc(&c->lslist, (size_t)max_rows);
    if (e == hipSuccess) e = dalloc(&c->rflag, (size_t)max_rows);
    if (e == hipSuccess) e = dalloc(&c->rsse, (size_t)max_rows);
    if (e == hipSuccess) e = dalloc(&c->fold_ls, 8);
    if (e == hipSuccess) e = noalloc_scratch(c->device, &c->noalloc);
    if (e == hipSuccess) e = dalloc(&c->xsq, 1);
    if (e == hipSuccess) e = dalloc(&c->scal, 4);
    if (e == hipSuccess) e = dalloc(&c->iter_ctr, 1);
    if (e != hipSuccess) {
        ptk_destroy(c);
        return e == hipErrorOutOfMemory ? PTK_E_NOMEM : PTK_E_HIP;
    }
    *out = c;
    return PTK_OK;
}

ptk_status ptk_destroy(ptk_ctx *c) {
    if (!c) return PTK_OK;
    if (c->st) (void)hipStreamSynchronize(c->st);
    else (void)hipDeviceSynchronize();
    free_modes(c);
    for (int n = 0; n < kMaxN; ++n) {
        dfree(c->gp[n]);
        dfree(c->frag[n]);
    }
    dfree(c->gpe);
    dfree(c->red);
    dfree(c->ctr);
    dfree(c->lslist);
    dfree(c->rflag);
    dfree(c->rsse);
    dfree(c->fold_ls);
    dfree(c->xsq);
    dfree(c->scal);
    dfree(c->dres);
    dfree(c->iter_ctr);
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->gstream) (void)hipStreamDestroy(c->gstream);
    dfree(c->qr_work);
    dfree(c->fold_bbuf);
    dfree(c->fold_part);
    dfree(c->fold_rowptr);
    dfree(c->fold_split);
    if (c->host) (void)hipHostFree(c->host);
    for (auto &t : c->pending) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    for (auto e : c->pool) (void)hipEventDestroy(e);
    delete c;
    return PTK_OK;
}

const char *ptk_last_error(const ptk_ctx *c) {
    if (!c) return global_error();
    return c->err.c_str();
}

ptk_status ptk_set_options(ptk_ctx *c, const ptk_options *o) {
    if (!c || !o) return PTK_E_INVALID;
    if (o->precision < PTK_PREC_FP64_ACC || o->precision > PTK_PREC_BF16X3)
        return fail(c, PTK_E_INVALID, "unknown precision %d", o->precision);
    const bool bf_new = o->precision == PTK_PREC_BF16 || o->precision == PTK_PREC_BF16X3;
    const bool bf_old =
        c->opt.precision == PTK_PREC_BF16 || c->opt.precision == PTK_PREC_BF16X3;
    if (bf_new && !(equal_ranks(c->s) && mfma_available(c->s.N, c->s.ranks[0])))
        return fail(c, PTK_E_UNSUPPORTED, "no matrix-core kernel for this shape");
    const bool rebf = bf_new != bf_old || (bf_new && o->precision != c->opt.precision);
    if (rebf && c->nnz >= 0)
        return fail(c, PTK_E_STATE, "BF16 form must be chosen before ptk_set_observed");
    if (o->chunk_nnz < 0 || (o->chunk_nnz % kWave) != 0)
        return fail(c, PTK_E_INVALID, "chunk_nnz must be a multiple of 64");
    const bool rechunk = o->chunk_nnz != c->opt.chunk_nnz;
    if (rechunk && c->nnz >= 0)
        return fail(c, PTK_E_STATE, "chunk_nnz must be set before ptk_set_observed");
    if (o->pair_cache != 0 && o->pair_cache != 1)
        return fail(c, PTK_E_INVALID, "pair_cache must be 0 or 1");
    if (o->pair_cache &&
        (bf_new || !equal_ranks(c->s) || !cache_available(c->s.N, c->s.ranks[0])))
        return fail(c, PTK_E_UNSUPPORTED,
                    "no pair-cache kernel for this shape and precision");
    if (o->pair_cache != c->opt.pair_cache && c->nnz >= 0)
        return fail(c, PTK_E_STATE, "pair_cache must be set before ptk_set_observed");
    if (!(o->tol >= 0.0) || !std::isfinite(o->tol))
        return fail(c, PTK_E_INVALID, "tol must be finite and >= 0");
    if (o->delta_slices < 0 || o->delta_slices > 65535)
        return fail(c, PTK_E_INVALID, "delta_slices must be in [0, 65535]");
    if (o->delta_slices != c->opt.delta_slices && c->nnz >= 0)
        return fail(c, PTK_E_STATE, "delta_slices must be set before ptk_set_observed");
    if (!(o->approx_rate >= 0.0 && o->approx_rate < 1.0))
        return fail(c, PTK_E_INVALID, "approx_rate must be in [0, 1)");
    if (o->approx_form < 0 || o->approx_form > 2)
        return fail(c, PTK_E_INVALID, "approx_form must be 0, 1 or 2");
    if (o->approx_rate > 0.0 &&
        !(equal_ranks(c->s) && approx_available(c->s.N, c->s.ranks[0])))
        return fail(c, PTK_E_UNSUPPORTED, "no Approx kernels for this shape");
    if (!(o->cond_limit >= 0.0) || !std::isfinite(o->cond_limit))
        return fail(c, PTK_E_INVALID, "cond_limit must be finite and >= 0");
    if (!(o->sparse_limit <= 1.0) || !std::isfinite(o->sparse_limit))
        return fail(c, PTK_E_INVALID, "sparse_limit must be finite and <= 1");
    const int su = o->shared_units;
    if (su != -1 && su != 0 && su != 1 && su != 2 && su != 4 && su != 8 && su != 16)
        return fail(c, PTK_E_INVALID, "shared_units must be -1, 0, 1, 2, 4, 8 or 16");
    if (su != c->opt.shared_units && c->nnz >= 0)
        return fail(c, PTK_E_STATE, "shared_units must be set before ptk_set_observed");
    c->opt = *o;
    c->epoch++;
    return PTK_OK;
}

ptk_status ptk_set_observed(ptk_ctx *c, int64_t nnz, const int32_t *idx,
                            const float *val) {
    if (!c) return PTK_E_INVALID;
    if (nnz < 0 || nnz >= (int64_t(1) << 31))
        return fail(c, PTK_E_INVALID, "nnz out of range");
    if (nnz > 0 && (!idx || !val)) return fail(c, PTK_E_INVALID, "null input");
    HIPCHK(c, hipStreamSynchronize(c->st));
    free_modes(c);
    c->epoch++;
    const Shape &s = c->s;
    const int N = s.N;

    // validate indices and values on the device
    if (nnz > 0) {
        unsigned long long *dbad = nullptr;
        HIPCHK(c, dalloc(&dbad, 2));
        hipError_t e = hipMemsetAsync(dbad, 0, 2 * sizeof(unsigned long long), c->st);
        if (e == hipSuccess) e = launch_validate(idx, val, nnz, s, dbad, c->st);
        unsigned long long hb[2] = {0, 0};
        if (e == hipSuccess)
            e = hipMemcpyAsync(hb, dbad, sizeof hb, hipMemcpyDeviceToHost, c->st);
        if (e == hipSuccess) e = hipStreamSynchronize(c->st);
        dfree(dbad);
        HIPCHK(c, e);
        if (hb[0] || hb[1])
            return fail(c, PTK_E_INVALID,
                        "%llu index(es) out of range, %llu non-finite value(s)", hb[0],
                        hb[1]);
    }

    // per-mode CSR; with the pair cache also the position map from each
    // reader's grouping to its writer's (perm: grouped position -> entry)
    void *work = nullptr;
    HIPCHK(c, hipMalloc(&work, sort_workspace_bytes(nnz)));
    int32_t *perm = nullptr, *inv = nullptr;
    if (c->opt.pair_cache && nnz > 0) {
        hipError_t e = dalloc(&perm, nnz);
        if (e == hipSuccess) e = dalloc(&inv, nnz);
        if (e != hipSuccess) {
            dfree(work);
            dfree(perm);
            return fail(c, PTK_E_NOMEM, "pair-cache position maps");
        }
    }
    const bool eq = equal_ranks(s);
    for (int n = 0; n < N; ++n) {
        ModeData &m = c->md[n];
        const int role = cache_role(c, n);
        hipError_t e = dalloc(&m.rowptr, s.dims[n] + 1);
        if (e == hipSuccess) e = dalloc(&m.rows, nnz + 64);
        if (e == hipSuccess) e = dalloc(&m.oidx, (size_t)(N - 1) * nnz + 64);
        if (e == hipSuccess) e = dalloc(&m.vals, nnz + 64);
        if (e == hipSuccess && role == 2) e = dalloc(&m.cmap, nnz + 64);
        if (e == hipSuccess)
            e = build_mode_csr(idx, val, nnz, s, n, work, m.rowptr, m.rows, m.oidx,
                               m.vals, c->st, role && nnz > 0 ? perm : nullptr,
                               units_sub(c, n));
        if (e == hipSuccess && role == 1 && nnz > 0)
            e = launch_invert_perm(perm, nnz, inv, c->st);
        if (e == hipSuccess && role == 2 && nnz > 0)
            e = launch_compose_perm(inv, perm, nnz, m.cmap, c->st);
        if (e != hipSuccess) {
            dfree(work);
            dfree(perm);
            dfree(inv);
            free_modes(c);
            return fail(c, e == hipErrorOutOfMemory ? PTK_E_NOMEM : PTK_E_HIP,
                        "CSR build of mode %d: %s", n, hipGetErrorString(e));
        }
        m.fast = eq && fast_available(N, s.ranks[n], kArithF64);
        const bool bf = c->opt.precision == PTK_PREC_BF16 ||
                        c->opt.precision == PTK_PREC_BF16X3;
        m.slices = m.slice_sub = m.slice_w = 1;
        if (!m.fast && !bf && role != 2) {
            const SlicePlan sp = slice_plan(s, n, role == 1 ? n + 1 : -1, nnz, c->num_cu,
                                            c->opt.delta_slices);
            m.slices = sp.S;
            m.slice_sub = sp.sub;
            m.slice_w = sp.W;
        }
    }
    hipError_t e = hipStreamSynchronize(c->st);
    dfree(work);
    dfree(perm);
    dfree(inv);
    if (e != hipSuccess) {
        free_modes(c);
        HIPCHK(c, e);
    }
    int64_t dpart_need = 0;
    for (int n = 0; n < N; ++n)
        if (c->md[n].slices > 1)
            dpart_need = std::max(
                dpart_need, slice_part_doubles(s.ranks[n], nnz,
                                               SlicePlan{c->md[n].slices, c->md[n].slice_sub,
                                                         c->md[n].slice_w}));
    if (dpart_need > 0 && dalloc(&c->dpart, (size_t)dpart_need) != hipSuccess) {
        free_modes(c);
        return fail(c, PTK_E_NOMEM, "slice partials: %.2f GB of device memory",
                    dpart_need * 8e-9);
    }
    if (c->opt.pair_cache) {
        const int64_t rec = cache_record_doubles(s.ranks[0]);
        if (dalloc(&c->pcache, (size_t)(nnz + 1) * rec) != hipSuccess) {
            free_modes(c);
            return fail(c, PTK_E_NOMEM, "pair cache: %.2f GB of device memory",
                        (nnz + 1) * rec * 8e-9);
        }
    }
    c->nnz = nnz;
    {
        ptk_status us = build_unit_lists(c);
        if (us != PTK_OK) return us;
    }

    // work ranges and rows that cross them
    int64_t bbuf_elems = 0;
    for (int n = 0; n < N; ++n) {
        ModeData &m = c->md[n];
        const int E = sys_entries(s.ranks[n]);
        m.rp_host.resize(s.dims[n] + 1);
        HIPCHK(c, hipMemcpy(m.rp_host.data(), m.rowptr, m.rp_host.size() * 8,
                            hipMemcpyDeviceToHost));
        const std::vector<int64_t> &rp = m.rp_host;
        if (c->opt.precision == PTK_PREC_BF16 || c->opt.precision == PTK_PREC_BF16X3) {
            // blocks of <= 32 entries of one row
            m.bf16 = true;
            m.split_bf16 = c->opt.precision == PTK_PREC_BF16X3 ? 3 : 1;
            std::vector<int32_t> br, bst, bc;
            m.first_blk.assign(s.dims[n], -1);
            m.last_blk.assign(s.dims[n], -1);
            for (int64_t r = 0; r < s.dims[n]; ++r)
                for (int64_t q = rp[r]; q < rp[r + 1]; q += 32) {
                    if (m.first_blk[r] < 0) m.first_blk[r] = (int32_t)br.size();
                    m.last_blk[r] = (int32_t)br.size();
                    br.push_back((int32_t)r);
                    bst.push_back((int32_t)q);
                    bc.push_back((int32_t)std::min<int64_t>(32, rp[r + 1] - q));
                }
            m.nblk = (int64_t)br.size();
            HIPCHK(c, dalloc(&m.blk_row, br.size()));
            HIPCHK(c, dalloc(&m.blk_start, bst.size()));
            HIPCHK(c, dalloc(&m.blk_cnt, bc.size()));
            if (m.nblk) {
                HIPCHK(c, hipMemcpy(m.blk_row, br.data(), br.size() * 4, hipMemcpyHostToDevice));
                HIPCHK(c, hipMemcpy(m.blk_start, bst.data(), bst.size() * 4, hipMemcpyHostToDevice));
                HIPCHK(c, hipMemcpy(m.blk_cnt, bc.data(), bc.size() * 4, hipMemcpyHostToDevice));
            }
            if (!c->frag[n])
                HIPCHK(c, hipMalloc(&c->frag[n], 2 * (size_t)mfma_tiles(N, s.ranks[n]) * kWave * 8));
        }
        ptk_status st = configure_ranges(c, n, c->opt.chunk_nnz > 0 && !m.bf16
                                                   ? c->opt.chunk_nnz : 0);
        if (st != PTK_OK) return st;
        bbuf_elems = std::max(bbuf_elems, s.dims[n] * E);
    }
    HIPCHK(c, dalloc(&c->bbuf, bbuf_elems));
    // least-squares solve: heavy rows, their tasks and the tasks' triangles
    {
        int jmax = 1;
        for (int n = 0; n < s.N; ++n) jmax = std::max(jmax, (int)s.ranks[n]);
        // every row may be heavy; tasks up to 2 nnz / task_len, within a
        // memory budget for their triangles (rows beyond it take one
        // wavefront each)
        c->ls_hcap = c->max_rows;
        c->ls_tcap = std::max<int64_t>(
            1, std::min<int64_t>(2 * (nnz / kLsTaskLen) + 1,
                                 (int64_t)(kLsTriBytes / (sizeof(double) * jmax * (jmax + 1)))));
        HIPCHK(c, dalloc(&c->ls_hrow, (size_t)c->ls_hcap));
        HIPCHK(c, dalloc(&c->ls_hoff, (size_t)c->ls_hcap));
        HIPCHK(c, dalloc(&c->ls_tri, (size_t)c->ls_tcap * jmax * (jmax + 1)));
        // deltas kept for the next update's least-squares rows: an eighth of
        // the entries (at least 65536), within kKeepBytes; a plan per mode,
        // empty until a mode update has flagged rows
        int64_t rows = 0;
        for (int n = 0; n < s.N; ++n) {
            c->kb_off[n] = rows;
            rows += s.dims[n];
        }
        c->ls_kcap = std::min<int64_t>(
            nnz, std::min<int64_t>(std::max<int64_t>(65536, nnz / 8),
                                   (int64_t)(kKeepBytes / (sizeof(double) * jmax))));
        if (c->ls_kcap > 0) {
            HIPCHK(c, dalloc(&c->ls_kbase, (size_t)rows));
            HIPCHK(c, dalloc(&c->ls_keep, (size_t)c->ls_kcap * jmax));
            HIPCHK(c, dalloc(&c->ls_kused, 1));
            for (int n = 0; n < s.N; ++n)
                HIPCHK(c, launch_keep_plan(nullptr, c->md[n].rowptr, s.dims[n], c->ls_kcap,
                                           c->ls_kbase + c->kb_off[n], c->ls_kused, c->st));
        }
    }
    // sum of x^2 for the error identity of the fused pass
    if (nnz > 0) {
        HIPCHK(c, launch_sumsq(c->md[0].vals, nnz, c->red, kRedBlocks, c->st));
        HIPCHK(c, launch_reduce(c->red, kRedBlocks, c->xsq, c->st));
    } else {
        hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, c->st, c->xsq, 0.0, (int64_t)1);
        HIPCHK(c, hipGetLastError());
    }
    HIPCHK(c, hipStreamSynchronize(c->st));
    return PTK_OK;
}

ptk_status ptk_bind_model(ptk_ctx *c, float *core, float *const *factors_host) {
    if (!c || !core || !factors_host) return fail(c, PTK_E_INVALID, "null model");
    for (int n = 0; n < c->s.N; ++n)
        if (!factors_host[n]) return fail(c, PTK_E_INVALID, "null factor %d", n);
    c->core = core;
    for (int n = 0; n < c->s.N; ++n) c->fac[n] = factors_host[n];
    c->epoch++;
    return PTK_OK;
}

ptk_status ptk_update_mode(ptk_ctx *c, int32_t n, double lambda) {
    if (!c) return PTK_E_INVALID;
    if (n < 0 || n >= c->s.N) return fail(c, PTK_E_INVALID, "mode %d out of range", n);
    if (!(lambda > 0.0) || !std::isfinite(lambda))
        return fail(c, PTK_E_INVALID, "lambda must be > 0");
    ptk_status s = need_model(c);
    if (s != PTK_OK) return s;
    HIPCHK(c, permute(c, n));
    HIPCHK(c, zero_bad(c));
    s = update_mode_impl(c, n, lambda);
    if (s != PTK_OK) return s;
    return check_bad(c, "ptk_update_mode");
}

ptk_status ptk_iterate(ptk_ctx *c, int32_t iters, double lambda, double *sse_host,
                       double *loss_host) {
    if (!c) return PTK_E_INVALID;
    if (iters < 0) return fail(c, PTK_E_INVALID, "iters < 0");
    if (!(lambda > 0.0) || !std::isfinite(lambda))
        return fail(c, PTK_E_INVALID, "lambda must be > 0");
    ptk_status s = need_model(c);
    if (s != PTK_OK) return s;
    c->last_iters = 0;
    if (iters == 0) return PTK_OK;
    s = ensure_host(c, 2 * (size_t)iters);
    if (s != PTK_OK) return s;
    if (c->dres_cap < iters) {
        dfree(c->dres);
        c->dres = nullptr;
        c->dres_cap = 0;
        HIPCHK(c, dalloc(&c->dres, 2 * (size_t)iters));
        c->dres_cap = iters;
        c->epoch++;
    }
    const int N = c->s.N;
    for (int n = 0; n < N; ++n) HIPCHK(c, permute(c, n, cache_role(c, n)));
    HIPCHK(c, zero_bad(c));
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, c->st, c->iter_ctr, 0, (int64_t)1);
    HIPCHK(c, hipGetLastError());
    if (c->opt.approx_rate > 0.0) {
        s = ensure_approx(c);
        if (s != PTK_OK) return s;
    }
    const bool use_graph = c->opt.use_graph && !c->opt.profile;
    if (use_graph) {
        s = ensure_iteration_graph(c, lambda);
        if (s != PTK_OK) return s;
    }
    const double tol = c->opt.tol;
    int done = 0;
    while (done < iters) {
        if (use_graph) {
            HIPCHK(c, hipGraphLaunch(c->gexec, c->st));
        } else {
            s = iteration_body(c, lambda);
            if (s != PTK_OK) return s;
        }
        ++done;
        if (tol > 0.0 && done >= 2) {
            // the errors of the last two iterations (Alg. 2's stopping test)
            HIPCHK(c, hipMemcpyAsync(c->host, c->dres + 2 * (done - 2), 4 * sizeof(double),
                                     hipMemcpyDeviceToHost, c->st));
            HIPCHK(c, hipStreamSynchronize(c->st));
            const double e0 = std::sqrt(std::max(c->host[0], 0.0));
            const double e1 = std::sqrt(std::max(c->host[2], 0.0));
            if (std::fabs(e1 - e0) <= tol * e0) break;
        }
    }
    c->last_iters = done;
    HIPCHK(c, hipMemcpyAsync(c->host, c->dres, 2 * sizeof(double) * done,
                             hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    int diverged = -1;
    double prev = 0.0;
    for (int t = 0; t < iters; ++t) {
        const bool ran = t < done;
        const double sse = ran ? c->host[2 * t] : std::nan("");
        const double loss = ran ? c->host[2 * t] + lambda * c->host[2 * t + 1] : std::nan("");
        if (sse_host) sse_host[t] = sse;
        if (loss_host) loss_host[t] = loss;
        if (ran && diverged < 0) {
            const bool rise = t > 0 && c->opt.approx_rate == 0.0 && loss > prev * (1.0 + 1e-6);
            if (!std::isfinite(sse) || !std::isfinite(loss) || rise) diverged = t;
        }
        prev = loss;
    }
    s = check_bad(c, "ptk_iterate");
    if (s != PTK_OK || diverged < 0) return s;
    return fail(c, PTK_E_DIVERGED,
                "ptk_iterate: iteration %d: error %.17g, loss %.17g (previous loss %.17g)",
                diverged, c->host[2 * diverged],
                c->host[2 * diverged] + lambda * c->host[2 * diverged + 1],
                diverged > 0 ? c->host[2 * (diverged - 1)] +
                                   lambda * c->host[2 * (diverged - 1) + 1]
                             : std::nan(""));
}

ptk_status ptk_iterations_done(const ptk_ctx *c, int32_t *n_host) {
    if (!c || !n_host) return PTK_E_INVALID;
    *n_host = c->last_iters;
    return PTK_OK;
}

ptk_status ptk_recon_error(ptk_ctx *c, double lambda, double *sse_host,
                           double *rmse_host, double *loss_host) {
    if (!c) return PTK_E_INVALID;
    ptk_status s = need_model(c);
    if (s != PTK_OK) return s;
    s = ensure_host(c, 2);
    if (s != PTK_OK) return s;
    double *partial = c->red;
    double *scal = c->scal;
    HIPCHK(c, timed(c, "error", [&] { return sse_direct(c, partial, scal); }));
    HIPCHK(c, timed(c, "norms", [&] { return factor_norms(c, partial, scal + 1); }));
    HIPCHK(c, hipMemcpyAsync(c->host, scal, 2 * sizeof(double), hipMemcpyDeviceToHost,
                             c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    const double sse = c->host[0];
    if (sse_host) *sse_host = sse;
    if (rmse_host) *rmse_host = c->nnz > 0 ? std::sqrt(sse / (double)c->nnz) : 0.0;
    if (loss_host) *loss_host = sse + lambda * c->host[1];
    return PTK_OK;
}

ptk_status ptk_orthogonalize(ptk_ctx *c) {
    if (!c) return PTK_E_INVALID;
    if (!c->core) return fail(c, PTK_E_STATE, "no model bound (ptk_bind_model)");
    const Shape &s = c->s;
    for (int n = 0; n < s.N; ++n)
        if (s.dims[n] < s.ranks[n])
            return fail(c, PTK_E_INVALID, "mode %d has fewer rows than its rank", n);
    size_t need = (size_t)kMaxN * kMaxJ * kMaxJ * 8 + 2 * (size_t)c->core_cells * 8 + 256;
    size_t qr = 0;
    for (int n = 0; n < s.N; ++n) qr = std::max(qr, qr_workspace_bytes(s.dims[n], s.ranks[n]));
    need += qr;
    if (need > c->qr_cap) {
        dfree(c->qr_work);
        c->qr_work = nullptr;
        c->qr_cap = 0;
        HIPCHK(c, hipMalloc(&c->qr_work, need));
        c->qr_cap = need;
    }
    double *Rs = (double *)c->qr_work;
    char *qrw = (char *)c->qr_work + (size_t)kMaxN * kMaxJ * kMaxJ * 8 +
                2 * (size_t)c->core_cells * 8 + 256;
    HIPCHK(c, zero_bad(c));
    for (int n = 0; n < s.N; ++n)
        HIPCHK(c, timed(c, "qr", [&] {
            return launch_thin_qr(c->fac[n], s.dims[n], s.ranks[n], qrw,
                                  Rs + (size_t)n * kMaxJ * kMaxJ, c->bad, c->st);
        }));
    HIPCHK(c, timed(c, "core_update", [&] {
        return launch_core_mode_product(c->core, c->core, s, 0, Rs, c->st);
    }));
    return check_bad(c, "ptk_orthogonalize");
}

ptk_status ptk_predict(ptk_ctx *c, int64_t m, const int32_t *idx, float *out) {
    if (!c) return PTK_E_INVALID;
    if (m < 0) return fail(c, PTK_E_INVALID, "m < 0");
    if (!c->core) return fail(c, PTK_E_STATE, "no model bound (ptk_bind_model)");
    if (m == 0) return PTK_OK;
    if (!idx || !out) return fail(c, PTK_E_INVALID, "null buffer");
    HIPCHK(c, permute_entries(c, 0));
    EntryArgs a{};
    const int32_t *other[kMaxN];
    for (int k = 1; k < c->s.N; ++k) other[k - 1] = idx + (int64_t)k * m;
    fill_common(c, 0, a, other);
    a.gp = c->gpe;
    a.own_idx = idx;
    a.own = c->fac[0];
    a.m = m;
    a.out = out;
    const bool fast = equal_ranks(c->s) && fast_available(c->s.N, c->s.ranks[0], kArithF64);
    const int64_t blocks = std::min<int64_t>((m + kWave - 1) / kWave, (int64_t)c->num_cu * 16);
    HIPCHK(c, timed(c, "predict", [&] {
        return launch_entries(a, c->s, 0, kOutPredict, fast, blocks, c->st);
    }));
    return PTK_OK;
}

ptk_status ptk_entry_error(ptk_ctx *c, int64_t m, const int32_t *idx, const float *val,
                           double *sse_host, double *rmse_host) {
    if (!c) return PTK_E_INVALID;
    if (m < 0) return fail(c, PTK_E_INVALID, "m < 0");
    if (!c->core) return fail(c, PTK_E_STATE, "no model bound (ptk_bind_model)");
    if (m > 0 && (!idx || !val)) return fail(c, PTK_E_INVALID, "null buffer");
    ptk_status s = ensure_host(c, 1);
    if (s != PTK_OK) return s;
    double sse = 0.0;
    if (m > 0) {
        HIPCHK(c, permute_entries(c, 0));
        EntryArgs a{};
        const int32_t *other[kMaxN];
        for (int k = 1; k < c->s.N; ++k) other[k - 1] = idx + (int64_t)k * m;
        fill_common(c, 0, a, other);
        a.gp = c->gpe;
        a.own_idx = idx;
        a.own = c->fac[0];
        a.val = val;
        a.m = m;
        a.partial = c->red;
        const bool fast =
            equal_ranks(c->s) && fast_available(c->s.N, c->s.ranks[0], kArithF64);
        const int64_t nb =
            std::max<int64_t>(1, std::min<int64_t>(kSseBlocks, (m + kWave - 1) / kWave));
        HIPCHK(c, timed(c, "entry_error", [&] {
            hipError_t e = launch_entries(a, c->s, 0, kOutSSE, fast, nb, c->st);
            if (e != hipSuccess) return e;
            return launch_reduce(c->red, (int)nb, c->scal, c->st);
        }));
        HIPCHK(c, hipMemcpyAsync(c->host, c->scal, sizeof(double), hipMemcpyDeviceToHost,
                                 c->st));
        HIPCHK(c, hipStreamSynchronize(c->st));
        sse = c->host[0];
    }
    if (sse_host) *sse_host = sse;
    if (rmse_host) *rmse_host = m > 0 ? std::sqrt(sse / (double)m) : 0.0;
    return PTK_OK;
}

ptk_status ptk_delta(ptk_ctx *c, int32_t n, int64_t m, const int32_t *idx, float *out) {
    if (!c) return PTK_E_INVALID;
    if (n < 0 || n >= c->s.N) return fail(c, PTK_E_INVALID, "mode %d out of range", n);
    if (m < 0) return fail(c, PTK_E_INVALID, "m < 0");
    if (!c->core) return fail(c, PTK_E_STATE, "no model bound (ptk_bind_model)");
    if (m == 0) return PTK_OK;
    HIPCHK(c, permute_entries(c, n));
    EntryArgs a{};
    const int32_t *other[kMaxN];
    int t = 0;
    for (int k = 0; k < c->s.N; ++k)
        if (k != n) other[t++] = idx + (int64_t)k * m;
    fill_common(c, n, a, other);
    a.gp = c->gpe;
    a.own_idx = idx + (int64_t)n * m;
    a.own = c->fac[n];
    a.m = m;
    a.out = out;
    const bool fast = equal_ranks(c->s) && fast_available(c->s.N, c->s.ranks[n], kArithF64);
    const int64_t blocks = std::min<int64_t>((m + kWave - 1) / kWave, (int64_t)c->num_cu * 16);
    HIPCHK(c, launch_entries(a, c->s, n, kOutDelta, fast, blocks, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    return PTK_OK;
}

ptk_status ptk_partial_error(ptk_ctx *c, double *R_out) {
    if (!c) return PTK_E_INVALID;
    if (!R_out) return fail(c, PTK_E_INVALID, "null output");
    ptk_status s = need_model(c);
    if (s != PTK_OK) return s;
    if ((s = ensure_approx(c)) != PTK_OK) return s;
    if ((s = approx_step(c, 0.0, false)) != PTK_OK) return s;
    HIPCHK(c, hipMemcpyAsync(R_out, c->ap_R, sizeof(double) * c->core_cells,
                             hipMemcpyDeviceToDevice, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    return PTK_OK;
}

ptk_status ptk_truncate(ptk_ctx *c, double p, int32_t *removed_host) {
    if (!c) return PTK_E_INVALID;
    if (!(p >= 0.0 && p < 1.0)) return fail(c, PTK_E_INVALID, "p must be in [0, 1)");
    ptk_status s = need_model(c);
    if (s != PTK_OK) return s;
    if ((s = ensure_approx(c)) != PTK_OK) return s;
    if ((s = approx_step(c, p, true)) != PTK_OK) return s;
    int32_t k = 0;
    HIPCHK(c, hipMemcpyAsync(&k, c->ap_removed, sizeof k, hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    if (removed_host) *removed_host = k;
    return PTK_OK;
}

ptk_status ptk_row_systems(ptk_ctx *c, int32_t n, double *B_out, double *c_out) {
    if (!c) return PTK_E_INVALID;
    if (n < 0 || n >= c->s.N) return fail(c, PTK_E_INVALID, "mode %d out of range", n);
    ptk_status s = need_model(c);
    if (s != PTK_OK) return s;
    if (!B_out || !c_out) return fail(c, PTK_E_INVALID, "null output");
    HIPCHK(c, permute(c, n));
    s = systems(c, n);
    if (s != PTK_OK) return s;
    HIPCHK(c, launch_expand_systems(c->bbuf, c->md[n].rowptr, c->s.dims[n],
                                    c->s.ranks[n], B_out, c_out, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    return PTK_OK;
}

}  // extern "C"

namespace {

__global__ void k_fold_setup(int64_t *rowptr, int32_t *split, int64_t k,
                             int32_t nchunks, int32_t *ls) {
    if (threadIdx.x < 4) ls[threadIdx.x] = 0;   // least-squares list counters
    if (threadIdx.x == 0) {
        rowptr[0] = 0;
        rowptr[1] = k;
        split[0] = 0;
        split[1] = 0;
        split[2] = nchunks - 1;
    }
}

constexpr int64_t kFoldMaxChunks = 1024;

}  // namespace

namespace {

// Device buffers of one fold-in: the row system, the partial systems of at
// most max_chunks work ranges (reused for the triangles of at most `tasks`
// least-squares tasks), the row pointers, the merge list, and the
// least-squares counters and lists (8 ints).
struct FoldBufs {
    double *bbuf;
    double *part;
    int64_t max_chunks;
    int64_t *rowptr;
    int32_t *split;
    int32_t *ls;
    int64_t tasks;
};

ptk_status fold_check(ptk_ctx *c, int32_t n, int64_t k, const int32_t *idx, const float *val,
                      double lambda, float *row_out) {
    if (n < 0 || n >= c->s.N) return fail(c, PTK_E_INVALID, "mode %d out of range", n);
    if (k < 0 || k >= (int64_t(1) << 31)) return fail(c, PTK_E_INVALID, "k out of range");
    if (!(lambda > 0.0) || !std::isfinite(lambda))
        return fail(c, PTK_E_INVALID, "lambda must be > 0");
    if (!c->core) return fail(c, PTK_E_STATE, "no model bound (ptk_bind_model)");
    if (!row_out || (k > 0 && (!idx || !val)))
        return fail(c, PTK_E_INVALID, "null buffer");
    return PTK_OK;
}

// The fold-in of eq. "rowupdate" on the given buffers: delta + Gram over
// work ranges, merge, Cholesky solve, least-squares solve if flagged.
// Kernels only; no allocation.
ptk_status fold_in_impl(ptk_ctx *c, int32_t n, int64_t k, const int32_t *idx,
                        const float *val, double lambda, float *row_out, const FoldBufs &b) {
    const int J = c->s.ranks[n];
    const int E = sys_entries(J);
    int64_t chunk = round_up((k + c->num_cu * 4 - 1) / (c->num_cu * 4), kWave);
    chunk = std::max<int64_t>(chunk, 4 * kWave);
    while ((k + chunk - 1) / chunk > b.max_chunks) chunk *= 2;
    const int64_t nchunks = (k + chunk - 1) / chunk;
    hipLaunchKernelGGL(k_fold_setup, dim3(1), dim3(64), 0, c->st, b.rowptr, b.split, k,
                       (int32_t)std::max<int64_t>(nchunks, 1), b.ls);
    HIPCHK(c, hipGetLastError());
    GramArgs a{};
    const int32_t *other[kMaxN];
    int t = 0;
    for (int q = 0; q < c->s.N; ++q)
        if (q != n) other[t++] = idx + (int64_t)q * k;
    fill_common(c, n, a, other);
    a.skip_row = -1;
    a.E = E;
    a.rows = nullptr;
    a.val = val;
    a.rowptr = b.rowptr;
    a.nnz = k;
    a.chunk = chunk;
    a.bbuf = b.bbuf;
    a.part = b.part;
    const bool fast = equal_ranks(c->s) && fast_available(c->s.N, J, kArithF64);
    const Arith ar = (fast && c->opt.precision == PTK_PREC_FP32) ? kArithF32 : kArithF64;
    HIPCHK(c, timed(c, "permute_core", [&] {
        return launch_permute_core(c->core, c->gp[n], c->s, n, ar, c->st);
    }));
    HIPCHK(c, timed(c, "fold_gram", [&] {
        return launch_gram(a, c->s, n, ar, nchunks, fast, c->st);
    }));
    if (nchunks > 1) HIPCHK(c, launch_merge(b.part, b.split, 1, E, b.bbuf, c->st));
    // the row's least-squares solve, if the Cholesky solve flags it: tasks
    // long enough that at most b.tasks are needed, their triangles in
    // part (free after the merge)
    SolveFlags f{};
    f.rflag = (uint8_t *)(b.ls + 7);
    f.cnt = b.ls;
    f.list = b.ls + 4;
    f.cap = 1;
    f.hrow = b.ls + 5;
    f.hoff = b.ls + 6;
    f.hcap = 1;
    f.tcap = b.tasks;
    f.task_len = (int32_t)std::max<int64_t>(
        kLsTaskLen, round_up((k + b.tasks - 1) / b.tasks, kWave));
    f.pack = J < kLsPack;
    f.cond_limit = c->opt.cond_limit > 0.0 ? c->opt.cond_limit : kCondLimitDefault;
    HIPCHK(c, timed(c, "fold_solve", [&] {
        return launch_solve(b.bbuf, b.rowptr, 1, J, lambda, row_out, f, c->st);
    }));
    HIPCHK(c, launch_ls_lists(b.rowptr, 1, f, c->st));
    LsArgs r{};
    if (ar == kArithF64) {
        r.gp = c->gp[n];
    } else {
        r.gp = c->gpe;
        HIPCHK(c, permute_entries(c, n));
    }
    for (int q = 0; q < c->s.N - 1; ++q) {
        r.fac[q] = a.fac[q];
        r.oidx[q] = a.oidx[q];
        r.jk[q] = a.jk[q];
        r.aoff[q] = a.aoff[q];
    }
    r.nother = a.nother;
    r.jn = J;
    r.val = val;
    r.rowptr = b.rowptr;
    r.f = f;
    r.tri = b.part;
    r.lambda = lambda;
    r.A = row_out;
    r.rsse = nullptr;
    r.stats = c->ctr;
    HIPCHK(c, timed(c, "fold_solve_ls", [&] {
        return launch_ls(r, c->s.N, fast, c->num_cu, c->st);
    }));
    return PTK_OK;
}

}  // namespace

// Scratch of ptk_fold_in_noalloc: a file-scope device array, one per device
// for the life of the process. Host code never passes its name to a kernel:
// the device address comes from hipGetSymbolAddress, once per device, at
// ptk_create (noalloc_scratch), and is kept in the context.
constexpr int64_t kNoAllocChunks = 128;         // work ranges of the Gram pass
constexpr int64_t kNoAllocTasks = 129;          // least-squares tasks
constexpr int64_t kNoAllocMaxEntries = int64_t(1) << 24;
constexpr size_t kNoAllocAlign = 256;
constexpr size_t na_up(size_t x) { return (x + kNoAllocAlign - 1) / kNoAllocAlign * kNoAllocAlign; }
constexpr size_t kNaBbuf = 0;
constexpr size_t kNaPart = kNaBbuf + na_up(sizeof(double) * sys_entries(kMaxJ));
constexpr size_t kNaPartDoubles =
    std::max<size_t>((size_t)kNoAllocChunks * 2 * sys_entries(kMaxJ),
                     (size_t)kNoAllocTasks * kMaxJ * (kMaxJ + 1));
constexpr size_t kNaRowptr = kNaPart + na_up(sizeof(double) * kNaPartDoubles);
constexpr size_t kNaSplit = kNaRowptr + na_up(2 * sizeof(int64_t));
constexpr size_t kNaLs = kNaSplit + na_up(3 * sizeof(int32_t));
constexpr size_t kNaEnd = kNaLs + na_up(8 * sizeof(int32_t));
constexpr size_t kNoAllocBytes = size_t(2) << 20;
static_assert(kNaEnd <= kNoAllocBytes, "no-allocation scratch layout");

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of this device's scratch (the current device), looked up
// once per device.
hipError_t noalloc_scratch(int device, void **out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

extern "C" ptk_status ptk_fold_in_noalloc(ptk_ctx *c, int32_t n, int64_t k,
                                          const int32_t *idx, const float *val,
                                          double lambda, float *row_out) {
    if (!c) return PTK_E_INVALID;
    ptk_status s = fold_check(c, n, k, idx, val, lambda, row_out);
    if (s != PTK_OK) return s;
    if (k > kNoAllocMaxEntries)
        return fail(c, PTK_E_INVALID,
                    "ptk_fold_in_noalloc: k = %lld entries exceeds its limit of %lld",
                    (long long)k, (long long)kNoAllocMaxEntries);
    if (!c->noalloc)
        return fail(c, PTK_E_STATE, "ptk_fold_in_noalloc: no scratch for this device");
    unsigned char *base = (unsigned char *)c->noalloc;
    const FoldBufs b{(double *)(base + kNaBbuf), (double *)(base + kNaPart), kNoAllocChunks,
                     (int64_t *)(base + kNaRowptr), (int32_t *)(base + kNaSplit),
                     (int32_t *)(base + kNaLs), kNoAllocTasks};
    // timing events would be created on demand: none in this call
    const int32_t profile = c->opt.profile;
    c->opt.profile = 0;
    s = fold_in_impl(c, n, k, idx, val, lambda, row_out, b);
    c->opt.profile = profile;
    return s;
}

extern "C" ptk_status ptk_fold_in(ptk_ctx *c, int32_t n, int64_t k, const int32_t *idx,
                                  const float *val, double lambda, float *row_out) {
    if (!c) return PTK_E_INVALID;
    ptk_status s = fold_check(c, n, k, idx, val, lambda, row_out);
    if (s != PTK_OK) return s;
    if (!c->fold_bbuf) {
        HIPCHK(c, dalloc(&c->fold_bbuf, (size_t)sys_entries(kMaxJ)));
        HIPCHK(c, dalloc(&c->fold_part, (size_t)kFoldMaxChunks * 2 * sys_entries(kMaxJ)));
        HIPCHK(c, dalloc(&c->fold_rowptr, 2));
        HIPCHK(c, dalloc(&c->fold_split, 3));
    }
    const FoldBufs b{c->fold_bbuf, c->fold_part, kFoldMaxChunks, c->fold_rowptr,
                     c->fold_split, c->fold_ls, kFoldTasks};
    return fold_in_impl(c, n, k, idx, val, lambda, row_out, b);
}

extern "C" ptk_status ptk_kernel_times(ptk_ctx *c, int32_t *count, const char **names,
                                       int64_t *calls, double *ms) {
    if (!c || !count) return PTK_E_INVALID;
    collect_timers(c);
    int32_t cap = *count, k = 0;
    for (auto &kv : c->totals) {
        if (k < cap) {
            if (names) names[k] = kv.first.c_str();
            if (calls) calls[k] = kv.second.first;
            if (ms) ms[k] = kv.second.second;
        }
        ++k;
    }
    *count = k;
    return PTK_OK;
}

namespace {

// Key of the autotuner cache: shape, arithmetic and the row-length
// histogram (rows per power-of-two length class) of the mode.
std::string tune_key(const ptk_ctx *c, int n) {
    const ModeData &m = c->md[n];
    int64_t bins[40] = {0};
    for (size_t r = 0; r + 1 < m.rp_host.size(); ++r) {
        const int64_t len = m.rp_host[r + 1] - m.rp_host[r];
        int b = 0;
        while ((int64_t(1) << b) <= len && b < 39) ++b;
        ++bins[b];
    }
    char buf[128];
    snprintf(buf, sizeof buf, "N=%d,J=%d,n=%d,prec=%d,cache=%d,nnz=%lld,I=%lld,hist=",
             c->s.N, c->s.ranks[n], n, c->opt.precision, cache_role(c, n),
             (long long)c->nnz, (long long)c->s.dims[n]);
    std::string k = buf;
    for (int b = 0; b < 40; ++b) {
        if (b) k += ':';
        k += std::to_string(bins[b]);
    }
    return k;
}

// A line is "key work" or "key work two" (two: 1 = two entries per lane,
// 0 = one; absent = the default).
bool tune_lookup(const char *path, const std::string &key, int64_t *value, int *two) {
    if (!path) return false;
    FILE *f = fopen(path, "r");
    if (!f) return false;
    char line[1024];
    bool hit = false;
    while (fgets(line, sizeof line, f)) {
        char *sp = strchr(line, ' ');
        if (!sp) continue;
        *sp = 0;
        if (key == line) {
            char *end = nullptr;
            *value = strtoll(sp + 1, &end, 10);
            *two = -1;
            if (end && *end == ' ') *two = (int)strtol(end + 1, nullptr, 10) ? 1 : 0;
            hit = true;        // the last entry for a key wins
        }
    }
    fclose(f);
    return hit && *value > 0;
}

void tune_store(const char *path, const std::string &key, int64_t value, int two) {
    if (!path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    if (two >= 0) fprintf(f, "%s %lld %d\n", key.c_str(), (long long)value, two);
    else fprintf(f, "%s %lld\n", key.c_str(), (long long)value);
    fclose(f);
}

}  // namespace

extern "C" ptk_status ptk_autotune(ptk_ctx *c, const char *cache_path, int64_t *work_host) {
    if (!c) return PTK_E_INVALID;
    ptk_status s = need_model(c);
    if (s != PTK_OK) return s;
    hipEvent_t e0 = get_event(c), e1 = get_event(c);
    const int saved_profile = c->opt.profile;
    c->opt.profile = 0;
    for (int n = 0; n < c->s.N && s == PTK_OK; ++n) {
        ModeData &m = c->md[n];
        const std::string key = tune_key(c, n);
        int64_t best = 0;
        int best_two = -1;
        // tile shape: one or two entries per lane, where both are compiled
        const int role = cache_role(c, n);
        const bool both = !m.bf16 && m.fast && role == 0 && m.slices <= 1 &&
                          gram2_available(c->s.N, c->s.ranks[n], arith_of(c, n));
        // Approx variant: the residuals reuse the deltas that the two-entry
        // kernel of the last mode keeps (approx_step), which saves a full
        // contraction per iteration that the timing here does not see; that
        // mode keeps the two-entry kernel
        const bool keep_two = both && c->opt.approx_rate > 0.0 && n == c->s.N - 1 &&
                              approx_mode(c) == c->s.N - 1;
        const int two_lo = both ? (keep_two ? 1 : 0) : -1;
        if (!tune_lookup(cache_path, key, &best, &best_two)) {
            const double mult[] = {0.125, 0.25, 0.5, 1.0, 2.0};
            double best_ms = 1e300;
            HIPCHK(c, permute(c, n, role));
            for (int two = both ? 1 : -1; two >= two_lo && s == PTK_OK; --two) {
                if (two >= 0) m.two = two != 0;
                const int64_t base = default_work(c, n);
                for (double f : mult) {
                    int64_t w = (int64_t)(base * f);
                    w = m.bf16 ? std::max<int64_t>(w, 1)
                               : std::max<int64_t>(round_up(w, kWave), kWave);
                    if ((s = configure_ranges(c, n, w)) != PTK_OK) break;
                    if ((s = systems(c, n, role)) != PTK_OK) break;    // warm-up
                    double ms_min = 1e300;
                    for (int rep = 0; rep < 3 && s == PTK_OK; ++rep) {
                        HIPCHK(c, hipEventRecord(e0, c->st));
                        s = systems(c, n, role);
                        HIPCHK(c, hipEventRecord(e1, c->st));
                        HIPCHK(c, hipEventSynchronize(e1));
                        float ms = 0.f;
                        HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
                        ms_min = std::min(ms_min, (double)ms);
                    }
                    if (s != PTK_OK) break;
                    if (ms_min < best_ms) {
                        best_ms = ms_min;
                        best = m.bf16 ? m.blk_per_wave : m.chunk;
                        best_two = two;
                    }
                }
            }
            if (s != PTK_OK) break;
            tune_store(cache_path, key, best, best_two);
        }
        m.two = keep_two || best_two != 0;
        c->epoch++;
        s = configure_ranges(c, n, best);
        if (work_host) work_host[n] = m.bf16 ? m.blk_per_wave : m.chunk;
    }
    c->opt.profile = saved_profile;
    c->pool.push_back(e0);
    c->pool.push_back(e1);
    return s;
}

extern "C" ptk_status ptk_not_pd_count(ptk_ctx *c, int64_t *count) {
    if (!c || !count) return PTK_E_INVALID;
    *count = c->last_not_pd;
    return PTK_OK;
}

extern "C" ptk_status ptk_solve_stats(ptk_ctx *c, int64_t *ls_rows, int64_t *ls_max) {
    if (!c || !ls_rows || !ls_max) return PTK_E_INVALID;
    *ls_rows = c->last_ls_rows;
    *ls_max = c->last_ls_max;
    return PTK_OK;
}

extern "C" ptk_status ptk_unit_stats(ptk_ctx *c, int32_t n, int64_t *counts, int32_t *on) {
    if (!c || !counts || !on) return PTK_E_INVALID;
    if (c->nnz < 0) return fail(c, PTK_E_STATE, "no observed set");
    if (n < 0 || n >= c->s.N) return fail(c, PTK_E_INVALID, "mode out of range");
    const ModeData &m = c->md[n];
    for (int k = 0; k < 4; ++k) counts[k] = m.ucount[k];
    counts[4] = m.lg.n_long;
    counts[5] = m.lg.n_tasks;
    counts[6] = m.ix.n_long;
    counts[7] = m.ix.n_tasks;
    counts[8] = m.ix.n_ntasks;
    *on = index_live(c, n) ? 2 : units_live(c, n) ? 1 : 0;
    return PTK_OK;
}

extern "C" ptk_status ptk_approx_stats(ptk_ctx *c, int64_t *nonzero_cells,
                                       int32_t *sparse_modes) {
    if (!c || !nonzero_cells || !sparse_modes) return PTK_E_INVALID;
    *nonzero_cells = -1;
    *sparse_modes = 0;
    if (!c->sp_lists || c->last_iters <= 0 || !c->sp_count) return PTK_OK;
    const int N = c->s.N, J = c->s.ranks[0];
    std::vector<int32_t> cnt((size_t)N * J), use((size_t)N);
    HIPCHK(c, hipMemcpyAsync(cnt.data(), c->sp_count, cnt.size() * sizeof(int32_t),
                             hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipMemcpyAsync(use.data(), c->sp_use, use.size() * sizeof(int32_t),
                             hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    int64_t nz = 0;
    for (int j = 0; j < J; ++j) nz += cnt[j];
    int32_t mask = 0;
    for (int n = 0; n < N; ++n)
        if (use[n]) mask |= 1 << n;
    *nonzero_cells = nz;
    *sparse_modes = mask;
    return PTK_OK;
}

extern "C" ptk_status ptk_reset_timers(ptk_ctx *c) {
    if (!c) return PTK_E_INVALID;
    collect_timers(c);
    c->totals.clear();
    return PTK_OK;
}
