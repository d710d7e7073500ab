// Least-squares row solves for the rows that the Cholesky kernels hand over
// (Sec. 3.2, eq. "rowupdate", Theorem 1), FP64.
//
// eq. "rowupdate" is the normal-equation form of the row's regularised least
// squares problem
//     min_a  sum_alpha (x_alpha - a^T delta_alpha)^2 + lambda ||a||^2,
// i.e. of the stacked system [sqrt(lambda) I ; Delta] a ~ [0 ; x]. Forming
// B_i = Delta^T Delta squares the conditioning: once ||B_i|| * 2^-52 nears
// lambda the FP64 factorisation of B_i + lambda I is wrong or breaks down,
// although the minimiser is unique and well defined. The solve kernels flag
// such rows (breakdown, or a large scaled condition estimate); these kernels
// solve them from the entries instead: every entry's delta is recomputed in
// FP64 (the unrolled contraction of the row-system kernels where the shape
// has one) and the QR factorisation of the stacked system is built with
// Householder reflections (Golub & Van Loan, Sec. 5.2), one chunk of entries
// at a time, then back-substituted. |R_jj| never falls below sqrt(lambda), so
// every row is solved.
//
// Layout of a triangle: lane q of a segment holds column q of [R | z]
// (column jn is z) in registers; lane l holds the delta row and value of one
// entry of the chunk; each reflection needs one segment sum per column.
// Segments are whole wavefronts, or 16-lane quarters for the packed rows.
//
// Work: k_ls takes, with every wavefront on its own, (1) the tasks of the
// heavy rows: task_len entries each (one 64-entry chunk in a fit), reduced to
// a triangle in memory (the first task of a row starts from sqrt(lambda) I,
// the others from 0); (2) the single rows: a row per wavefront, solved and
// its error term formed from the kept deltas (a second pass for a row longer
// than one chunk); (3) the packed rows: four per wavefront, 16 lanes each,
// deltas kept for the error term. k_ls_merge then merges the triangles of every
// heavy row (streams of 16 or 64 lanes each merge every NS-th task, then a
// fixed pairwise tree) and back-substitutes. A row's result
// depends only on its own entries, never on where it sits in the lists, so
// the results do not depend on the order in which rows were flagged.
#include "ptk_device.h"

namespace ptk {

namespace {

// Sum over a segment of SEG lanes; the butterfly gives every lane the same
// bits, and the same bits wherever the segment sits in the wavefront.
template <int SEG>
__device__ __forceinline__ double ssum(double v) {
#pragma unroll
    for (int off = SEG / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, SEG);
    return v;
}

// Reflect one chunk of rows [d | x] (one per lane, zero rows allowed) into
// the segment's triangle rc; e is the lane's index within its segment.
// Column j: v = [alpha - beta ; d_j] with beta = -sign(alpha) sqrt(alpha^2 +
// sigma), sigma = ||d_j||^2; H = I - tau v v^T, tau = 2 / v^T v = -1 / (beta
// v0). Applied to column q as rjq + g v0 / beta and d_q + g d_j / beta with
// g = rjq + s / v0, s = d_j . d_q: every factor is bounded (|v0 / beta| in
// [1, 2], |d_j / beta| <= 1, |s / v0| <= ||d_q||), so a column whose norm is
// tiny or subnormal (the rounding left in the later columns of a chunk of
// rank below J, which shrinks geometrically) gives no overflow, where tau
// itself would.
template <int JMAX, int SEG>
__device__ __forceinline__ void ls_merge(double (&rc)[JMAX], double (&d)[JMAX], double &x,
                                         int jn, int e) {
#pragma unroll
    for (int j = 0; j < JMAX; ++j) {
        if (j >= jn) break;
        const double dj = d[j];
        const double sig = ssum<SEG>(dj * dj);
        const bool skip = !(sig > 0.0);        // nothing to annihilate in column j
        const double alpha = __shfl(rc[j], j, SEG);
        const double mu = sqrt(alpha * alpha + sig);
        const double beta = alpha >= 0.0 ? -mu : mu;
        const double v0 = alpha - beta;        // |alpha| + mu: no cancellation
        // mu >= v0 / 2 >= sqrt(sig) >= 2.2e-162 when sig > 0: finite inverses
        const double rb = skip ? 0.0 : 1.0 / beta;
        const double rv = skip ? 0.0 : 1.0 / v0;
        const double vb = v0 * rb;             // in [-2, -1]
        const double db = dj * rb;             // |.| <= 1
#pragma unroll
        for (int q = j + 1; q < JMAX; ++q) {
            if (q >= jn) break;
            const double s = ssum<SEG>(dj * d[q]);
            const double rjq = __shfl(rc[j], q, SEG);
            const double g = rjq + s * rv;
            if (e == q) rc[j] = __builtin_fma(g, vb, rjq);
            d[q] = __builtin_fma(g, db, d[q]);
        }
        {
            const double s = ssum<SEG>(dj * x);
            const double rjz = __shfl(rc[j], jn, SEG);
            const double g = rjz + s * rv;
            if (e == jn) rc[j] = __builtin_fma(g, vb, rjz);
            x = __builtin_fma(g, db, x);
        }
        if (e == j && !skip) rc[j] = beta;
        d[j] = 0.0;
    }
}

// R a = z; lane q < jn of the segment returns a_q.
template <int JMAX, int SEG>
__device__ __forceinline__ double ls_back(const double (&rc)[JMAX], int jn, int e) {
    double aq = 0.0;
#pragma unroll
    for (int j = JMAX - 1; j >= 0; --j) {
        if (j >= jn) continue;
        const double t = ssum<SEG>((e > j && e < jn) ? rc[j] * aq : 0.0);
        const double zj = __shfl(rc[j], jn, SEG);
        const double rjj = __shfl(rc[j], j, SEG);
        const double aj = (zj - t) / rjj;
        if (e == j) aq = aj;
    }
    return aq;
}

// Initial triangle: diag I (sqrt(lambda) I, or 0), z = 0.
template <int JMAX>
__device__ __forceinline__ void ls_init(double (&rc)[JMAX], double diag, int jn, int e) {
#pragma unroll
    for (int p = 0; p < JMAX; ++p) rc[p] = (p == e && e < jn) ? diag : 0.0;
}

// delta (FP64) and value of the entry at pos, or zeros when !valid. NS, JS:
// an unrolled shape (N, J) of the row-system kernels, or 0 for the generic
// contraction. lds: the lane-private factor rows of this wavefront.
template <int JMAX, int NS, int JS>
__device__ __forceinline__ void entry_delta(const LsArgs &a, int64_t pos, bool valid,
                                            float *lds, int lane, double (&d)[JMAX],
                                            double &x) {
    if constexpr (NS > 0) {
        constexpr int NO = NS - 1;
        constexpr int U = fast_depth(NS, JS);
        double ain[U][JS];
        load_rows_fast<NO, JS, U, double>(a, pos, valid, lds, lane, ain);
        double out[JS];
        delta_fast<NO, JS, U, double>(a.gp, lds, lane, ain, out);
#pragma unroll
        for (int j = 0; j < JMAX; ++j) d[j] = (valid && j < JS) ? out[j] : 0.0;
    } else {
        load_rows_generic<JMAX>(a, pos, valid, lds, lane);
        delta_generic<JMAX>(a, lds, lane, d);
#pragma unroll
        for (int j = 0; j < JMAX; ++j)
            if (!valid || j >= a.jn) d[j] = 0.0;
    }
    x = valid ? (double)a.val[pos] : 0.0;
}

// The same from the deltas the row-system kernel kept for row i (kbase of
// the row, kNoKeep: recompute).
template <int JMAX, int NS, int JS>
__device__ __forceinline__ void row_delta(const LsArgs &a, int64_t kb, int64_t pos,
                                          bool valid, float *lds, int lane,
                                          double (&d)[JMAX], double &x) {
    if (kb != kNoKeep) {
        const double *src = a.keep + (kb + pos) * a.jn;
#pragma unroll
        for (int j = 0; j < JMAX; ++j) d[j] = (valid && j < a.jn) ? src[j] : 0.0;
        x = valid ? (double)a.val[pos] : 0.0;
        return;
    }
    entry_delta<JMAX, NS, JS>(a, pos, valid, lds, lane, d, x);
}

__device__ __forceinline__ int64_t row_kbase(const LsArgs &a, int64_t i) {
    return a.kbase ? a.kbase[i] : kNoKeep;
}

// Per-wavefront counts of the rows solved here, flushed with one atomic each
// at the end of a kernel.
struct LsStats {
    int32_t ok = 0, bad = 0, maxcnt = 0;
    __device__ void flush(int32_t *stats, int lane) {
        int32_t o = ok, b = bad, m = maxcnt;
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) {
            o += __shfl_xor(o, off, kWave);
            b += __shfl_xor(b, off, kWave);
            m = max(m, __shfl_xor(m, off, kWave));
        }
        if (lane == 0) {
            if (o) atomicAdd(&stats[1], o);
            if (b) atomicAdd(&stats[0], b);
            if (m) atomicMax(&stats[2], m);
        }
    }
};

// Count a solved row; write it if its result is finite (all lanes e < jn of
// the segment). Returns the stored value of a_e as a double (0 for e >= jn),
// or NaN when the row was left unsolved.
template <int SEG>
__device__ __forceinline__ double ls_store(const LsArgs &a, int64_t i, double aq, int e,
                                           int lane, bool has, int64_t cnt, LsStats &st) {
    const bool fin = !has || e >= a.jn || isfinite(aq);
    const unsigned long long m = __ballot(fin);
    const int base = lane - e;
    const unsigned long long seg =
        SEG == 64 ? ~0ull : (((1ull << SEG) - 1ull) << base);
    const bool all = (m & seg) == seg;
    if (has && e == 0) {
        if (all) ++st.ok;
        else ++st.bad;
        st.maxcnt = max(st.maxcnt, (int32_t)(cnt < INT32_MAX ? cnt : INT32_MAX));
    }
    if (!all) return __builtin_nan("");
    const float af = (float)aq;
    if (has && e < a.jn) a.A[i * a.jn + e] = af;
    return e < a.jn ? (double)af : 0.0;
}

}  // namespace

// Heavy row owning task t: the largest h < nheavy with hoff[h] <= t.
__device__ __forceinline__ int64_t task_row(const SolveFlags &f, int64_t nheavy, int64_t t) {
    int64_t lo = 0, hi = nheavy - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        if (f.hoff[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Sort the flagged rows (rflag[i] == 1) into the packed, single and heavy
// lists; one atomic per wavefront and list for the first two (ballot and
// prefix count within the wavefront), one per row for the rare heavy rows.
__global__ __launch_bounds__(256) void k_ls_lists(const int64_t *__restrict__ rowptr,
                                                  int64_t I, SolveFlags f) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x % kWave;
    const bool flagged = i < I && f.rflag[i] == 1;
    const int64_t cnt = flagged ? rowptr[i + 1] - rowptr[i] : 0;
    const bool packed = flagged && f.pack && cnt <= kLsPack;
    bool heavy = flagged && !packed && cnt > kWave && f.hrow;
    if (heavy) {
        const unsigned long long nt = (unsigned long long)((cnt + f.task_len - 1) / f.task_len);
        const unsigned long long old =
            atomicAdd((unsigned long long *)(f.cnt + 2), (1ull << 32) + nt);
        const int64_t t0 = (int64_t)(old & 0xffffffffull);
        const int64_t h = (int64_t)(old >> 32);
        const bool room = t0 + (int64_t)nt <= f.tcap && h < f.hcap;
        if (h < f.hcap) {
            f.hoff[h] = (int32_t)t0;
            f.hrow[h] = room ? (int32_t)i : -1;
        }
        heavy = room;
    }
    const bool single = flagged && !packed && !heavy;   // also heavy rows without room
    const unsigned long long mp = __ballot(packed), ms = __ballot(single);
    const unsigned long long below = (1ull << lane) - 1ull;
    int32_t bp = 0, bs = 0;
    if (lane == 0) {
        if (mp) bp = atomicAdd(&f.cnt[0], (int32_t)__popcll(mp));
        if (ms) bs = atomicAdd(&f.cnt[1], (int32_t)__popcll(ms));
    }
    bp = __shfl(bp, 0, kWave);
    bs = __shfl(bs, 0, kWave);
    if (packed) f.list[bp + __popcll(mp & below)] = (int32_t)i;
    if (single) f.list[f.cap - 1 - (bs + __popcll(ms & below))] = (int32_t)i;
    if (flagged) f.rflag[i] = heavy ? kLsIdentity : kLsOwnError;
}

hipError_t launch_ls_lists(const int64_t *rowptr, int64_t I, const SolveFlags &f,
                           hipStream_t st) {
    if (I <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ls_lists, dim3((unsigned)((I + 255) / 256)), dim3(256), 0, st, rowptr,
                       I, f);
    return hipGetLastError();
}

template <int JMAX, int NS, int JS>
__global__ __launch_bounds__(kWave) void k_ls(LsArgs a) {
    extern __shared__ __attribute__((aligned(16))) unsigned char s_dyn[];
    float *lds = (float *)s_dyn;
    const int lane = threadIdx.x;
    const int jn = a.jn;
    const double sl = sqrt(a.lambda);
    const int64_t gw = blockIdx.x, nw = gridDim.x;
    const SolveFlags &f = a.f;
    const int64_t L = f.task_len;
    LsStats st;

    // (1) tasks of heavy rows: a triangle per task
    const int64_t nheavy = min((int64_t)f.cnt[3], f.hcap);
    const int64_t ntask = nheavy > 0 ? min((int64_t)f.cnt[2], f.tcap) : 0;
    for (int64_t t = gw; t < ntask; t += nw) {
        const int64_t h = task_row(f, nheavy, t);
        const int64_t i = f.hrow[h];
        if (i < 0) continue;
        const int64_t q = t - f.hoff[h];
        const int64_t r1row = a.rowptr[i + 1];
        const int64_t r0 = a.rowptr[i] + q * L;
        const int64_t r1 = min(r0 + L, r1row);
        const int64_t kb = row_kbase(a, i);
        double rc[JMAX];
        ls_init<JMAX>(rc, q == 0 ? sl : 0.0, jn, lane);
        for (int64_t c0 = r0; c0 < r1; c0 += kWave) {
            double d[JMAX], x;
            row_delta<JMAX, NS, JS>(a, kb, c0 + lane, c0 + lane < r1, lds, lane, d, x);
            ls_merge<JMAX, kWave>(rc, d, x, jn, lane);
        }
        double *tri = a.tri + t * (int64_t)jn * (jn + 1);
        if (lane <= jn) {
#pragma unroll
            for (int p = 0; p < JMAX; ++p)
                if (p < jn) tri[p * (jn + 1) + lane] = rc[p];
        }
    }

    // (2) single rows: a row per wavefront; a row of one chunk keeps its
    // deltas for the error term, a longer one recomputes them
    const int64_t nsingle = f.cnt[1];
    for (int64_t s = gw; s < nsingle; s += nw) {
        const int64_t i = f.list[f.cap - 1 - s];
        const int64_t r0 = a.rowptr[i], r1 = a.rowptr[i + 1];
        const int64_t kb = row_kbase(a, i);
        double rc[JMAX], d0[JMAX], x0 = 0.0;
        ls_init<JMAX>(rc, sl, jn, lane);
        for (int64_t c0 = r0; c0 < r1; c0 += kWave) {
            double d[JMAX], x;
            row_delta<JMAX, NS, JS>(a, kb, c0 + lane, c0 + lane < r1, lds, lane, d, x);
#pragma unroll
            for (int j = 0; j < JMAX; ++j) d0[j] = d[j];
            x0 = x;
            ls_merge<JMAX, kWave>(rc, d, x, jn, lane);
        }
        const double af = ls_store<kWave>(a, i, ls_back<JMAX, kWave>(rc, jn, lane), lane,
                                          lane, true, r1 - r0, st);
        if (a.rsse) {
            double acc = 0.0;
            if (isnan(__shfl(af, 0, kWave))) {
                acc = __builtin_nan("");
            } else if (r1 - r0 <= kWave) {
                double pr = 0.0;
#pragma unroll
                for (int j = 0; j < JMAX; ++j)
                    if (j < jn) pr = __builtin_fma(__shfl(af, j, kWave), d0[j], pr);
                acc = ssum<kWave>(pr * (pr - 2.0 * x0));
            } else {
                for (int64_t c0 = r0; c0 < r1; c0 += kWave) {
                    double d[JMAX], x;
                    row_delta<JMAX, NS, JS>(a, kb, c0 + lane, c0 + lane < r1, lds, lane, d, x);
                    double pr = 0.0;
#pragma unroll
                    for (int j = 0; j < JMAX; ++j)
                        if (j < jn) pr = __builtin_fma(__shfl(af, j, kWave), d[j], pr);
                    acc += ssum<kWave>(pr * (pr - 2.0 * x));
                }
            }
            if (lane == 0) a.rsse[i] = acc;
        }
    }

    // (3) packed rows: four per wavefront, 16 lanes each
    if (f.pack) {
        constexpr int SEG = kLsPack;
        const int64_t npack = f.cnt[0];
        const int slot = lane / SEG, e = lane % SEG;
        for (int64_t g = gw; g * 4 < npack; g += nw) {
            const int64_t t = g * 4 + slot;
            const bool has = t < npack;
            const int64_t i = has ? f.list[t] : 0;
            const int64_t r0 = has ? a.rowptr[i] : 0, r1 = has ? a.rowptr[i + 1] : 0;
            double d[JMAX], x;
            row_delta<JMAX, NS, JS>(a, has ? row_kbase(a, i) : kNoKeep, r0 + e, r0 + e < r1,
                                    lds, lane, d, x);
            double d0[JMAX];
#pragma unroll
            for (int j = 0; j < JMAX; ++j) d0[j] = d[j];
            const double x0 = x;
            double rc[JMAX];
            ls_init<JMAX>(rc, sl, jn, e);
            ls_merge<JMAX, SEG>(rc, d, x, jn, e);
            const double af = ls_store<SEG>(a, i, ls_back<JMAX, SEG>(rc, jn, e), e, lane, has,
                                            r1 - r0, st);
            if (a.rsse) {
                double pr = 0.0;
#pragma unroll
                for (int j = 0; j < JMAX; ++j)
                    if (j < jn) pr = __builtin_fma(__shfl(af, j, SEG), d0[j], pr);
                const double acc = ssum<SEG>(pr * (pr - 2.0 * x0));
                if (has && e == 0) a.rsse[i] = acc;     // NaN when unsolved
            }
        }
    }
    st.flush(a.stats, lane);
}

// Merge the task triangles of every heavy row and back-substitute. The
// workgroup's W wavefronts are cut into segments of SEG lanes (16 when
// J_n < 16), NS = W * 64 / SEG streams in all; stream s merges tasks s,
// s + NS, ... in order, then the streams' triangles are merged pairwise in a
// fixed tree through LDS (stream s takes s + 1, s + 2, s + 4, ...), and
// stream 0 back-substitutes.
template <int JMAX, int W, int SEG>
__global__ __launch_bounds__(kWave *W) void k_ls_merge(LsArgs a) {
    constexpr int NSEG = kWave / SEG;
    constexpr int NS = W * NSEG;
    __shared__ double s_tri[NS][JMAX][JMAX + 1];
    const int lane = threadIdx.x % kWave;
    const int w = threadIdx.x / kWave;
    const int e = lane % SEG;
    const int stream = w * NSEG + lane / SEG;
    const int jn = a.jn;
    const SolveFlags &f = a.f;
    LsStats st;
    const int64_t nheavy = min((int64_t)f.cnt[3], f.hcap);
    for (int64_t h = blockIdx.x; h < nheavy; h += gridDim.x) {
        const int64_t i = f.hrow[h];
        if (i < 0) continue;
        const int64_t cnt = a.rowptr[i + 1] - a.rowptr[i];
        const int64_t t0 = f.hoff[h];
        const int64_t nt = (cnt + f.task_len - 1) / f.task_len;
        double rc[JMAX];
        ls_init<JMAX>(rc, 0.0, jn, e);
        for (int64_t k = stream; k < nt; k += NS) {
            const double *tri = a.tri + (t0 + k) * (int64_t)jn * (jn + 1);
            double d[JMAX], x = 0.0;
#pragma unroll
            for (int q = 0; q < JMAX; ++q)
                d[q] = (e < jn && q < jn) ? tri[e * (jn + 1) + q] : 0.0;
            if (e < jn) x = tri[e * (jn + 1) + jn];
            ls_merge<JMAX, SEG>(rc, d, x, jn, e);
        }
        // pairwise tree over the streams that hold tasks (a stream without
        // one holds a zero triangle, whose merge changes nothing): row p of
        // [R | z] at s_tri[stream][p]
        const int used = (int)min((int64_t)NS, nt);
        for (int step = 1; step < used; step *= 2) {
            if (e <= jn && stream < used) {
#pragma unroll
                for (int p = 0; p < JMAX; ++p)
                    if (p < jn) s_tri[stream][p][e] = rc[p];
            }
            __syncthreads();
            if (stream % (2 * step) == 0 && stream + step < used) {
                double d[JMAX], x = 0.0;
#pragma unroll
                for (int q = 0; q < JMAX; ++q)
                    d[q] = (e < jn && q < jn) ? s_tri[stream + step][e][q] : 0.0;
                if (e < jn) x = s_tri[stream + step][e][jn];
                ls_merge<JMAX, SEG>(rc, d, x, jn, e);
            }
            __syncthreads();
        }
        if (w == 0 && lane < SEG)
            (void)ls_store<SEG>(a, i, ls_back<JMAX, SEG>(rc, jn, e), e, lane, true, cnt, st);
        __syncthreads();
    }
    if (w == 0) st.flush(a.stats, lane);
}

// Plan of the kept deltas: slots by one atomic per wavefront (their order
// varies, the deltas stored in them do not), then, when the rows do not all
// fit, no row is kept, so the set of kept rows never depends on that order.
__global__ void k_keep_zero(unsigned long long *used) { *used = 0; }

__global__ __launch_bounds__(256) void k_keep_slots(const uint8_t *__restrict__ rflag,
                                                    const int64_t *__restrict__ rowptr,
                                                    int64_t I, int64_t *__restrict__ kbase,
                                                    unsigned long long *used) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x % kWave;
    const bool keep = rflag && i < I && rflag[i] != 0;
    const int64_t cnt = keep ? rowptr[i + 1] - rowptr[i] : 0;
    int64_t incl = cnt;                      // inclusive prefix within the wavefront
#pragma unroll
    for (int off = 1; off < kWave; off *= 2) {
        const int64_t v = __shfl_up(incl, off, kWave);
        if (lane >= off) incl += v;
    }
    unsigned long long base = 0;
    if (lane == kWave - 1 && incl > 0) base = atomicAdd(used, (unsigned long long)incl);
    base = __shfl(base, kWave - 1, kWave);
    if (i < I) kbase[i] = keep ? (int64_t)base + (incl - cnt) - rowptr[i] : kNoKeep;
}

__global__ __launch_bounds__(256) void k_keep_check(int64_t I, int64_t kcap,
                                                    int64_t *__restrict__ kbase,
                                                    const unsigned long long *used) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < I && *used > (unsigned long long)kcap) kbase[i] = kNoKeep;
}

hipError_t launch_keep_plan(const uint8_t *rflag, const int64_t *rowptr, int64_t I,
                            int64_t kcap, int64_t *kbase, unsigned long long *used,
                            hipStream_t st) {
    if (I <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((I + 255) / 256);
    hipLaunchKernelGGL(k_keep_zero, dim3(1), dim3(1), 0, st, used);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_keep_slots, dim3(blocks), dim3(256), 0, st, rflag, rowptr, I, kbase,
                       used);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_keep_check, dim3(blocks), dim3(256), 0, st, I, kcap, kbase, used);
    return hipGetLastError();
}

namespace {

size_t ls_lds(const LsArgs &a, int N, bool fast) {
    if (fast) {
        const int J = a.jn;
        const int nout = (N - 1) - fast_depth(N, J);
        return (size_t)(nout > 0 ? nout : 1) * J * kWave * 4;
    }
    int sumj = 0;
    for (int k = 0; k < a.nother; ++k) sumj += a.jk[k];
    return (size_t)sumj * kWave * 4;
}

template <int JMAX, int NS, int JS>
hipError_t launch_ls_t(const LsArgs &a, size_t lds, int num_cu, hipStream_t st) {
    hipLaunchKernelGGL((k_ls<JMAX, NS, JS>), dim3((unsigned)(16 * num_cu)), dim3(kWave),
                       lds, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // LDS of the merge: W * 64 / SEG triangles of JMAX x (JMAX + 1) doubles
    if constexpr (JMAX <= 16) {
        constexpr int WS = JMAX <= 11 ? 8 : 4;
        if (a.jn < kLsPack) {
            hipLaunchKernelGGL((k_ls_merge<JMAX, WS, kLsPack>), dim3((unsigned)(2 * num_cu)),
                               dim3(kWave * WS), 0, st, a);
            return hipGetLastError();
        }
    }
    constexpr int W = JMAX <= 16 ? 8 : 4;
    hipLaunchKernelGGL((k_ls_merge<JMAX, W, kWave>), dim3((unsigned)(2 * num_cu)),
                       dim3(kWave * W), 0, st, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_ls(const LsArgs &a, int N, bool equal_fast, int num_cu, hipStream_t st) {
    const int J = a.jn;
    const size_t lds = ls_lds(a, N, equal_fast);
    if (equal_fast) {
#define PTK_X(n_, j_) \
    if (N == n_ && J == j_) return launch_ls_t<j_, n_, j_>(a, lds, num_cu, st);
        PTK_X(3, 3) PTK_X(3, 4) PTK_X(3, 5) PTK_X(3, 7) PTK_X(3, 8) PTK_X(3, 9)
        PTK_X(3, 10) PTK_X(3, 11) PTK_X(3, 16) PTK_X(4, 3) PTK_X(4, 5) PTK_X(4, 8)
        PTK_X(4, 10) PTK_X(5, 3) PTK_X(5, 5) PTK_X(5, 8)
#undef PTK_X
    }
    if (J <= 4) return launch_ls_t<4, 0, 0>(a, lds, num_cu, st);
    if (J <= 8) return launch_ls_t<8, 0, 0>(a, lds, num_cu, st);
    if (J <= 16) return launch_ls_t<16, 0, 0>(a, lds, num_cu, st);
    return launch_ls_t<32, 0, 0>(a, lds, num_cu, st);
}

}  // namespace ptk
