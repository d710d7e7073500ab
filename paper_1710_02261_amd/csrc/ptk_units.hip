// Shared-index units of the row systems.
//
// For the update of mode n every entry needs delta = G contracted with the
// factor rows of all other modes (eq. "delta", Alg. 3). The permuted core is
// gp[m_1 .. m_{N-1}][j_n] with the other modes in ascending order, so for a
// fixed index o of the leading N-2 other modes the block gp[o] is a J x J
// matrix over (m_s, j_n), s being the last other mode. Then
//
//   delta[j] = sum_o w(o) t_o[j],   t_o[j] = sum_m gp[o][m][j] a^(s)[m],
//
// where w(o) is the product of the leading modes' factor values. t_o depends
// on the entry only through i_s: a unit of e entries of one row that share
// i_s forms t_o once (J^2 multiply-adds per o) and applies it to each of its
// entries (J each), instead of J^2 + J per entry. With the entries of every
// row ordered by i_s (ptk_sort.hip) the units are runs of consecutive
// entries. One lane per unit (two for units of one or two entries, so that
// every core value read through the scalar cache feeds two or more
// multiply-adds); the shared row and the accumulators sit in VGPRs, the
// unit's entries' rows of the leading modes but the first in lane-private
// LDS, and those of the first leading mode, whose value changes once per J^(N-3)
// outer indices, are read from memory one value ahead. Deltas are written in the
// grouped order ([nnz][J], a unit's deltas contiguous), and k_gram_stored
// sweeps them into the row systems tile by tile, in the same entry order as
// the fused kernels.
#include <algorithm>

#include "ptk_device.h"
#include "ptk_units.h"

namespace ptk {

// One lane holds P units of E entries. The leading other modes' rows of the
// lane's entries sit in lane-private LDS, except, with G0, those of the
// first leading mode (its value changes once per J^(N-3) outer indices),
// which are read from memory where they are used (cache hits). JS > 1 forms
// delta in JS passes over slices of J / JS of its components, so that the
// accumulators of large units fit in fewer registers; the core is read once
// over all passes. W is the occupancy the registers are allocated for.
template <int N, int J, int E, int P, int JS, bool G0, int W, int WG>
__global__ __launch_bounds__(kWave * WG, W) void k_delta_units(UnitArgs a) {
    constexpr int NO = N - 1;
    constexpr int NOUT = NO - 1;                 // leading other modes
    constexpr int K0 = G0 ? 1 : 0;               // leading modes read from memory
    constexpr int NL = NOUT - K0;                // leading modes in LDS
    constexpr int OUTER = ipow(J, NOUT);
    constexpr int SLOTS = P * E;                 // entries per lane
    constexpr int JW = J / JS;                   // delta components per pass
    static_assert(NOUT >= 1, "order 3 or more");
    static_assert(J % JS == 0, "passes split J evenly");
    // [wave][slot][k][j][lane]
    __shared__ float s_all[WG * (NL > 0 ? NL : 1) * J * SLOTS * kWave];

    const int lane = threadIdx.x % kWave;
    const int wave = threadIdx.x / kWave;
    float *s_a = s_all + wave * ((NL > 0 ? NL : 1) * J * SLOTS * kWave);
    const int64_t u0 = ((int64_t)blockIdx.x * WG + wave) * (P * kWave) + lane;
    int64_t pos[P];
    bool valid[P];
    double as[P][J];
    const float *r0[SLOTS];                      // rows of the first leading mode (G0)
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int64_t u = u0 + (int64_t)p * kWave;
        valid[p] = u < a.count;
        pos[p] = valid[p] ? a.units[u] : 0;
        const float *r = a.fac[NO - 1] + (int64_t)a.oidx[NO - 1][pos[p]] * J;
#pragma unroll
        for (int j = 0; j < J; ++j) as[p][j] = (double)r[j];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int64_t q = valid[p] ? pos[p] + e : 0;
            if constexpr (G0) r0[p * E + e] = a.fac[0] + (int64_t)a.oidx[0][q] * J;
#pragma unroll
            for (int k = K0; k < NOUT; ++k) {
                const float *row = a.fac[k] + (int64_t)a.oidx[k][q] * J;
#pragma unroll
                for (int j = 0; j < J; ++j)
                    s_a[(((p * E + e) * NL + k - K0) * J + j) * kWave + lane] = row[j];
            }
        }
    }
    __syncthreads();

    cptr<double> gp = (cptr<double>)(JS > 1 ? a.gph : a.gp);
#pragma unroll 1
    for (int h = 0; h < JS; ++h) {
        double c[SLOTS][JW];
#pragma unroll
        for (int sl = 0; sl < SLOTS; ++sl)
#pragma unroll
            for (int j = 0; j < JW; ++j) c[sl][j] = 0.0;
        float w0[SLOTS];                         // first leading mode's values (G0)
        for (int o = 0; o < OUTER; ++o) {
            int d[NOUT];
            int rest = o;
#pragma unroll
            for (int k = NOUT - 1; k >= 0; --k) {
                d[k] = rest % J;
                rest /= J;
            }
            // the waves of the workgroup read each core block together, so
            // that the scalar cache serves all but the first of them
            if constexpr (WG > 1) __syncthreads();
            if constexpr (G0) {
                if (o % (OUTER / J) == 0) {      // its digit changed (uniform branch)
#pragma unroll
                    for (int sl = 0; sl < SLOTS; ++sl) w0[sl] = r0[sl][d[0]];
                }
            }
            // the entries' weights first: their LDS reads share a wait
            // counter with the scalar loads of the core, so they are issued
            // together, ahead of them
            double w[SLOTS];
#pragma unroll
            for (int sl = 0; sl < SLOTS; ++sl) {
                double x = G0 ? (double)w0[sl] : 1.0;
#pragma unroll
                for (int k = 0; k < NL; ++k)
                    x *= (double)s_a[((sl * NL + k) * J + d[k + K0]) * kWave + lane];
                w[sl] = x;
            }
            // block (h, o) of the pass-major core: J rows of JW values
            cptr<double> g = gp + ((int64_t)h * OUTER + o) * (J * JW);
            double t[P][JW];
#pragma unroll
            for (int j = 0; j < JW; ++j) {
                const double gv = g[j];
#pragma unroll
                for (int p = 0; p < P; ++p) t[p][j] = gv * as[p][0];
            }
#pragma unroll
            for (int m = 1; m < J; ++m)
#pragma unroll
                for (int j = 0; j < JW; ++j) {
                    const double gv = g[m * JW + j];
#pragma unroll
                    for (int p = 0; p < P; ++p) t[p][j] = __builtin_fma(gv, as[p][m], t[p][j]);
                }
#pragma unroll
            for (int sl = 0; sl < SLOTS; ++sl)
#pragma unroll
                for (int j = 0; j < JW; ++j)
                    c[sl][j] = __builtin_fma(t[sl / E][j], w[sl], c[sl][j]);
        }
#pragma unroll
        for (int p = 0; p < P; ++p) {
            if (!valid[p]) continue;
            double *dst = a.dout + pos[p] * J + h * JW;
#pragma unroll
            for (int e = 0; e < E; ++e)
#pragma unroll
                for (int j = 0; j < JW; ++j) dst[e * J + j] = c[p * E + e][j];
        }
    }
}

// Single-entry units, two per lane, J <= 10: the general kernel with E = 1
// and P = 2 written out plainly (in this form the compiler keeps several
// scalar loads of the core in flight and needs no scalar spills).
template <int N, int J>
__global__ __launch_bounds__(kWave) void k_delta_singles(UnitArgs a) {
    constexpr int NO = N - 1;
    constexpr int NOUT = NO - 1;
    constexpr int OUTER = ipow(J, NOUT);
    constexpr int P = 2;
    __shared__ float s_a[NOUT * J * P * kWave];     // [unit][k][j][lane]
    const int lane = threadIdx.x;
    const int64_t u0 = (int64_t)blockIdx.x * (P * kWave) + lane;
    int64_t pos[P];
    bool valid[P];
    double as[P][J];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int64_t u = u0 + (int64_t)p * kWave;
        valid[p] = u < a.count;
        pos[p] = valid[p] ? a.units[u] : 0;
        const float *r = a.fac[NO - 1] + (int64_t)a.oidx[NO - 1][pos[p]] * J;
#pragma unroll
        for (int j = 0; j < J; ++j) as[p][j] = (double)r[j];
#pragma unroll
        for (int k = 0; k < NOUT; ++k) {
            const float *row = a.fac[k] + (int64_t)a.oidx[k][pos[p]] * J;
#pragma unroll
            for (int j = 0; j < J; ++j) s_a[((p * NOUT + k) * J + j) * kWave + lane] = row[j];
        }
    }
    __syncthreads();
    double c[P][J];
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int j = 0; j < J; ++j) c[p][j] = 0.0;
    cptr<double> gp = (cptr<double>)a.gp;
    for (int o = 0; o < OUTER; ++o) {
        int d[NOUT];
        int rest = o;
#pragma unroll
        for (int k = NOUT - 1; k >= 0; --k) {
            d[k] = rest % J;
            rest /= J;
        }
        double w[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            double x = (double)s_a[((p * NOUT + 0) * J + d[0]) * kWave + lane];
#pragma unroll
            for (int k = 1; k < NOUT; ++k)
                x *= (double)s_a[((p * NOUT + k) * J + d[k]) * kWave + lane];
            w[p] = x;
        }
        cptr<double> g = gp + (int64_t)o * (J * J);
        double t[P][J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const double gv = g[j];
#pragma unroll
            for (int p = 0; p < P; ++p) t[p][j] = gv * as[p][0];
        }
#pragma unroll
        for (int m = 1; m < J; ++m)
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const double gv = g[m * J + j];
#pragma unroll
                for (int p = 0; p < P; ++p) t[p][j] = __builtin_fma(gv, as[p][m], t[p][j]);
            }
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int j = 0; j < J; ++j) c[p][j] = __builtin_fma(t[p][j], w[p], c[p][j]);
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
        if (!valid[p]) continue;
        double *dst = a.dout + pos[p] * J;
#pragma unroll
        for (int j = 0; j < J; ++j) dst[j] = c[p][j];
    }
}

// gph[h][o][m][jj] = gp[o][m][h * JW + jj]: the core in the order of the
// passes of a JS-pass unit kernel, so that each pass reads contiguous rows.
__global__ void k_core_passes(const double *__restrict__ gp, double *__restrict__ gph, int J,
                              int JS, int64_t outer) {
    const int JW = J / JS;
    const int64_t total = outer * J * J;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t o = i / (J * J);
        const int r = (int)(i - o * J * J);
        const int m = r / J, j = r - m * J;
        const int h = j / JW, jj = j - h * JW;
        gph[((h * outer + o) * J + m) * JW + jj] = gp[i];
    }
}

hipError_t launch_core_passes(const double *gp, double *gph, int N, int J, hipStream_t st) {
    int64_t outer = 1;
    for (int k = 0; k < N - 2; ++k) outer *= J;
    const int JS = units_passes(N, J);
    if (JS <= 1) return hipSuccess;
    const int64_t total = outer * J * J;
    const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 1024);
    hipLaunchKernelGGL(k_core_passes, dim3(blocks), dim3(256), 0, st, gp, gph, J, JS, outer);
    return hipGetLastError();
}

// Tables of the long runs, two runs per lane and a slice of the outer
// indices per workgroup row: T[r][o][j] = sum_m gp[o][m][j] a^(s)_{i_s}[m],
// the core values read through the scalar cache as in k_delta_singles.
template <int N, int J>
__global__ __launch_bounds__(kWave) void k_run_tables(LongArgs a) {
    constexpr int NO = N - 1;
    constexpr int OUTER = ipow(J, N - 2);
    constexpr int P = 2;
    const int lane = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * (P * kWave) + lane;
    int64_t run[P];
    bool valid[P];
    double as[P][J];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        run[p] = r0 + (int64_t)p * kWave;
        valid[p] = run[p] < a.lg.n_long;
        const float *r;
        if (a.index_tables) {             // run_pos names the value
            r = a.fac[NO - 1] + (int64_t)(valid[p] ? a.lg.run_pos[run[p]] : 0) * J;
        } else {
            const int64_t pos = valid[p] ? a.lg.run_pos[run[p]] : 0;
            r = a.fac[NO - 1] + (int64_t)a.oidx[NO - 1][pos] * J;
        }
#pragma unroll
        for (int j = 0; j < J; ++j) as[p][j] = (double)r[j];
    }
    cptr<double> gp = (cptr<double>)a.gp;
    // the outer indices are cut into gridDim.y slices, one per workgroup row
    const int o_begin = (int)((int64_t)blockIdx.y * OUTER / gridDim.y);
    const int o_end = (int)((int64_t)(blockIdx.y + 1) * OUTER / gridDim.y);
#pragma unroll 1
    for (int o = o_begin; o < o_end; ++o) {
        cptr<double> g = gp + (int64_t)o * (J * J);
        double t[P][J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const double gv = g[j];
#pragma unroll
            for (int p = 0; p < P; ++p) t[p][j] = gv * as[p][0];
        }
#pragma unroll
        for (int m = 1; m < J; ++m)
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const double gv = g[m * J + j];
#pragma unroll
                for (int p = 0; p < P; ++p) t[p][j] = __builtin_fma(gv, as[p][m], t[p][j]);
            }
#pragma unroll
        for (int p = 0; p < P; ++p) {
            if (!valid[p]) continue;
            // tables [run][o][j]: each contiguous, so that a task's scalar
            // loads walk one block in order
            double *dst = a.tab + (run[p] * OUTER + o) * J;
#pragma unroll
            for (int j = 0; j < J; ++j) dst[j] = t[p][j];
        }
    }
}

// Deltas of a long run's task: one wavefront, two entries per lane. The
// run's table is uniform over the wavefront and is read through the scalar
// cache, J values per outer index, each feeding two multiply-adds; the row
// of the fastest leading mode sits in VGPRs, the slower ones' rows in LDS
// (read once per J outer indices).
template <int N, int J, int P>
__global__ __launch_bounds__(kWave) void k_delta_long(LongArgs a) {
    constexpr int NO = N - 1;
    constexpr int NOUT = NO - 1;                 // leading other modes
    constexpr int NS = NOUT - 1;                 // slow ones (LDS)
    constexpr int OUTER = ipow(J, NOUT);
    constexpr int OB = OUTER / J;                // outer indices of the slow modes
    __shared__ float s_a[(NS > 0 ? NS : 1) * J * P * kWave];   // [p][k][j][lane]
    const int lane = threadIdx.x;
    const int64_t task = blockIdx.x;
    const int64_t tpos = a.lg.task_pos[task];
    const int tlen = a.lg.task_len[task];
    const int64_t run = a.lg.task_run[task];
    int64_t pos[P];
    bool valid[P];
    double af[P][J];                             // fastest leading mode's row
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int off = lane + p * kWave;
        valid[p] = off < tlen;
        const int64_t k = tpos + (valid[p] ? off : 0);
        pos[p] = a.perm ? (int64_t)a.perm[k] : k;
        const float *r = a.fac[NOUT - 1] + (int64_t)a.oidx[NOUT - 1][pos[p]] * J;
#pragma unroll
        for (int j = 0; j < J; ++j) af[p][j] = (double)r[j];
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            const float *row = a.fac[k] + (int64_t)a.oidx[k][pos[p]] * J;
#pragma unroll
            for (int j = 0; j < J; ++j) s_a[((p * NS + k) * J + j) * kWave + lane] = row[j];
        }
    }
    __syncthreads();
    double c[P][J];
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int j = 0; j < J; ++j) c[p][j] = 0.0;
    // this task's table, [o][j] contiguous
    const int64_t os = J;
    cptr<double> tab = (cptr<double>)(a.tab + run * (OUTER * J));
#pragma unroll 1
    for (int ob = 0; ob < OB; ++ob) {
        double ws[P];
#pragma unroll
        for (int p = 0; p < P; ++p) ws[p] = 1.0;
        if constexpr (NS > 0) {
            int d[NS > 0 ? NS : 1];
            int rest = ob;
#pragma unroll
            for (int k = NS - 1; k >= 0; --k) {
                d[k] = rest % J;
                rest /= J;
            }
#pragma unroll
            for (int p = 0; p < P; ++p)
#pragma unroll
                for (int k = 0; k < NS; ++k)
                    ws[p] *= (double)s_a[((p * NS + k) * J + d[k]) * kWave + lane];
        }
        cptr<double> tb = tab + (int64_t)ob * J * os;
#pragma unroll(J <= 10 ? J : 4)
        for (int dl = 0; dl < J; ++dl) {
            double w[P];
#pragma unroll
            for (int p = 0; p < P; ++p) w[p] = ws[p] * af[p][dl];
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const double tv = tb[dl * os + j];
#pragma unroll
                for (int p = 0; p < P; ++p) c[p][j] = __builtin_fma(tv, w[p], c[p][j]);
            }
        }
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
        if (!valid[p]) continue;
        double *dst = a.dout + pos[p] * J;
#pragma unroll
        for (int j = 0; j < J; ++j) dst[j] = c[p][j];
    }
}

// Row systems from stored deltas: per work range, tiles of 64 entries in
// grouped order; the tile's deltas (64 * J contiguous doubles) are read with
// coalesced loads into the LDS layout of sweep_tile.
template <int J>
__global__ __launch_bounds__(kWave) void k_gram_stored(GramArgs a, const double *din) {
    constexpr int E = sys_entries(J);
    constexpr int EPL = (E + kWave - 1) / kWave;
    __shared__ double s_dl[(J + 1) * kDlStride];
    __shared__ int s_row[kWave];
    const int lane = threadIdx.x;
    const int64_t chunk = blockIdx.x;
    const int64_t cs = chunk * a.chunk;
    const int64_t ce = min(cs + a.chunk, a.nnz);
    SysLane<EPL> sl;
    sl.init(lane, J);
    int cur = -1;
    for (int64_t base = cs; base < ce; base += kWave) {
        const int nb = (int)min((int64_t)kWave, ce - base);
        const double *src = din + base * J;
        for (int q = lane; q < nb * J; q += kWave) {
            const int e = q / J;
            s_dl[(q - e * J) * kDlStride + e] = src[q];
        }
        const int64_t p = base + lane;
        const bool v = lane < nb;
        const int row = v ? a.rows[p] : 0;
        s_dl[J * kDlStride + lane] = v ? (double)a.val[p] : 0.0;
        s_row[lane] = row;
        __syncthreads();
        if (a.kbase && v) {                      // deltas of least-squares rows
            const int64_t kb = a.kbase[row];
            if (kb != kNoKeep) {
#pragma unroll
                for (int j = 0; j < J; ++j) a.keep[(kb + p) * J + j] = s_dl[j * kDlStride + lane];
            }
        }
        if (cur >= 0 && __ballot(v && row != cur) == 0) {
            // the whole tile continues the open row: no row checks; a
            // slot that only a few lanes use is summed by a wave reduction
            // over the tile's entries instead of a masked pass per entry
#pragma unroll
            for (int t = 0; t < EPL; ++t) {
                constexpr int kFull = E / kWave;
                if (t < kFull) {
                    const double *pp = s_dl + sl.p[t] * kDlStride;
                    const double *qq = s_dl + sl.q[t] * kDlStride;
                    double acc = sl.acc[t];
#pragma unroll 8
                    for (int b = 0; b < nb; ++b) acc = __builtin_fma(pp[b], qq[b], acc);
                    sl.acc[t] = acc;
                } else if constexpr (E - kFull * kWave <= 4) {
#pragma unroll
                    for (int k = 0; k < E - kFull * kWave; ++k) {
                        const int pk = __shfl(sl.p[t], k), qk = __shfl(sl.q[t], k);
                        double x = v ? s_dl[pk * kDlStride + lane] * s_dl[qk * kDlStride + lane]
                                     : 0.0;
#pragma unroll
                        for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_xor(x, off);
                        if (lane == k) sl.acc[t] += x;
                    }
                } else {
                    if (sl.e[t] >= 0) {
                        const double *pp = s_dl + sl.p[t] * kDlStride;
                        const double *qq = s_dl + sl.q[t] * kDlStride;
                        double acc = sl.acc[t];
                        for (int b = 0; b < nb; ++b) acc = __builtin_fma(pp[b], qq[b], acc);
                        sl.acc[t] = acc;
                    }
                }
            }
        } else {
            sweep_tile<EPL>(a, sl, s_dl, s_row, nb, cur, chunk, cs, ce);
        }
        __syncthreads();
    }
    if (cur >= 0) flush_row<EPL>(a, sl, cur, chunk, cs, ce);
}

#define PTK_UNIT_SHAPES(X) X(3, 16) X(4, 10) X(5, 8)

bool units_available(int N, int J) {
#define PTK_X(n_, j_) \
    if (N == n_ && J == j_) return true;
    PTK_UNIT_SHAPES(PTK_X)
#undef PTK_X
    return false;
}

// Passes of the multi-pass unit kernels at (N, J) (the pass-major core they
// read).
constexpr int passes_of(int N, int J) { return N == 5 ? 1 : 2; }

int units_passes(int N, int J) { return passes_of(N, J); }

// Per class c (units of 2^c entries): units per lane P, passes JS (1 or
// passes_of), first leading mode from memory G0, and the occupancy W the
// registers are allocated for (1: the compiler's choice). Chosen by
// measurement on the order-4 workload; single-entry units at J <= 10 use
// k_delta_singles.
template <int N, int J, int C>
struct UnitCfg {
    static constexpr int E = 1 << C;
    static constexpr int P = E == 1 ? 2 : 1;
    static constexpr int JS = (E == 8 || J > 10) ? passes_of(N, J) : 1;
    static constexpr bool G0 = E >= 4 && N >= 4;
    static constexpr int W = E == 2 ? 4 : E == 4 ? 3 : E == 8 ? 2 : 1;
    static constexpr int WG = 1;
};

template <int N, int J, int C>
hipError_t launch_units_c(const UnitArgs &a, hipStream_t st) {
    using K = UnitCfg<N, J, C>;
    if constexpr (C == 0 && J <= 10) {
        const int64_t per = K::P * (int64_t)kWave;
        const unsigned blocks = (unsigned)((a.count + per - 1) / per);
        hipLaunchKernelGGL((k_delta_singles<N, J>), dim3(blocks), dim3(kWave), 0, st, a);
    } else {
        const int64_t per = K::P * (int64_t)kWave * K::WG;
        const unsigned blocks = (unsigned)((a.count + per - 1) / per);
        hipLaunchKernelGGL((k_delta_units<N, J, K::E, K::P, K::JS, K::G0, K::W, K::WG>),
                           dim3(blocks), dim3(kWave * K::WG), 0, st, a);
    }
    return hipGetLastError();
}

template <int N, int J>
hipError_t launch_units_nj(const UnitArgs &a, int c, hipStream_t st) {
    constexpr int EMAX = units_emax(N, J);
    switch (c) {
    case 0: return launch_units_c<N, J, 0>(a, st);
    case 1: return launch_units_c<N, J, 1>(a, st);
    case 2: return launch_units_c<N, J, 2>(a, st);
    case 3:
        if constexpr (EMAX >= 8) return launch_units_c<N, J, 3>(a, st);
        return hipErrorInvalidValue;
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_delta_units(const UnitArgs &a, int N, int J, int c, hipStream_t st) {
    if (a.count <= 0) return hipSuccess;
    if (a.count >= (int64_t(1) << 31)) return hipErrorInvalidValue;
#define PTK_X(n_, j_) \
    if (N == n_ && J == j_) return launch_units_nj<n_, j_>(a, c, st);
    PTK_UNIT_SHAPES(PTK_X)
#undef PTK_X
    return hipErrorInvalidValue;
}

template <int N, int J>
hipError_t launch_tables_nj(const LongArgs &a, hipStream_t st) {
    if (a.lg.n_long <= 0) return hipSuccess;
    const unsigned rb = (unsigned)((a.lg.n_long + 2 * kWave - 1) / (2 * kWave));
    // enough workgroups to fill the chip: slices of the outer indices
    constexpr int OUTER = ipow(J, N - 2);
    const unsigned slices = (unsigned)std::max<int64_t>(
        1, std::min<int64_t>(OUTER, (8192 + rb - 1) / rb));
    hipLaunchKernelGGL((k_run_tables<N, J>), dim3(rb, slices), dim3(kWave), 0, st, a);
    return hipGetLastError();
}

template <int N, int J>
hipError_t launch_tasks_nj(const LongArgs &a, int P, hipStream_t st) {
    if (a.lg.n_long <= 0) return hipSuccess;
    if (a.lg.n_tasks > 0 && P == 1)
        hipLaunchKernelGGL((k_delta_long<N, J, 1>), dim3((unsigned)a.lg.n_tasks), dim3(kWave),
                           0, st, a);
    else if (a.lg.n_tasks > 0)
        hipLaunchKernelGGL((k_delta_long<N, J, 2>), dim3((unsigned)a.lg.n_tasks), dim3(kWave),
                           0, st, a);
    return hipGetLastError();
}

hipError_t launch_run_tables(const LongArgs &a, int N, int J, hipStream_t st) {
#define PTK_X(n_, j_) \
    if (N == n_ && J == j_) return launch_tables_nj<n_, j_>(a, st);
    PTK_UNIT_SHAPES(PTK_X)
#undef PTK_X
    return hipErrorInvalidValue;
}

hipError_t launch_long_tasks(const LongArgs &a, int N, int J, int P, hipStream_t st) {
    if (a.lg.n_tasks >= (int64_t(1) << 31) || (P != 1 && P != 2)) return hipErrorInvalidValue;
#define PTK_X(n_, j_) \
    if (N == n_ && J == j_) return launch_tasks_nj<n_, j_>(a, P, st);
    PTK_UNIT_SHAPES(PTK_X)
#undef PTK_X
    return hipErrorInvalidValue;
}

hipError_t launch_long_runs(const LongArgs &a, int N, int J, int P, hipStream_t st) {
    hipError_t e = launch_run_tables(a, N, J, st);
    if (e != hipSuccess) return e;
    return launch_long_tasks(a, N, J, P, st);
}

int gram_stored_blocks_per_cu(int J) {
    if (J == 8) return blocks_per_cu(k_gram_stored<8>, 0);
    if (J == 10) return blocks_per_cu(k_gram_stored<10>, 0);
    if (J == 16) return blocks_per_cu(k_gram_stored<16>, 0);
    return 8;
}

hipError_t launch_gram_stored(const GramArgs &a, int J, const double *din, int64_t nchunks,
                              hipStream_t st) {
    if (nchunks <= 0) return hipSuccess;
    if (!a.rows) return hipErrorInvalidValue;
#define PTK_G(j_)                                                                         \
    if (J == j_) {                                                                        \
        hipLaunchKernelGGL((k_gram_stored<j_>), dim3((unsigned)nchunks), dim3(kWave), 0, \
                           st, a, din);                                                   \
        return hipGetLastError();                                                         \
    }
    PTK_G(8)
    PTK_G(10)
    PTK_G(16)
#undef PTK_G
    return hipErrorInvalidValue;
}

double plain_fma_per_entry(int N, int J) {
    double f = 0.0, p = 1.0;
    for (int k = 0; k < N; ++k) {
        p *= J;
        if (k >= 1) f += p;           // J^2 + ... + J^N
    }
    return f;
}

double unit_fma(int N, int J, int e) {
    double outer = 1.0;
    for (int k = 0; k < N - 2; ++k) outer *= J;
    // per outer index: J^2 for t, then J per entry and N-3 weight products
    return outer * ((double)J * J + e * ((double)J + (N - 3)));
}

double stored_delta_fma(int J) { return 15.0 * (8.0 * J + 8.0); }

double long_fma(int N, int J, double runs, double entries) {
    double cells = 1.0, inner = 1.0;
    for (int k = 0; k < N; ++k) cells *= J;
    for (int k = 0; k < N - 1; ++k) inner *= J;
    return runs * cells + entries * (inner + inner / J);
}

}  // namespace ptk
