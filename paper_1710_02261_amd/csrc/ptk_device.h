// Device building blocks shared by the row-system kernels (ptk_kernels.hip)
// and the pair-cache kernels (ptk_cache.hip): the delta contraction with
// the core in SGPRs, the loading of the other factor rows, and the sweep
// that forms the packed row systems from a tile of deltas in LDS.
#pragma once

#include "ptk_internal.h"

namespace ptk {

template <typename T>
using cptr = const __attribute__((address_space(4))) T *;

template <typename T>
__device__ __forceinline__ T fma_t(T a, T b, T c);
template <>
__device__ __forceinline__ float fma_t<float>(float a, float b, float c) {
    return __builtin_fmaf(a, b, c);
}
template <>
__device__ __forceinline__ double fma_t<double>(double a, double b, double c) {
    return __builtin_fma(a, b, c);
}

// unrolled (VGPR-resident) other modes of the fast kernels
constexpr int fast_depth(int N, int J) {
    return (N - 1 <= 1) ? 1 : ((J >= 12) ? 1 : 2);
}

// ---------------------------------------------------------------------------
// fast delta: equal ranks J, N-1 other modes, the last U of them unrolled
// ---------------------------------------------------------------------------
template <int J, int U, int L, typename T>
__device__ __forceinline__ void inner_accum(cptr<T> g, T w, const T (&ain)[U][J],
                                            T (&acc)[J]) {
    if constexpr (L == U) {
#pragma unroll
        for (int j = 0; j < J; ++j) acc[j] = fma_t<T>(g[j], w, acc[j]);
    } else {
        constexpr int st = ipow(J, U - L);
#pragma unroll
        for (int m = 0; m < J; ++m)
            inner_accum<J, U, L + 1, T>(g + m * st, w * ain[L][m], ain, acc);
    }
}

// aout: lane-private LDS rows of the leading NO-U other modes, [k][j][64].
template <int NO, int J, int U, typename T>
__device__ __forceinline__ void delta_fast(const void *gp_raw, const float *aout,
                                           int lane, const T (&ain)[U][J],
                                           double (&out)[J]) {
    constexpr int NOUT = NO - U;
    constexpr int OUTER = ipow(J, NOUT);
    constexpr int BLOCK = ipow(J, U) * J;
    const void *gq = gp_raw;
    // With every other mode unrolled (NOUT = 0), or a core small enough for
    // the outer loop to be unrolled, the core loads do not depend on the
    // entry: without this opaque copy of the pointer the compiler hoists all
    // J^N scalar loads out of the caller's loop over tiles and spills them.
    // The core is then read again per tile from the scalar cache, like the
    // blocks of the larger shapes.
    if constexpr (NOUT == 0 || OUTER * BLOCK <= 256) asm volatile("" : "+s"(gq));
    cptr<T> gp = (cptr<T>)gq;
#pragma unroll
    for (int j = 0; j < J; ++j) out[j] = 0.0;
    for (int o = 0; o < OUTER; ++o) {
        T w = (T)1;
        int t = o;
#pragma unroll
        for (int k = NOUT - 1; k >= 0; --k) {
            const int d = t % J;
            t /= J;
            w *= (T)aout[(k * J + d) * kWave + lane];
        }
        if constexpr (sizeof(T) == 8) {
            inner_accum<J, U, 0, T>(gp + (int64_t)o * BLOCK, w, ain, out);
        } else {
            T acc[J];
#pragma unroll
            for (int j = 0; j < J; ++j) acc[j] = (T)0;
            inner_accum<J, U, 0, T>(gp + (int64_t)o * BLOCK, w, ain, acc);
#pragma unroll
            for (int j = 0; j < J; ++j) out[j] += (double)acc[j];
        }
    }
}

// Load the other-mode rows of one entry: leading modes to LDS, last U to VGPRs.
template <int NO, int J, int U, typename T, typename Args>
__device__ __forceinline__ void load_rows_fast(const Args &a, int64_t pos,
                                               bool valid, float *aout, int lane,
                                               T (&ain)[U][J]) {
    constexpr int NOUT = NO - U;
#pragma unroll
    for (int k = 0; k < NO; ++k) {
        const int32_t i = valid ? a.oidx[k][pos] : 0;
        const float *r = a.fac[k] + (int64_t)i * J;
        if (k < NOUT) {
#pragma unroll
            for (int j = 0; j < J; ++j) aout[(k * J + j) * kWave + lane] = r[j];
        } else {
#pragma unroll
            for (int j = 0; j < J; ++j) ain[k - NOUT][j] = (T)r[j];
        }
    }
}

// ---------------------------------------------------------------------------
// generic delta: any ranks (J_k <= 32), any order; mode-n rank <= JMAX
// ---------------------------------------------------------------------------
constexpr int kMaxOther = kMaxN - 1;

template <int JMAX, typename Args>
__device__ __forceinline__ void load_rows_generic(const Args &a, int64_t pos,
                                                  bool valid, float *arow,
                                                  int lane) {
    for (int k = 0; k < a.nother; ++k) {
        const int32_t i = valid ? a.oidx[k][pos] : 0;
        const int jk = a.jk[k];
        const float *r = a.fac[k] + (int64_t)i * jk;
        for (int j = 0; j < jk; ++j) arow[(a.aoff[k] + j) * kWave + lane] = r[j];
    }
}

template <int JMAX, typename Args>
__device__ __forceinline__ void delta_generic(const Args &a, const float *arow,
                                              int lane, double (&out)[JMAX]) {
    cptr<double> gp = (cptr<double>)a.gp;
    const int jn = a.jn;
    const int no = a.nother;
    int jk[kMaxOther], off[kMaxOther], dig[kMaxOther];
    int64_t P = 1;
#pragma unroll
    for (int k = 0; k < kMaxOther; ++k) {
        jk[k] = (k < no) ? a.jk[k] : 1;
        off[k] = (k < no) ? a.aoff[k] : 0;
        dig[k] = 0;
        P *= jk[k];
    }
#pragma unroll
    for (int j = 0; j < JMAX; ++j) out[j] = 0.0;
    for (int64_t o = 0; o < P; ++o) {
        double w = 1.0;
#pragma unroll
        for (int k = 0; k < kMaxOther; ++k)
            if (k < no) w *= (double)arow[(off[k] + dig[k]) * kWave + lane];
        cptr<double> g = gp + o * jn;
#pragma unroll
        for (int j = 0; j < JMAX; ++j)
            if (j < jn) out[j] = __builtin_fma(g[j], w, out[j]);
        // advance the odometer, last other mode fastest
        bool carry = true;
#pragma unroll
        for (int k = kMaxOther - 1; k >= 0; --k) {
            if (carry && k < no) {
                if (++dig[k] == jk[k])
                    dig[k] = 0;
                else
                    carry = false;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// row-system sweep over one tile of deltas in LDS
// ---------------------------------------------------------------------------
// s_dl layout: [j][65] doubles, row J holds the values x (stride 65 keeps the
// per-lane writes and the per-entry reads free of bank conflicts).
constexpr int kDlStride = kWave + 1;

template <int EPL>
struct SysLane {
    int p[EPL], q[EPL];
    int e[EPL];
    double acc[EPL];

    __device__ void init(int lane, int J) {
        const int T = J * (J + 1) / 2;
        const int E = T + J;
#pragma unroll
        for (int t = 0; t < EPL; ++t) {
            int ee = lane + kWave * t;
            e[t] = ee < E ? ee : -1;
            int pp = 0, qq = 0;
            if (ee < T) {
                // invert tri_pos: row pp holds J - pp entries
                int r = ee;
                while (r >= J - pp) {
                    r -= J - pp;
                    ++pp;
                }
                qq = pp + r;
            } else if (ee < E) {
                pp = ee - T;
                qq = J;      // the value row
            }
            p[t] = pp;
            q[t] = qq;
            acc[t] = 0.0;
        }
    }
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int t = 0; t < EPL; ++t) acc[t] = 0.0;
    }
    __device__ __forceinline__ void add(const double *s_dl, int b) {
#pragma unroll
        for (int t = 0; t < EPL; ++t)
            if (e[t] >= 0)
                acc[t] = __builtin_fma(s_dl[p[t] * kDlStride + b],
                                       s_dl[q[t] * kDlStride + b], acc[t]);
    }
    __device__ __forceinline__ void store(double *dst) const {
#pragma unroll
        for (int t = 0; t < EPL; ++t)
            if (e[t] >= 0) dst[e[t]] = acc[t];
    }
};

template <int EPL>
__device__ __forceinline__ void flush_row(const GramArgs &a, SysLane<EPL> &sl,
                                          int cur, int64_t chunk, int64_t cs,
                                          int64_t ce) {
    if (cur == a.skip_row) return;     // padding entries of a request batch
    const int64_t r0 = a.rowptr[cur], r1 = a.rowptr[cur + 1];
    double *dst;
    if (r0 < cs)
        dst = a.part + (chunk * 2 + 0) * a.E;
    else if (r1 > ce)
        dst = a.part + (chunk * 2 + 1) * a.E;
    else
        dst = a.bbuf + (int64_t)cur * a.E;
    sl.store(dst);
}

// Sweep the nb deltas of a tile into the open row systems.
template <int EPL>
__device__ __forceinline__ void sweep_tile(const GramArgs &a, SysLane<EPL> &sl,
                                           const double *s_dl, const int *s_row,
                                           int nb, int &cur, int64_t chunk,
                                           int64_t cs, int64_t ce) {
    for (int b = 0; b < nb; ++b) {
        const int r = __builtin_amdgcn_readfirstlane(s_row[b]);
        if (r != cur) {
            if (cur >= 0) flush_row<EPL>(a, sl, cur, chunk, cs, ce);
            cur = r;
            sl.zero();
        }
        sl.add(s_dl, b);
    }
}

// Resident single-wave blocks of a kernel per CU (host side).
template <typename K>
inline int blocks_per_cu(K kernel, size_t dyn) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, kWave, dyn) !=
        hipSuccess)
        return 8;
    return nb > 0 ? nb : 1;
}

}  // namespace ptk
