// Row-system kernel with two entries per lane (same contraction as
// k_gram_fast). Every core value read from the scalar cache feeds two
// multiply-adds, one per entry, instead of one: the scalar loads per FMA are
// halved, at the price of twice the accumulator and factor-row registers.
// A tile is 128 entries: lane l owns entries base + l and base + 64 + l,
// whose deltas are swept into the row systems as two 64-entry halves in
// entry order, so the sums are formed in the same order as k_gram_fast.
#include "ptk_device.h"

namespace ptk {

template <int J, int U, int L, typename T>
__device__ __forceinline__ void inner_accum2(cptr<T> g, T w0, T w1, const T (&a0)[U][J],
                                             const T (&a1)[U][J], T (&c0)[J], T (&c1)[J]) {
    if constexpr (L == U) {
#pragma unroll
        for (int j = 0; j < J; ++j) {
            c0[j] = fma_t<T>(g[j], w0, c0[j]);
            c1[j] = fma_t<T>(g[j], w1, c1[j]);
        }
    } else {
        constexpr int st = ipow(J, U - L);
#pragma unroll
        for (int m = 0; m < J; ++m)
            inner_accum2<J, U, L + 1, T>(g + m * st, w0 * a0[L][m], w1 * a1[L][m], a0, a1, c0,
                                         c1);
    }
}

// aout: lane-private LDS rows of the leading NO-U other modes for both
// entries, [k][j][128] (entry base + l in column l, base + 64 + l in 64 + l).
template <int NO, int J, int U, typename T>
__device__ __forceinline__ void delta_fast2(const void *gp_raw, const float *aout, int lane,
                                            const T (&a0)[U][J], const T (&a1)[U][J],
                                            double (&o0)[J], double (&o1)[J]) {
    constexpr int NOUT = NO - U;
    constexpr int OUTER = ipow(J, NOUT);
    constexpr int BLOCK = ipow(J, U) * J;
    const void *gq = gp_raw;
    // keep small cores from being hoisted out of the tile loop (see delta_fast)
    if constexpr (NOUT == 0 || OUTER * BLOCK <= 256) asm volatile("" : "+s"(gq));
    cptr<T> gp = (cptr<T>)gq;
#pragma unroll
    for (int j = 0; j < J; ++j) o0[j] = o1[j] = 0.0;
    for (int o = 0; o < OUTER; ++o) {
        T w0 = (T)1, w1 = (T)1;
        int t = o;
#pragma unroll
        for (int k = NOUT - 1; k >= 0; --k) {
            const int d = t % J;
            t /= J;
            w0 *= (T)aout[(k * J + d) * (2 * kWave) + lane];
            w1 *= (T)aout[(k * J + d) * (2 * kWave) + kWave + lane];
        }
        if constexpr (sizeof(T) == 8) {
            inner_accum2<J, U, 0, T>(gp + (int64_t)o * BLOCK, w0, w1, a0, a1, o0, o1);
        } else {
            T c0[J], c1[J];
#pragma unroll
            for (int j = 0; j < J; ++j) c0[j] = c1[j] = (T)0;
            inner_accum2<J, U, 0, T>(gp + (int64_t)o * BLOCK, w0, w1, a0, a1, c0, c1);
#pragma unroll
            for (int j = 0; j < J; ++j) {
                o0[j] += (double)c0[j];
                o1[j] += (double)c1[j];
            }
        }
    }
}

// KEEP: also store every entry's delta to a.dstore ([J][nnz], grouped order).
template <int N, int J, int U, typename T, bool KEEP>
__global__ __launch_bounds__(kWave) void k_gram_fast2(GramArgs a) {
    if (a.skip_if && *a.skip_if) return;
    constexpr int NO = N - 1;
    constexpr int NOUT = NO - U;
    constexpr int E = sys_entries(J);
    constexpr int EPL = (E + kWave - 1) / kWave;
    constexpr int AOUT = (NOUT > 0 ? NOUT : 1) * J * 2 * kWave;   // floats
    constexpr int DL = (J + 1) * kDlStride;                       // doubles
    constexpr int LDS_BYTES = (AOUT * 4 > DL * 8) ? AOUT * 4 : DL * 8;
    __shared__ __attribute__((aligned(16))) unsigned char s_raw[LDS_BYTES];
    __shared__ int s_row[kWave];
    float *s_aout = (float *)s_raw;
    double *s_dl = (double *)s_raw;

    const int lane = threadIdx.x;
    const int64_t chunk = blockIdx.x;
    const int64_t cs = chunk * a.chunk;
    const int64_t ce = min(cs + a.chunk, a.nnz);
    SysLane<EPL> sl;
    sl.init(lane, J);
    int cur = -1;
    for (int64_t base = cs; base < ce; base += 2 * kWave) {
        const int64_t p0 = base + lane, p1 = base + kWave + lane;
        const bool v0 = p0 < ce, v1 = p1 < ce;
        const int nb0 = (int)min((int64_t)kWave, ce - base);
        const int nb1 = (int)max((int64_t)0, min((int64_t)kWave, ce - base - kWave));
        T a0[U][J], a1[U][J];
#pragma unroll
        for (int k = 0; k < NO; ++k) {
            const float *r0 = a.fac[k] + (int64_t)(v0 ? a.oidx[k][p0] : 0) * J;
            const float *r1 = a.fac[k] + (int64_t)(v1 ? a.oidx[k][p1] : 0) * J;
            if (k < NOUT) {
#pragma unroll
                for (int j = 0; j < J; ++j) {
                    s_aout[(k * J + j) * (2 * kWave) + lane] = r0[j];
                    s_aout[(k * J + j) * (2 * kWave) + kWave + lane] = r1[j];
                }
            } else {
#pragma unroll
                for (int j = 0; j < J; ++j) {
                    a0[k - NOUT][j] = (T)r0[j];
                    a1[k - NOUT][j] = (T)r1[j];
                }
            }
        }
        __syncthreads();
        double d0[J], d1[J];
        delta_fast2<NO, J, U, T>(a.gp, s_aout, lane, a0, a1, d0, d1);
        if constexpr (KEEP) {
#pragma unroll
            for (int j = 0; j < J; ++j) {
                if (v0) a.dstore[(int64_t)j * a.nnz + p0] = d0[j];
                if (v1) a.dstore[(int64_t)j * a.nnz + p1] = d1[j];
            }
        }
        if (a.kbase) {                       // deltas of least-squares rows
            const int64_t k0 = v0 ? a.kbase[a.rows ? a.rows[p0] : 0] : kNoKeep;
            const int64_t k1 = v1 ? a.kbase[a.rows ? a.rows[p1] : 0] : kNoKeep;
            if (k0 != kNoKeep) {
#pragma unroll
                for (int j = 0; j < J; ++j) a.keep[(k0 + p0) * J + j] = d0[j];
            }
            if (k1 != kNoKeep) {
#pragma unroll
                for (int j = 0; j < J; ++j) a.keep[(k1 + p1) * J + j] = d1[j];
            }
        }
        __syncthreads();
        // first half: entries base .. base + 63
#pragma unroll
        for (int j = 0; j < J; ++j) s_dl[j * kDlStride + lane] = d0[j];
        s_dl[J * kDlStride + lane] = v0 ? (double)a.val[p0] : 0.0;
        s_row[lane] = v0 ? a.rows[p0] : 0;
        __syncthreads();
        sweep_tile<EPL>(a, sl, s_dl, s_row, nb0, cur, chunk, cs, ce);
        __syncthreads();
        if (nb1 > 0) {                             // uniform
#pragma unroll
            for (int j = 0; j < J; ++j) s_dl[j * kDlStride + lane] = d1[j];
            s_dl[J * kDlStride + lane] = v1 ? (double)a.val[p1] : 0.0;
            s_row[lane] = v1 ? a.rows[p1] : 0;
            __syncthreads();
            sweep_tile<EPL>(a, sl, s_dl, s_row, nb1, cur, chunk, cs, ce);
            __syncthreads();
        }
    }
    if (cur >= 0) flush_row<EPL>(a, sl, cur, chunk, cs, ce);
}

#define PTK_FAST2_SHAPES(X) X(4, 10, double, 1) X(5, 8, double, 2)

bool gram2_available(int N, int J, Arith ar) {
#define PTK_X(n_, j_, t_, u_) \
    if (N == n_ && J == j_ && (sizeof(t_) == 8) == (ar == kArithF64)) return true;
    PTK_FAST2_SHAPES(PTK_X)
#undef PTK_X
    return false;
}

int gram2_blocks_per_cu(int N, int J, Arith ar) {
#define PTK_X(n_, j_, t_, u_)                                                             \
    if (N == n_ && J == j_ && (sizeof(t_) == 8) == (ar == kArithF64))                   \
        return blocks_per_cu(k_gram_fast2<n_, j_, u_, t_, false>, 0);
    PTK_FAST2_SHAPES(PTK_X)
#undef PTK_X
    return 1;
}

hipError_t launch_gram2(const GramArgs &a, int N, int J, Arith ar, int64_t nchunks,
                        hipStream_t st) {
    if (nchunks <= 0) return hipSuccess;
#define PTK_X(n_, j_, t_, u_)                                                             \
    if (N == n_ && J == j_ && (sizeof(t_) == 8) == (ar == kArithF64)) {                 \
        if (a.dstore)                                                                     \
            hipLaunchKernelGGL((k_gram_fast2<n_, j_, u_, t_, true>),                     \
                               dim3((unsigned)nchunks), dim3(kWave), 0, st, a);           \
        else                                                                              \
            hipLaunchKernelGGL((k_gram_fast2<n_, j_, u_, t_, false>),                    \
                               dim3((unsigned)nchunks), dim3(kWave), 0, st, a);           \
        return hipGetLastError();                                                         \
    }
    PTK_FAST2_SHAPES(PTK_X)
#undef PTK_X
    return hipErrorInvalidValue;
}

}  // namespace ptk
