// delta / row-system kernels of the row-wise ALS (gfx950, wave64).
//
// delta^(n)_alpha (Sec. 3.2, eq. "delta") is G contracted with the factor
// rows of every mode except n. With the core permuted so that the mode-n
// index is fastest (gp[m_1..m_{N-1}][j]), it is
//     delta[j] = sum_m w(m) gp[m][j],   w(m) = prod_{k != n} a^(k)_{i_k m_k},
// i.e. the Kronecker vector of the other rows times the mode-n unfolding of
// G. One lane owns one entry. The core is read with wavefront-uniform
// addresses, so it streams through the scalar cache into SGPRs and every
// multiply-add is a single v_fma with an SGPR operand; the factor rows of the
// last U other modes sit in VGPRs, those of the leading modes in lane-private
// LDS. The row systems B_i = sum delta delta^T, c_i = sum x delta
// (eqs. "rowB", "rowC") are then formed from the 64 deltas of a tile held in
// LDS: each lane owns entries of the packed system and sweeps the tile, so a
// row of any length is reduced by the same code.
//
// Work split (the GPU form of the dynamic schedule of Sec. 3.4): the entries
// of mode n, grouped by row, are cut into equal ranges of `chunk` entries,
// one wavefront each. Rows wholly inside a range are written to bbuf; the
// pieces of rows that cross range boundaries go to two partial slots per
// range and are merged in range order afterwards (deterministic).
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

// ---------------------------------------------------------------------------
// core permutation: gp[others in mode order][j_n] <- G (C order)
// ---------------------------------------------------------------------------
struct PermArgs {
    int32_t N, n;
    int32_t J[kMaxN];
    int32_t order[kMaxN];   // the other modes, leading first
    int64_t S;
};

template <typename T>
__global__ void k_permute_core(const float *__restrict__ G, T *__restrict__ gp,
                               PermArgs p) {
    int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= p.S) return;
    // decode d: last digit is j_n, then the other modes from last to first
    int64_t t = d;
    int digit[kMaxN];
    digit[p.n] = (int)(t % p.J[p.n]);
    t /= p.J[p.n];
    for (int q = p.N - 2; q >= 0; --q) {
        const int k = p.order[q];
        digit[k] = (int)(t % p.J[k]);
        t /= p.J[k];
    }
    int64_t src = 0;
    for (int k = 0; k < p.N; ++k) src = src * p.J[k] + digit[k];
    gp[d] = (T)G[src];
}

hipError_t launch_permute_core(const float *G, void *gp, const Shape &s, int n,
                               Arith ar, hipStream_t st, int lead) {
    PermArgs p;
    p.N = s.N;
    p.n = n;
    p.S = 1;
    for (int k = 0; k < s.N; ++k) {
        p.J[k] = s.ranks[k];
        p.S *= s.ranks[k];
    }
    int q = 0;
    if (lead >= 0) p.order[q++] = lead;
    for (int k = 0; k < s.N; ++k)
        if (k != n && k != lead) p.order[q++] = k;
    dim3 grid((unsigned)((p.S + 255) / 256));
    if (ar == kArithF64)
        hipLaunchKernelGGL(k_permute_core<double>, grid, dim3(256), 0, st, G,
                           (double *)gp, p);
    else
        hipLaunchKernelGGL(k_permute_core<float>, grid, dim3(256), 0, st, G,
                           (float *)gp, p);
    return hipGetLastError();
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
    cptr<T> gp = (cptr<T>)gp_raw;
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

// ---------------------------------------------------------------------------
// Gram kernels
// ---------------------------------------------------------------------------
template <int N, int J, int U, typename T>
__global__ __launch_bounds__(kWave) void k_gram_fast(GramArgs a) {
    constexpr int NO = N - 1;
    constexpr int NOUT = NO - U;
    constexpr int E = sys_entries(J);
    constexpr int EPL = (E + kWave - 1) / kWave;
    constexpr int AOUT = (NOUT > 0 ? NOUT : 1) * J * kWave;      // floats
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
    for (int64_t base = cs; base < ce; base += kWave) {
        const int64_t pos = base + lane;
        const bool valid = pos < ce;
        const int nb = (int)min((int64_t)kWave, ce - base);
        const int row = valid ? (a.rows ? a.rows[pos] : 0) : 0;
        const float x = valid ? a.val[pos] : 0.0f;
        T ain[U][J];
        load_rows_fast<NO, J, U, T>(a, pos, valid, s_aout, lane, ain);
        __syncthreads();
        double d[J];
        delta_fast<NO, J, U, T>(a.gp, s_aout, lane, ain, d);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < J; ++j) s_dl[j * kDlStride + lane] = d[j];
        s_dl[J * kDlStride + lane] = (double)x;
        s_row[lane] = row;
        __syncthreads();
        sweep_tile<EPL>(a, sl, s_dl, s_row, nb, cur, chunk, cs, ce);
        __syncthreads();
    }
    if (cur >= 0) flush_row<EPL>(a, sl, cur, chunk, cs, ce);
}

// ---------------------------------------------------------------------------
// pair cache: writer and reader kernels
// ---------------------------------------------------------------------------
// One record per entry: T[m_p][j_n] (J*J doubles, padded to an even count so
// that records are 16-byte aligned), i.e. G contracted with the rows of every
// mode except n (the writer) and its partner p.
constexpr int cache_record(int J) { return (J * J + 1) / 2 * 2; }

// Writer delta: the partner p is the leading other mode (outer loop over
// m_p), then NO-1-U runtime levels, then U unrolled levels. The sum over all
// but the partner, for one m_p, is T[m_p][:]; it is stored, and weighted by
// a^(p)[m_p] into delta.
template <int NO, int J, int U, typename T>
__device__ __forceinline__ void delta_fast_store(const void *gp_raw, const float *aout,
                                                 const float *ones, int lane,
                                                 const T (&ain)[U][J],
                                                 double (&out)[J], double *tdst) {
    constexpr int NMID = NO - 1 - U;
    constexpr int MID = ipow(J, NMID);
    constexpr int BLOCK = ipow(J, U) * J;
    cptr<T> gp = (cptr<T>)gp_raw;
#pragma unroll
    for (int j = 0; j < J; ++j) out[j] = 0.0;
#pragma unroll 1
    for (int o = 0; o < J; ++o) {
        T acc[J];
#pragma unroll
        for (int j = 0; j < J; ++j) acc[j] = (T)0;
#pragma unroll 1
        for (int mo = 0; mo < MID; ++mo) {
            // unit weight read from LDS at index o: the J^U inner weight
            // products (the same for every o when NMID = 0) are then not
            // hoisted out of the loop into registers
            T w = (T)ones[o];
            int t = mo;
#pragma unroll
            for (int k = NMID; k >= 1; --k) {
                const int d = t % J;
                t /= J;
                w *= (T)aout[(k * J + d) * kWave + lane];
            }
            inner_accum<J, U, 0, T>(gp + ((int64_t)o * MID + mo) * BLOCK, w, ain, acc);
        }
        const double wp = (double)aout[o * kWave + lane];
        // unconditional store (no lane branch inside the loop: a branch here
        // forces the scalar-loaded core values to be spilled)
#pragma unroll
        for (int j = 0; j < J; ++j) {
            tdst[o * J + j] = (double)acc[j];
            out[j] = __builtin_fma(wp, (double)acc[j], out[j]);
        }
    }
}

constexpr int cache_depth(int N, int J) {
    return fast_depth(N, J) < N - 2 ? fast_depth(N, J) : N - 2;
}

template <int N, int J, typename T>
__global__ __launch_bounds__(kWave) void k_gram_cache_write(GramArgs a) {
    constexpr int NO = N - 1;
    constexpr int U = cache_depth(N, J);
    constexpr int NOUT = NO - U;
    constexpr int RS = cache_record(J);
    constexpr int E = sys_entries(J);
    constexpr int EPL = (E + kWave - 1) / kWave;
    constexpr int AOUT = NOUT * J * kWave;                         // floats
    constexpr int DL = (J + 1) * kDlStride;                        // doubles
    constexpr int LDS_BYTES = (AOUT * 4 > DL * 8) ? AOUT * 4 : DL * 8;
    __shared__ __attribute__((aligned(16))) unsigned char s_raw[LDS_BYTES];
    __shared__ int s_row[kWave];
    __shared__ float s_ones[J];
    float *s_aout = (float *)s_raw;
    double *s_dl = (double *)s_raw;
    const int lane = threadIdx.x;
    const int64_t chunk = blockIdx.x;
    const int64_t cs = chunk * a.chunk;
    const int64_t ce = min(cs + a.chunk, a.nnz);
    if (lane < J) s_ones[lane] = 1.0f;
    SysLane<EPL> sl;
    sl.init(lane, J);
    int cur = -1;
    for (int64_t base = cs; base < ce; base += kWave) {
        const int64_t pos = base + lane;
        const bool valid = pos < ce;
        const int nb = (int)min((int64_t)kWave, ce - base);
        const int row = valid ? a.rows[pos] : 0;
        const float x = valid ? a.val[pos] : 0.0f;
        T ain[U][J];
        load_rows_fast<NO, J, U, T>(a, pos, valid, s_aout, lane, ain);
        __syncthreads();
        double d[J];
        // lanes past the range write the spare record at index nnz
        delta_fast_store<NO, J, U, T>(a.gp, s_aout, s_ones, lane, ain, d,
                                      a.cache + (valid ? pos : a.nnz) * RS);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < J; ++j) s_dl[j * kDlStride + lane] = d[j];
        s_dl[J * kDlStride + lane] = (double)x;
        s_row[lane] = row;
        __syncthreads();
        sweep_tile<EPL>(a, sl, s_dl, s_row, nb, cur, chunk, cs, ce);
        __syncthreads();
    }
    if (cur >= 0) flush_row<EPL>(a, sl, cur, chunk, cs, ce);
}

// Reader: delta^(p)[m] = sum_j a^(n)_{i_n}[j] T[m][j] with T written by the
// partner's update (same sweep, so the other modes have not changed since).
// Records sit at random writer positions: the wavefront loads them whole,
// one record per load instruction (full cache lines), eight in flight, into
// LDS, NR records per pass; each lane then reads its own record from LDS.
constexpr int cache_pass_records(int J) {
    return (64 * (cache_record(J) + 1) * 8 <= 32768)   ? 64
           : (32 * (cache_record(J) + 1) * 8 <= 32768) ? 32
           : (16 * (cache_record(J) + 1) * 8 <= 32768) ? 16
                                                       : 8;
}

template <int J>
__global__ __launch_bounds__(kWave) void k_gram_cache_read(GramArgs a) {
    constexpr int E = sys_entries(J);
    constexpr int EPL = (E + kWave - 1) / kWave;
    constexpr int RS = cache_record(J);
    constexpr int S = RS + 1;                 // odd LDS stride (in doubles)
    constexpr int NP = RS / 2;                // 16-byte pieces of a record
    constexpr int NR = cache_pass_records(J);
    __shared__ double s_dl[(J + 1) * kDlStride];
    __shared__ int s_row[kWave];
    __shared__ double s_t[NR * S];
    const int lane = threadIdx.x;
    const int64_t chunk = blockIdx.x;
    const int64_t cs = chunk * a.chunk;
    const int64_t ce = min(cs + a.chunk, a.nnz);
    SysLane<EPL> sl;
    sl.init(lane, J);
    int cur = -1;
    for (int64_t base = cs; base < ce; base += kWave) {
        const int64_t pos = base + lane;
        const bool valid = pos < ce;
        const int nb = (int)min((int64_t)kWave, ce - base);
        const int row = valid ? a.rows[pos] : 0;
        const float x = valid ? a.val[pos] : 0.0f;
        const int32_t q = valid ? a.cmap[pos] : 0;
        double av[J];
        {
            const int32_t in = valid ? a.oidx[a.cslot][pos] : 0;
            const float *an = a.fac[a.cslot] + (int64_t)in * J;
#pragma unroll
            for (int j = 0; j < J; ++j) av[j] = valid ? (double)an[j] : 0.0;
        }
        double d[J];
#pragma unroll
        for (int m = 0; m < J; ++m) d[m] = 0.0;
        for (int h = 0; h < kWave; h += NR) {
            if (h >= nb) break;                            // wave-uniform
            for (int e0 = 0; e0 < NR; e0 += 8) {
                double2 v[8][(NP + kWave - 1) / kWave];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int e = h + e0 + u;
                    const int64_t qe = __shfl(q, e);
#pragma unroll
                    for (int r = 0; r < (NP + kWave - 1) / kWave; ++r) {
                        const int k = lane + r * kWave;
                        v[u][r] = make_double2(0.0, 0.0);
                        if (e < nb && k < NP)
                            v[u][r] = *(const double2 *)(a.cache + qe * RS + 2 * k);
                    }
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
#pragma unroll
                    for (int r = 0; r < (NP + kWave - 1) / kWave; ++r) {
                        const int k = lane + r * kWave;
                        if (k < NP) {
                            s_t[(e0 + u) * S + 2 * k] = v[u][r].x;
                            s_t[(e0 + u) * S + 2 * k + 1] = v[u][r].y;
                        }
                    }
                }
            }
            __syncthreads();
            const int me = lane - h;
            if (me >= 0 && me < NR && valid) {
                const double *t = s_t + me * S;
#pragma unroll
                for (int m = 0; m < J; ++m) {
                    double acc = 0.0;
#pragma unroll
                    for (int j = 0; j < J; ++j) acc = __builtin_fma(av[j], t[m * J + j], acc);
                    d[m] = acc;
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int j = 0; j < J; ++j) s_dl[j * kDlStride + lane] = d[j];
        s_dl[J * kDlStride + lane] = (double)x;
        s_row[lane] = row;
        __syncthreads();
        sweep_tile<EPL>(a, sl, s_dl, s_row, nb, cur, chunk, cs, ce);
        __syncthreads();
    }
    if (cur >= 0) flush_row<EPL>(a, sl, cur, chunk, cs, ce);
}

template <int JMAX>
__global__ __launch_bounds__(kWave) void k_gram_generic(GramArgs a) {
    constexpr int EPL = (sys_entries(JMAX) + kWave - 1) / kWave;
    extern __shared__ __attribute__((aligned(16))) unsigned char s_dyn[];
    __shared__ int s_row[kWave];
    const int lane = threadIdx.x;
    const int J = a.jn;
    // LDS: [arow: sum jk x 64 floats][dl: (J+1) x 65 doubles], not aliased
    int sumj = 0;
    for (int k = 0; k < a.nother; ++k) sumj += a.jk[k];
    float *s_arow = (float *)s_dyn;
    double *s_dl = (double *)(s_dyn + ((sumj * kWave * 4 + 15) / 16) * 16);

    const int64_t chunk = blockIdx.x;
    const int64_t cs = chunk * a.chunk;
    const int64_t ce = min(cs + a.chunk, a.nnz);
    SysLane<EPL> sl;
    sl.init(lane, J);
    int cur = -1;
    for (int64_t base = cs; base < ce; base += kWave) {
        const int64_t pos = base + lane;
        const bool valid = pos < ce;
        const int nb = (int)min((int64_t)kWave, ce - base);
        const int row = valid ? (a.rows ? a.rows[pos] : 0) : 0;
        const float x = valid ? a.val[pos] : 0.0f;
        load_rows_generic<JMAX>(a, pos, valid, s_arow, lane);
        __syncthreads();
        double d[JMAX];
        delta_generic<JMAX>(a, s_arow, lane, d);
#pragma unroll
        for (int j = 0; j < JMAX; ++j)
            if (j < J) s_dl[j * kDlStride + lane] = d[j];
        s_dl[J * kDlStride + lane] = (double)x;
        s_row[lane] = row;
        __syncthreads();
        sweep_tile<EPL>(a, sl, s_dl, s_row, nb, cur, chunk, cs, ce);
        __syncthreads();
    }
    if (cur >= 0) flush_row<EPL>(a, sl, cur, chunk, cs, ce);
}

static size_t generic_lds_bytes(const GramArgs &a) {
    int sumj = 0;
    for (int k = 0; k < a.nother; ++k) sumj += a.jk[k];
    size_t arow = ((size_t)sumj * kWave * 4 + 15) / 16 * 16;
    return arow + (size_t)(a.jn + 1) * kDlStride * 8;
}

// ---------------------------------------------------------------------------
// per-entry kernels: deltas, predictions, squared residuals
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_reduce_sum(double v, double *s_red) {
    // one wavefront per block
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
    return v;   // lane 0 holds the sum
}

template <int J>
__device__ __forceinline__ void entry_out(const EntryArgs &a, int kind,
                                          int64_t pos, bool valid,
                                          const double (&d)[J], int jn,
                                          double &sse) {
    if (!valid) return;
    if (kind == kOutDelta) {
#pragma unroll
        for (int j = 0; j < J; ++j)
            if (j < jn) a.out[pos * jn + j] = (float)d[j];
        return;
    }
    const int32_t i = a.own_idx[pos];
    const float *r = a.own + (int64_t)i * jn;
    double xh = 0.0;
#pragma unroll
    for (int j = 0; j < J; ++j)
        if (j < jn) xh = __builtin_fma((double)r[j], d[j], xh);
    if (kind == kOutPredict) {
        a.out[pos] = (float)xh;
    } else {
        const double res = (double)a.val[pos] - xh;
        sse = __builtin_fma(res, res, sse);
    }
}

template <int N, int J, int U, typename T>
__global__ __launch_bounds__(kWave) void k_entries_fast(EntryArgs a, int kind) {
    constexpr int NO = N - 1;
    constexpr int NOUT = NO - U;
    __shared__ float s_aout[(NOUT > 0 ? NOUT : 1) * J * kWave];
    const int lane = threadIdx.x;
    double sse = 0.0;
    for (int64_t base = (int64_t)blockIdx.x * kWave; base < a.m;
         base += (int64_t)gridDim.x * kWave) {
        const int64_t pos = base + lane;
        const bool valid = pos < a.m;
        T ain[U][J];
        load_rows_fast<NO, J, U, T>(a, pos, valid, s_aout, lane, ain);
        __syncthreads();
        double d[J];
        delta_fast<NO, J, U, T>(a.gp, s_aout, lane, ain, d);
        __syncthreads();
        entry_out<J>(a, kind, pos, valid, d, J, sse);
    }
    if (kind == kOutSSE) {
        sse = block_reduce_sum(sse, nullptr);
        if (lane == 0) a.partial[blockIdx.x] = sse;
    }
}

template <int JMAX>
__global__ __launch_bounds__(kWave) void k_entries_generic(EntryArgs a, int kind) {
    extern __shared__ __attribute__((aligned(16))) unsigned char s_dyn[];
    float *s_arow = (float *)s_dyn;
    const int lane = threadIdx.x;
    double sse = 0.0;
    for (int64_t base = (int64_t)blockIdx.x * kWave; base < a.m;
         base += (int64_t)gridDim.x * kWave) {
        const int64_t pos = base + lane;
        const bool valid = pos < a.m;
        load_rows_generic<JMAX>(a, pos, valid, s_arow, lane);
        __syncthreads();
        double d[JMAX];
        delta_generic<JMAX>(a, s_arow, lane, d);
        __syncthreads();
        entry_out<JMAX>(a, kind, pos, valid, d, a.jn, sse);
    }
    if (kind == kOutSSE) {
        sse = block_reduce_sum(sse, nullptr);
        if (lane == 0) a.partial[blockIdx.x] = sse;
    }
}

// ---------------------------------------------------------------------------
// instantiation tables
// ---------------------------------------------------------------------------
// Unrolled depth U per (N, J): the unrolled body has J^(U+1) multiply-adds.

#define PTK_FAST_SHAPES(X) \
    X(3, 3) X(3, 4) X(3, 5) X(3, 8) X(3, 10) X(3, 16) \
    X(4, 3) X(4, 5) X(4, 8) X(4, 10) \
    X(5, 3) X(5, 5) X(5, 8)

bool fast_available(int N, int J, Arith) {
#define PTK_X(n_, j_) if (N == n_ && J == j_) return true;
    PTK_FAST_SHAPES(PTK_X)
#undef PTK_X
    return false;
}

static int generic_jmax(int jn) {
    return jn <= 4 ? 4 : jn <= 8 ? 8 : jn <= 16 ? 16 : 32;
}

template <typename K>
static int blocks_per_cu(K kernel, size_t dyn) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, kWave, dyn) !=
        hipSuccess)
        return 8;
    return nb > 0 ? nb : 1;
}

int gram_blocks_per_cu(const Shape &s, int n, Arith ar, bool fast) {
    const int J = s.ranks[n];
    if (fast) {
#define PTK_X(n_, j_)                                                           \
    if (s.N == n_ && J == j_) {                                                 \
        constexpr int U = fast_depth(n_, j_);                                   \
        return ar == kArithF64                                                  \
                   ? blocks_per_cu(k_gram_fast<n_, j_, U, double>, 0)          \
                   : blocks_per_cu(k_gram_fast<n_, j_, U, float>, 0);          \
    }
        PTK_FAST_SHAPES(PTK_X)
#undef PTK_X
    }
    GramArgs a{};
    a.nother = s.N - 1;
    a.jn = J;
    int t = 0;
    for (int k = 0; k < s.N; ++k)
        if (k != n) a.jk[t++] = s.ranks[k];
    const size_t lds = generic_lds_bytes(a);
    switch (generic_jmax(J)) {
        case 4: return blocks_per_cu(k_gram_generic<4>, lds);
        case 8: return blocks_per_cu(k_gram_generic<8>, lds);
        case 16: return blocks_per_cu(k_gram_generic<16>, lds);
        default: return blocks_per_cu(k_gram_generic<32>, lds);
    }
}

hipError_t launch_gram(const GramArgs &a, const Shape &s, int n, Arith ar,
                       int64_t nchunks, bool fast, hipStream_t st) {
    if (nchunks <= 0) return hipSuccess;
    dim3 grid((unsigned)nchunks), block(kWave);
    const int J = s.ranks[n];
    if (fast) {
#define PTK_X(n_, j_)                                                           \
    if (s.N == n_ && J == j_) {                                                 \
        constexpr int U = fast_depth(n_, j_);                                   \
        if (ar == kArithF64)                                                    \
            hipLaunchKernelGGL((k_gram_fast<n_, j_, U, double>), grid, block, 0, \
                               st, a);                                         \
        else                                                                    \
            hipLaunchKernelGGL((k_gram_fast<n_, j_, U, float>), grid, block, 0,  \
                               st, a);                                         \
        return hipGetLastError();                                               \
    }
        PTK_FAST_SHAPES(PTK_X)
#undef PTK_X
        return hipErrorInvalidValue;
    }
    const size_t lds = generic_lds_bytes(a);
    switch (generic_jmax(J)) {
        case 4:
            hipLaunchKernelGGL(k_gram_generic<4>, grid, block, lds, st, a);
            break;
        case 8:
            hipLaunchKernelGGL(k_gram_generic<8>, grid, block, lds, st, a);
            break;
        case 16:
            hipLaunchKernelGGL(k_gram_generic<16>, grid, block, lds, st, a);
            break;
        default:
            hipLaunchKernelGGL(k_gram_generic<32>, grid, block, lds, st, a);
            break;
    }
    return hipGetLastError();
}

#define PTK_CACHE_SHAPES(X) \
    X(3, 3) X(3, 4) X(3, 5) X(3, 8) X(3, 10) X(3, 16) \
    X(4, 3) X(4, 5) X(4, 8) X(4, 10) \
    X(5, 3) X(5, 5) X(5, 8)

int cache_record_doubles(int J) { return cache_record(J); }

bool cache_available(int N, int J) {
#define PTK_X(n_, j_) if (N == n_ && J == j_) return true;
    PTK_CACHE_SHAPES(PTK_X)
#undef PTK_X
    return false;
}

int gram_cache_blocks_per_cu(const Shape &s, int n, Arith ar, int cm) {
    const int J = s.ranks[n];
    if (cm == 2) {
        switch (J) {
            case 3: return blocks_per_cu(k_gram_cache_read<3>, 0);
            case 4: return blocks_per_cu(k_gram_cache_read<4>, 0);
            case 5: return blocks_per_cu(k_gram_cache_read<5>, 0);
            case 8: return blocks_per_cu(k_gram_cache_read<8>, 0);
            case 10: return blocks_per_cu(k_gram_cache_read<10>, 0);
            default: return blocks_per_cu(k_gram_cache_read<16>, 0);
        }
    }
#define PTK_X(n_, j_)                                                             \
    if (s.N == n_ && J == j_)                                                     \
        return ar == kArithF64 ? blocks_per_cu(k_gram_cache_write<n_, j_, double>, 0) \
                               : blocks_per_cu(k_gram_cache_write<n_, j_, float>, 0);
    PTK_CACHE_SHAPES(PTK_X)
#undef PTK_X
    return 1;
}

hipError_t launch_gram_cache(const GramArgs &a, const Shape &s, int n, Arith ar,
                             int64_t nchunks, int cm, hipStream_t st) {
    if (nchunks <= 0) return hipSuccess;
    dim3 grid((unsigned)nchunks), block(kWave);
    const int J = s.ranks[n];
    if (cm == 2) {
        switch (J) {
            case 3: hipLaunchKernelGGL(k_gram_cache_read<3>, grid, block, 0, st, a); break;
            case 4: hipLaunchKernelGGL(k_gram_cache_read<4>, grid, block, 0, st, a); break;
            case 5: hipLaunchKernelGGL(k_gram_cache_read<5>, grid, block, 0, st, a); break;
            case 8: hipLaunchKernelGGL(k_gram_cache_read<8>, grid, block, 0, st, a); break;
            case 10: hipLaunchKernelGGL(k_gram_cache_read<10>, grid, block, 0, st, a); break;
            case 16: hipLaunchKernelGGL(k_gram_cache_read<16>, grid, block, 0, st, a); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
#define PTK_X(n_, j_)                                                                \
    if (s.N == n_ && J == j_) {                                                      \
        if (ar == kArithF64)                                                         \
            hipLaunchKernelGGL((k_gram_cache_write<n_, j_, double>), grid, block, 0,  \
                               st, a);                                              \
        else                                                                         \
            hipLaunchKernelGGL((k_gram_cache_write<n_, j_, float>), grid, block, 0,   \
                               st, a);                                              \
        return hipGetLastError();                                                    \
    }
    PTK_CACHE_SHAPES(PTK_X)
#undef PTK_X
    return hipErrorInvalidValue;
}

hipError_t launch_entries(const EntryArgs &a, const Shape &s, int n, int kind,
                          bool fast, int64_t nblocks, hipStream_t st) {
    if (a.m <= 0 || nblocks <= 0) return hipSuccess;
    dim3 grid((unsigned)nblocks), block(kWave);
    const int J = s.ranks[n];
    if (fast) {
#define PTK_X(n_, j_)                                                           \
    if (s.N == n_ && J == j_) {                                                 \
        constexpr int U = fast_depth(n_, j_);                                   \
        hipLaunchKernelGGL((k_entries_fast<n_, j_, U, double>), grid, block, 0,  \
                           st, a, kind);                                       \
        return hipGetLastError();                                               \
    }
        PTK_FAST_SHAPES(PTK_X)
#undef PTK_X
        return hipErrorInvalidValue;
    }
    int sumj = 0;
    for (int k = 0; k < a.nother; ++k) sumj += a.jk[k];
    const size_t lds = (size_t)sumj * kWave * 4;
    switch (generic_jmax(J)) {
        case 4:
            hipLaunchKernelGGL(k_entries_generic<4>, grid, block, lds, st, a, kind);
            break;
        case 8:
            hipLaunchKernelGGL(k_entries_generic<8>, grid, block, lds, st, a, kind);
            break;
        case 16:
            hipLaunchKernelGGL(k_entries_generic<16>, grid, block, lds, st, a, kind);
            break;
        default:
            hipLaunchKernelGGL(k_entries_generic<32>, grid, block, lds, st, a, kind);
            break;
    }
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_sumsq(const float *__restrict__ x,
                                               int64_t n,
                                               double *__restrict__ partial) {
    __shared__ double s_part[4];
    double s = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x) {
        const double v = (double)x[e];
        s = __builtin_fma(v, v, s);
    }
    s = block_reduce_sum(s, nullptr);
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x % kWave) == 0) s_part[w] = s;
    __syncthreads();
    if (threadIdx.x == 0)
        partial[blockIdx.x] = ((s_part[0] + s_part[1]) + (s_part[2] + s_part[3]));
}

hipError_t launch_sumsq(const float *x, int64_t n, double *partial, int nblocks,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_sumsq, dim3(nblocks), dim3(256), 0, st, x, n, partial);
    return hipGetLastError();
}

// Sum n partials in a fixed order (one block; deterministic).
__global__ __launch_bounds__(256) void k_reduce(const double *__restrict__ partial,
                                                int n, double *__restrict__ out) {
    __shared__ double s[256];
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) v += partial[i];
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0];
}

hipError_t launch_reduce(const double *partial, int n, double *out,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, st, partial, n, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// packed row systems -> dense B [I][J][J], c [I][J] (inspection)
// ---------------------------------------------------------------------------
__global__ void k_expand(const double *__restrict__ bbuf,
                         const int64_t *__restrict__ rowptr, int64_t I, int J,
                         double *__restrict__ B, double *__restrict__ c) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= I) return;
    const int E = sys_entries(J);
    const bool empty = rowptr[i] == rowptr[i + 1];
    const double *s = bbuf + i * E;
    for (int p = 0; p < J; ++p) {
        for (int q = 0; q < J; ++q) {
            const int a = p <= q ? tri_pos(p, q, J) : tri_pos(q, p, J);
            B[(i * J + p) * J + q] = empty ? 0.0 : s[a];
        }
        c[i * J + p] = empty ? 0.0 : s[J * (J + 1) / 2 + p];
    }
}

hipError_t launch_expand_systems(const double *bbuf, const int64_t *rowptr,
                                 int64_t I, int J, double *B, double *c,
                                 hipStream_t st) {
    hipLaunchKernelGGL(k_expand, dim3((unsigned)((I + 127) / 128)), dim3(128), 0,
                       st, bbuf, rowptr, I, J, B, c);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// input validation: indices in range, values finite
// ---------------------------------------------------------------------------
struct ValArgs {
    int32_t N;
    int64_t dims[kMaxN];
};

__global__ void k_validate(const int32_t *__restrict__ idx,
                           const float *__restrict__ val, int64_t nnz, ValArgs v,
                           unsigned long long *bad) {
    unsigned long long nb_idx = 0, nb_val = 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x) {
        for (int k = 0; k < v.N; ++k) {
            const int32_t i = idx[(int64_t)k * nnz + e];
            if (i < 0 || (int64_t)i >= v.dims[k]) ++nb_idx;
        }
        if (!isfinite(val[e])) ++nb_val;
    }
    if (nb_idx) atomicAdd(&bad[0], nb_idx);
    if (nb_val) atomicAdd(&bad[1], nb_val);
}

hipError_t launch_validate(const int32_t *idx, const float *val, int64_t nnz,
                           const Shape &s, unsigned long long *bad,
                           hipStream_t st) {
    ValArgs v;
    v.N = s.N;
    for (int k = 0; k < s.N; ++k) v.dims[k] = s.dims[k];
    int64_t blocks = (nnz + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_validate, dim3((unsigned)blocks), dim3(256), 0, st, idx,
                       val, nnz, v, bad);
    return hipGetLastError();
}

}  // namespace ptk
