// Pair-cache kernels of the row-wise ALS sweep (the reduced Cache variant of
// Alg. 3, Sec. 3.3). Modes are paired (n, n+1): while mode n is updated,
// every entry stores G contracted with the rows of all modes except n and
// n+1 (one record of J*J doubles), and mode n+1 then forms its deltas from
// that record and the new mode-n row, J*J multiply-adds instead of J^N.
#include "ptk_device.h"

namespace ptk {

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

// Writer with EL entries per lane (as k_gram_multi for the plain path): each
// core value from the scalar cache feeds EL multiply-adds. U is the number
// of unrolled (VGPR) levels after the partner; the records of a lane's EL
// entries are stored as in k_gram_cache_write.
template <int J, int U, int L, typename T, int EL>
__device__ __forceinline__ void inner_accum_el(cptr<T> g, const T (&w)[EL],
                                               const T (&a)[EL][U][J], T (&c)[EL][J]) {
    if constexpr (L == U) {
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const T gj = g[j];
#pragma unroll
            for (int e = 0; e < EL; ++e) c[e][j] = fma_t<T>(gj, w[e], c[e][j]);
        }
    } else {
        constexpr int st = ipow(J, U - L);
#pragma unroll
        for (int m = 0; m < J; ++m) {
            T wm[EL];
#pragma unroll
            for (int e = 0; e < EL; ++e) wm[e] = w[e] * a[e][L][m];
            inner_accum_el<J, U, L + 1, T, EL>(g + m * st, wm, a, c);
        }
    }
}

template <int N, int J, int U, typename T, int EL>
__global__ __launch_bounds__(kWave) void k_gram_cache_write_el(GramArgs a) {
    constexpr int NO = N - 1;
    constexpr int NOUT = NO - U;                 // partner + NMID mid levels
    constexpr int NMID = NO - 1 - U;
    constexpr int MID = ipow(J, NMID);
    constexpr int BLOCK = ipow(J, U) * J;
    constexpr int RS = cache_record(J);
    constexpr int E = sys_entries(J);
    constexpr int EPL = (E + kWave - 1) / kWave;
    constexpr int W = EL * kWave;                // LDS row stride
    constexpr int AOUT = NOUT * J * W;           // floats
    constexpr int DL = (J + 1) * kDlStride;      // doubles
    constexpr int LDS_BYTES = (AOUT * 4 > DL * 8) ? AOUT * 4 : DL * 8;
    static_assert(NOUT >= 1, "the partner is the leading LDS level");
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
    cptr<T> gp = (cptr<T>)a.gp;
    for (int64_t base = cs; base < ce; base += W) {
        T av[EL][U][J];
#pragma unroll
        for (int k = 0; k < NO; ++k) {
#pragma unroll
            for (int e = 0; e < EL; ++e) {
                const int64_t p = base + e * kWave + lane;
                const float *r = a.fac[k] + (int64_t)(p < ce ? a.oidx[k][p] : 0) * J;
                if (k < NOUT) {
#pragma unroll
                    for (int j = 0; j < J; ++j) s_aout[(k * J + j) * W + e * kWave + lane] = r[j];
                } else {
#pragma unroll
                    for (int j = 0; j < J; ++j) av[e][k - NOUT][j] = (T)r[j];
                }
            }
        }
        __syncthreads();
        double d[EL][J];
#pragma unroll
        for (int e = 0; e < EL; ++e)
#pragma unroll
            for (int j = 0; j < J; ++j) d[e][j] = 0.0;
#pragma unroll 1
        for (int o = 0; o < J; ++o) {
            T acc[EL][J];
#pragma unroll
            for (int e = 0; e < EL; ++e)
#pragma unroll
                for (int j = 0; j < J; ++j) acc[e][j] = (T)0;
#pragma unroll 1
            for (int mo = 0; mo < MID; ++mo) {
                T w[EL];
                // unit weight from LDS (keeps the inner weight products in the loop)
#pragma unroll
                for (int e = 0; e < EL; ++e) w[e] = (T)s_ones[o];
                int t = mo;
#pragma unroll
                for (int k = NMID; k >= 1; --k) {
                    const int dg = t % J;
                    t /= J;
#pragma unroll
                    for (int e = 0; e < EL; ++e)
                        w[e] *= (T)s_aout[(k * J + dg) * W + e * kWave + lane];
                }
                inner_accum_el<J, U, 0, T, EL>(gp + ((int64_t)o * MID + mo) * BLOCK, w, av, acc);
            }
#pragma unroll
            for (int e = 0; e < EL; ++e) {
                const int64_t p = base + e * kWave + lane;
                double *tdst = a.cache + (p < ce ? p : a.nnz) * RS;   // spare record
                const double wp = (double)s_aout[o * W + e * kWave + lane];
#pragma unroll
                for (int j = 0; j < J; ++j) {
                    tdst[o * J + j] = (double)acc[e][j];
                    d[e][j] = __builtin_fma(wp, (double)acc[e][j], d[e][j]);
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < EL; ++e) {
            const int64_t p = base + e * kWave + lane;
            const int nb = (int)max((int64_t)0, min((int64_t)kWave, ce - base - e * kWave));
            if (nb == 0) break;                    // uniform
#pragma unroll
            for (int j = 0; j < J; ++j) s_dl[j * kDlStride + lane] = d[e][j];
            s_dl[J * kDlStride + lane] = p < ce ? (double)a.val[p] : 0.0;
            s_row[lane] = p < ce ? a.rows[p] : 0;
            __syncthreads();
            sweep_tile<EPL>(a, sl, s_dl, s_row, nb, cur, chunk, cs, ce);
            __syncthreads();
        }
    }
    if (cur >= 0) flush_row<EPL>(a, sl, cur, chunk, cs, ce);
}

// shapes with a multi-entry writer: (N, J, type, U, entries per lane)
#define PTK_CACHE_EL_SHAPES(X) X(4, 10, double, 1, 2)

// Writer for any order (equal ranks J <= JMAX): the generic odometer walk
// over the other modes' cells with the partner p as the slowest digit. The
// J^(N-2) cells of one partner index m_p, summed without the partner's
// weight, are T[m_p][:]; delta adds a^(p)[m_p] T[m_p][:].
template <int JMAX, typename T>
__device__ __forceinline__ void delta_generic_store(const GramArgs &a, const float *arow,
                                                    int lane, double (&out)[JMAX],
                                                    double *tdst) {
    constexpr int KO = kMaxN - 1;
    cptr<T> gp = (cptr<T>)a.gp;
    const int jn = a.jn;
    const int no = a.nother;
    int jk[KO], off[KO];
    int64_t Q = 1;                                    // cells per partner index
#pragma unroll
    for (int k = 0; k < KO; ++k) {
        jk[k] = (k < no) ? a.jk[k] : 1;
        off[k] = (k < no) ? a.aoff[k] : 0;
        if (k >= 1) Q *= jk[k];
    }
#pragma unroll
    for (int j = 0; j < JMAX; ++j) out[j] = 0.0;
    for (int mp = 0; mp < jk[0]; ++mp) {
        double acc[JMAX];
#pragma unroll
        for (int j = 0; j < JMAX; ++j) acc[j] = 0.0;
        int dig[KO];
#pragma unroll
        for (int k = 0; k < KO; ++k) dig[k] = 0;
        cptr<T> g = gp + (int64_t)mp * Q * jn;
        for (int64_t o = 0; o < Q; ++o, g += jn) {
            double w = 1.0;
#pragma unroll
            for (int k = 1; k < KO; ++k)
                if (k < no) w *= (double)arow[(off[k] + dig[k]) * kWave + lane];
#pragma unroll
            for (int j = 0; j < JMAX; ++j)
                if (j < jn) acc[j] = __builtin_fma((double)g[j], w, acc[j]);
            // odometer over the non-partner modes, last one fastest
            bool carry = true;
#pragma unroll
            for (int k = KO - 1; k >= 1; --k) {
                if (carry && k < no) {
                    if (++dig[k] == jk[k])
                        dig[k] = 0;
                    else
                        carry = false;
                }
            }
        }
        const double wp = (double)arow[(off[0] + mp) * kWave + lane];
#pragma unroll
        for (int j = 0; j < JMAX; ++j) {
            if (j < jn) {
                tdst[mp * jn + j] = acc[j];
                out[j] = __builtin_fma(wp, acc[j], out[j]);
            }
        }
    }
}

template <int JMAX, typename T>
__global__ __launch_bounds__(kWave) void k_gram_cache_write_generic(GramArgs a) {
    constexpr int EPL = (sys_entries(JMAX) + kWave - 1) / kWave;
    extern __shared__ __attribute__((aligned(16))) unsigned char s_dyn[];
    __shared__ int s_row[kWave];
    const int lane = threadIdx.x;
    const int J = a.jn;
    const int RS = (J * J + 1) / 2 * 2;
    // LDS: [other-mode rows: sum jk x 64 floats][dl: (J+1) x kDlStride doubles]
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
        const int row = valid ? a.rows[pos] : 0;
        const float x = valid ? a.val[pos] : 0.0f;
        for (int k = 0; k < a.nother; ++k) {
            const int32_t i = valid ? a.oidx[k][pos] : 0;
            const int jk = a.jk[k];
            const float *r = a.fac[k] + (int64_t)i * jk;
            for (int j = 0; j < jk; ++j) s_arow[(a.aoff[k] + j) * kWave + lane] = r[j];
        }
        __syncthreads();
        double d[JMAX];
        // lanes past the range write the spare record at index nnz
        delta_generic_store<JMAX, T>(a, s_arow, lane, d,
                                     a.cache + (valid ? pos : a.nnz) * RS);
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

static size_t cache_generic_lds_bytes(const GramArgs &a) {
    int sumj = 0;
    for (int k = 0; k < a.nother; ++k) sumj += a.jk[k];
    const size_t arow = ((size_t)sumj * kWave * 4 + 15) / 16 * 16;
    return arow + (size_t)(a.jn + 1) * kDlStride * 8;
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


#define PTK_CACHE_SHAPES(X) \
    X(3, 3) X(3, 4) X(3, 5) X(3, 8) X(3, 10) X(3, 16) \
    X(4, 3) X(4, 5) X(4, 8) X(4, 10) \
    X(5, 3) X(5, 5) X(5, 8)

int cache_record_doubles(int J) { return cache_record(J); }

static bool cache_reader_rank(int J) {
    return J == 3 || J == 4 || J == 5 || J == 8 || J == 10 || J == 16;
}

// Any order from 3 up with a reader for rank J; the writer is the unrolled
// kernel for the listed shapes, else the generic one.
bool cache_available(int N, int J) {
    return N >= 3 && N <= kMaxN && cache_reader_rank(J);
}

template <typename T>
static int generic_writer_blocks(int J, size_t lds) {
    if (J <= 4) return blocks_per_cu(k_gram_cache_write_generic<4, T>, lds);
    if (J <= 8) return blocks_per_cu(k_gram_cache_write_generic<8, T>, lds);
    return blocks_per_cu(k_gram_cache_write_generic<16, T>, lds);
}

template <typename T>
static void launch_generic_writer(const GramArgs &a, dim3 grid, size_t lds, hipStream_t st) {
    dim3 block(kWave);
    if (a.jn <= 4)
        hipLaunchKernelGGL((k_gram_cache_write_generic<4, T>), grid, block, lds, st, a);
    else if (a.jn <= 8)
        hipLaunchKernelGGL((k_gram_cache_write_generic<8, T>), grid, block, lds, st, a);
    else
        hipLaunchKernelGGL((k_gram_cache_write_generic<16, T>), grid, block, lds, st, a);
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
#define PTK_Y(n_, j_, t_, u_, e_)                                                  \
    if (s.N == n_ && J == j_ && (sizeof(t_) == 8) == (ar == kArithF64))            \
        return blocks_per_cu(k_gram_cache_write_el<n_, j_, u_, t_, e_>, 0);
    PTK_CACHE_EL_SHAPES(PTK_Y)
#undef PTK_Y
#define PTK_X(n_, j_)                                                             \
    if (s.N == n_ && J == j_)                                                     \
        return ar == kArithF64 ? blocks_per_cu(k_gram_cache_write<n_, j_, double>, 0) \
                               : blocks_per_cu(k_gram_cache_write<n_, j_, float>, 0);
    PTK_CACHE_SHAPES(PTK_X)
#undef PTK_X
    GramArgs a{};
    a.nother = s.N - 1;
    a.jn = J;
    for (int k = 0; k < s.N - 1; ++k) a.jk[k] = J;
    const size_t lds = cache_generic_lds_bytes(a);
    return ar == kArithF64 ? generic_writer_blocks<double>(J, lds)
                           : generic_writer_blocks<float>(J, lds);
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
#define PTK_Y(n_, j_, t_, u_, e_)                                                     \
    if (s.N == n_ && J == j_ && (sizeof(t_) == 8) == (ar == kArithF64)) {             \
        hipLaunchKernelGGL((k_gram_cache_write_el<n_, j_, u_, t_, e_>), grid, block, 0, \
                           st, a);                                                    \
        return hipGetLastError();                                                     \
    }
    PTK_CACHE_EL_SHAPES(PTK_Y)
#undef PTK_Y
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
    if (J > 16 || a.nother != s.N - 1) return hipErrorInvalidValue;
    const size_t lds = cache_generic_lds_bytes(a);
    if (ar == kArithF64)
        launch_generic_writer<double>(a, grid, lds, st);
    else
        launch_generic_writer<float>(a, grid, lds, st);
    return hipGetLastError();
}

}  // namespace ptk
