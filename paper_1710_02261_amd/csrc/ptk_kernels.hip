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
#include "ptk_device.h"

namespace ptk {

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

// ---------------------------------------------------------------------------
// Gram kernels
// ---------------------------------------------------------------------------
template <int N, int J, int U, typename T>
__global__ __launch_bounds__(kWave) void k_gram_fast(GramArgs a) {
    if (a.skip_if && *a.skip_if) return;
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
        if (a.kbase && valid) {              // deltas of least-squares rows
            const int64_t kb = a.kbase[row];
            if (kb != kNoKeep) {
#pragma unroll
                for (int j = 0; j < J; ++j) a.keep[(kb + pos) * J + j] = d[j];
            }
        }
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

template <int JMAX>
__global__ __launch_bounds__(kWave) void k_gram_generic(GramArgs a) {
    if (a.skip_if && *a.skip_if) return;
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
    X(3, 3) X(3, 4) X(3, 5) X(3, 7) X(3, 8) X(3, 9) X(3, 10) X(3, 11) X(3, 16) \
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
