// Precision form of the row-system kernel: delta and the row Gram on the
// matrix cores in BF16 with FP32 accumulation (the solve stays FP64).
//
// delta^(n)_alpha (Sec. 3.2, eq. "delta") is contracted in two stages. With
// the other modes k_1 < ... < k_{N-1} of mode n, write the permuted core as
// gp[m_1..m_{N-2}][m_{N-1}][j]. Stage 1, on MFMA, contracts the last other
// mode for 16 entries at once: for every tile t = (m_1..m_{N-2}),
//     D_t[e][j] = sum_m a^(k_{N-1})_e[m] gp[t][m][j]
// (v_mfma_f32_16x16x16_bf16: A = the entries' factor rows, B = a core
// fragment kept in LDS). Stage 2, on the FP32 VALU, folds the remaining modes
// with the entries' own factor values: delta_e[j] = sum_t w_e(t) D_t[e][j].
// The row Gram B_i = sum delta delta^T (eq. "rowB") of a 32-entry block is
// one v_mfma_f32_16x16x32_bf16 whose A and B operands are the same registers:
// after stage 2 each lane holds delta_e[j] (j = lane % 16) for eight entries.
// The right-hand side c_i (eq. "rowC") is summed in FP32 on the VALU with the
// unrounded values. With SPLIT = 3 every FP32 operand x is carried as the pair
// hi = bf16(x), lo = bf16(x - hi) and each product as hi*hi + hi*lo + lo*hi
// (three MFMAs), which keeps about 16 significant bits instead of 8.
// Rows are padded to whole 32-entry blocks so that a block
// never spans two rows; wavefronts take equal runs of blocks, and rows that
// cross runs go to the partial slots merged by k_merge, as in the FP64 path.
#include "ptk_internal.h"

namespace ptk {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef short shortx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kMfmaWaves = 4;   // wavefronts per workgroup (share the core in LDS)
constexpr int kBlk = 32;        // entries per block (one Gram MFMA)

// LDS written by some lanes of a wavefront and read by other lanes of the
// same wavefront: keeps the compiler from moving LDS accesses across this
// point and waits for the wavefront's outstanding LDS operations. No other
// wavefront takes part, so the wavefronts of a workgroup run independently.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_s_waitcnt(0xc07f);         // lgkmcnt(0)
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// core fragments: frag[t][lane][u] = gp[t][4*(lane/16)+u][lane%16] (bf16, 0 pad)
// ---------------------------------------------------------------------------
struct FragArgs {
    int32_t N, n, J;
    int32_t rk[kMaxN];
    int64_t tiles;
};

// frag holds the hi parts; frag + tiles*256 the lo parts (x - hi).
__global__ void k_mfma_frags(const float *__restrict__ G, __bf16 *__restrict__ frag,
                             FragArgs f) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= f.tiles * kWave * 4) return;
    const int u = (int)(id % 4);
    const int lane = (int)((id / 4) % kWave);
    int64_t t = id / (4 * kWave);
    const int m = 4 * (lane / 16) + u;       // index of the last other mode
    const int j = lane % 16;                 // index of mode n
    float v = 0.0f;
    if (m < f.J && j < f.J) {
        // digits of the other modes: tile t enumerates all but the last
        int digit[kMaxN];
        digit[f.n] = j;
        int last = -1;
        for (int k = f.N - 1; k >= 0; --k)
            if (k != f.n) {
                last = k;
                break;
            }
        digit[last] = m;
        for (int k = f.N - 1; k >= 0; --k) {
            if (k == f.n || k == last) continue;
            digit[k] = (int)(t % f.J);
            t /= f.J;
        }
        int64_t src = 0;
        for (int k = 0; k < f.N; ++k) src = src * f.J + digit[k];
        v = G[src];
    }
    const __bf16 hi = (__bf16)v;
    frag[id] = hi;
    frag[f.tiles * kWave * 4 + id] = (__bf16)(v - (float)hi);
}

// ---------------------------------------------------------------------------
// the kernel
// ---------------------------------------------------------------------------
template <int N, int J, int SPLIT>
__global__ __launch_bounds__(kWave * kMfmaWaves, (N == 3 && SPLIT == 1) ? 8 : 4) void k_gram_mfma(
    MfmaArgs a) {
    constexpr int NO = N - 1;                 // other modes
    constexpr int NW = NO - 1;                // modes folded on the VALU
    constexpr int TILES = ipow(J, NW);
    constexpr int T = J * (J + 1) / 2;
    constexpr int NF = SPLIT == 3 ? 2 : 1;    // fragment sets (hi, lo)
    static_assert(J <= 16 && (N == 3 || N == 4), "shape");
    static_assert(SPLIT == 1 || SPLIT == 3, "split");
    extern __shared__ __attribute__((aligned(16))) unsigned char s_dyn[];
    bf16x4 *s_frag = (bf16x4 *)s_dyn;                                 // [NF][TILES][64]
    float *s_wall = (float *)(s_dyn + (size_t)NF * TILES * kWave * 8); // per wave
    const int wid = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    float *s_w = s_wall + wid * (NW * 16 * kBlk + kBlk);              // [NW][16][32]
    float *s_x = s_w + NW * 16 * kBlk;                                // [32]

    // core fragments -> LDS (whole workgroup)
    for (int i = threadIdx.x; i < NF * TILES * kWave; i += blockDim.x)
        s_frag[i] = ((const bf16x4 *)a.frag)[i];
    __syncthreads();

    const int64_t wave = (int64_t)blockIdx.x * kMfmaWaves + wid;
    const int64_t b0 = wave * a.blk_per_wave;
    const int64_t b1 = min(b0 + a.blk_per_wave, a.nblk);
    // after the fragments are in LDS the wavefronts only share read-only
    // data: each step synchronises its own wavefront only
    const int64_t cs = (b0 < b1) ? (int64_t)a.blk_start[b0] : 0;
    const int64_t ce = (b0 < b1) ? (int64_t)a.blk_start[b1 - 1] + a.blk_cnt[b1 - 1] : 0;
    const int g = lane / 16;                  // lane group
    const int j = lane % 16;                  // column (mode-n index)

    floatx4 Bacc = {0.f, 0.f, 0.f, 0.f};
    float cpart = 0.0f;
    int cur = -1;

    auto flush = [&](int row) {
        float c1 = cpart + __shfl_xor(cpart, 16, kWave);
        float c2 = c1 + __shfl_xor(c1, 32, kWave);
        const int64_t r0 = a.rowptr[row], r1 = a.rowptr[row + 1];
        double *dst;
        if (r0 < cs)
            dst = a.part + (wave * 2 + 0) * a.E;
        else if (r1 > ce)
            dst = a.part + (wave * 2 + 1) * a.E;
        else
            dst = a.bbuf + (int64_t)row * a.E;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 4 * g + r;
            if (i <= j && j < J) dst[tri_pos(i, j, J)] = (double)Bacc[r];
        }
        if (lane < J) dst[T + lane] = (double)c2;
    };

    for (int64_t step = 0; step < a.blk_per_wave; ++step) {
        const int64_t b = b0 + step;
        const bool active = b < b1;           // uniform per wavefront
        int row = 0, cnt = 0;
        int64_t start = 0;
        if (active) {
            row = a.blk_row[b];
            start = a.blk_start[b];
            cnt = a.blk_cnt[b];
            if (row != cur) {
                if (cur >= 0) flush(cur);
                cur = row;
                Bacc = floatx4{0.f, 0.f, 0.f, 0.f};
                cpart = 0.0f;
            }
        }
        // lanes 0..31 load their entry; stage-2 factor rows go to LDS
        const int e = lane;
        const bool valid = active && e < cnt;
        const int64_t pos = start + e;
        int32_t iL = 0;
        if (active && lane < kBlk) {
            iL = valid ? a.oidx[NO - 1][pos] : 0;
            s_x[e] = valid ? a.val[pos] : 0.0f;
#pragma unroll
            for (int k = 0; k < NW; ++k) {
                const int32_t ik = valid ? a.oidx[k][pos] : 0;
                const float *r = a.fac[k] + (int64_t)ik * J;
#pragma unroll
                for (int m = 0; m < J; ++m) s_w[(k * 16 + m) * kBlk + e] = r[m];
            }
        }
        // A operands: entry 16*mb + lane%16, columns 4g..4g+3 of its last row
        bf16x4 af[2], afl[2];
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
            const int32_t ie = __shfl(iL, 16 * mb + j, kWave);
            const float *r = a.fac[NO - 1] + (int64_t)ie * J;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int m = 4 * g + u;
                float v = 0.0f;
                if (m < J) v = r[m];
                af[mb][u] = (__bf16)v;
                afl[mb][u] = (__bf16)(v - (float)af[mb][u]);
            }
        }
        wave_lds_sync();
        if (active) {
        // D = A x B for one tile, with the split products when SPLIT = 3
        auto tile_product = [&](int mb, int t) -> floatx4 {
            const floatx4 z = {0.f, 0.f, 0.f, 0.f};
            const bf16x4 bf = s_frag[t * kWave + lane];
            floatx4 d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(
                __builtin_bit_cast(shortx4, af[mb]), __builtin_bit_cast(shortx4, bf), z,
                0, 0, 0);
            if constexpr (SPLIT == 3) {
                const bf16x4 bfl = s_frag[(TILES + t) * kWave + lane];
                d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(
                    __builtin_bit_cast(shortx4, af[mb]), __builtin_bit_cast(shortx4, bfl),
                    d, 0, 0, 0);
                d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(
                    __builtin_bit_cast(shortx4, afl[mb]), __builtin_bit_cast(shortx4, bf),
                    d, 0, 0, 0);
            }
            return d;
        };
        // stage 1 (MFMA) and stage 2 (VALU)
        floatx4 acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
        if constexpr (NW == 1) {
#pragma unroll 2
            for (int t = 0; t < TILES; ++t) {
#pragma unroll
                for (int mb = 0; mb < 2; ++mb) {
                    const floatx4 d = tile_product(mb, t);
                    const floatx4 w = *(const floatx4 *)&s_w[t * kBlk + 16 * mb + 4 * g];
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[mb][r] = __builtin_fmaf(w[r], d[r], acc[mb][r]);
                }
            }
        } else {
#pragma unroll 1
            for (int t1 = 0; t1 < J; ++t1) {
                floatx4 acc2[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
#pragma unroll 2
                for (int t2 = 0; t2 < J; ++t2) {
#pragma unroll
                    for (int mb = 0; mb < 2; ++mb) {
                        const floatx4 d = tile_product(mb, t1 * J + t2);
                        const floatx4 w =
                            *(const floatx4 *)&s_w[(16 + t2) * kBlk + 16 * mb + 4 * g];
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            acc2[mb][r] = __builtin_fmaf(w[r], d[r], acc2[mb][r]);
                    }
                }
#pragma unroll
                for (int mb = 0; mb < 2; ++mb) {
                    const floatx4 w = *(const floatx4 *)&s_w[t1 * kBlk + 16 * mb + 4 * g];
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        acc[mb][r] = __builtin_fmaf(w[r], acc2[mb][r], acc[mb][r]);
                }
            }
        }
        // this block's deltas: acc[mb][r] = delta_e[j], e = 16 mb + 4 g + r
        float dv[8];
        bf16x8 gv, gl;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int mb = u / 4, r = u % 4;
            const int ee = 16 * mb + 4 * g + r;
            const bool ok = ee < cnt && j < J;
            dv[u] = ok ? acc[mb][r] : 0.0f;
            gv[u] = (__bf16)dv[u];
            gl[u] = (__bf16)(dv[u] - (float)gv[u]);
            cpart = __builtin_fmaf(s_x[ee], dv[u], cpart);
        }
        Bacc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(gv, gv, Bacc, 0, 0, 0);
        if constexpr (SPLIT == 3) {
            Bacc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(gv, gl, Bacc, 0, 0, 0);
            Bacc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(gl, gv, Bacc, 0, 0, 0);
        }
        }
        wave_lds_sync();
    }
    if (cur >= 0) flush(cur);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
#define PTK_MFMA_SHAPES(X) X(3, 8) X(3, 10) X(3, 16) X(4, 8) X(4, 10)

bool mfma_available(int N, int J) {
#define PTK_X(n_, j_) if (N == n_ && J == j_) return true;
    PTK_MFMA_SHAPES(PTK_X)
#undef PTK_X
    return false;
}

int64_t mfma_tiles(int N, int J) { return ipow(J, N - 2); }

static size_t mfma_lds_bytes(int N, int J, int split) {
    const int NW = N - 2;
    const int nf = split == 3 ? 2 : 1;
    return (size_t)nf * mfma_tiles(N, J) * kWave * 8 +
           (size_t)kMfmaWaves * (NW * 16 * kBlk + kBlk) * 4;
}

hipError_t launch_mfma_frags(const float *G, void *frag, const Shape &s, int n,
                             hipStream_t st) {
    FragArgs f;
    f.N = s.N;
    f.n = n;
    f.J = s.ranks[n];
    for (int k = 0; k < s.N; ++k) f.rk[k] = s.ranks[k];
    f.tiles = mfma_tiles(s.N, f.J);
    const int64_t total = f.tiles * kWave * 4;
    hipLaunchKernelGGL(k_mfma_frags, dim3((unsigned)((total + 255) / 256)), dim3(256),
                       0, st, G, (__bf16 *)frag, f);
    return hipGetLastError();
}

int mfma_waves_per_cu(int N, int J, int split) {
    const size_t lds = mfma_lds_bytes(N, J, split);
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
#define PTK_X(n_, j_)                                                                   \
    if (N == n_ && J == j_)                                                             \
        e = split == 3 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(                  \
                             &nb, k_gram_mfma<n_, j_, 3>, kWave * kMfmaWaves, lds)      \
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(                  \
                             &nb, k_gram_mfma<n_, j_, 1>, kWave * kMfmaWaves, lds);
    PTK_MFMA_SHAPES(PTK_X)
#undef PTK_X
    if (e != hipSuccess || nb < 1) nb = 1;
    return nb * kMfmaWaves;
}

hipError_t launch_gram_mfma(const MfmaArgs &a, int N, int J, int split, int64_t nwaves,
                            hipStream_t st) {
    if (nwaves <= 0 || a.nblk <= 0) return hipSuccess;
    const unsigned grid = (unsigned)((nwaves + kMfmaWaves - 1) / kMfmaWaves);
    const size_t lds = mfma_lds_bytes(N, J, split);
#define PTK_X(n_, j_)                                                                   \
    if (N == n_ && J == j_) {                                                           \
        if (split == 3)                                                                 \
            hipLaunchKernelGGL((k_gram_mfma<n_, j_, 3>), dim3(grid),                     \
                               dim3(kWave * kMfmaWaves), lds, st, a);                  \
        else                                                                            \
            hipLaunchKernelGGL((k_gram_mfma<n_, j_, 1>), dim3(grid),                     \
                               dim3(kWave * kMfmaWaves), lds, st, a);                  \
        return hipGetLastError();                                                       \
    }
    PTK_MFMA_SHAPES(PTK_X)
#undef PTK_X
    return hipErrorInvalidValue;
}

}  // namespace ptk
