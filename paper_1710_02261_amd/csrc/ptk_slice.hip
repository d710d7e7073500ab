// Core-sliced row systems (see ptk_slice.h): the delta sum of Eq. 8 split
// over slices of the other modes' cells, one wavefront per (tile, slice).
#include "ptk_device.h"
#include "ptk_slice.h"

namespace ptk {

namespace {

constexpr int kOther = kMaxN - 1;
constexpr int kMinSliceCells = 16;

// Slices blockIdx.y * W .. + W - 1 (one per wavefront) of the 64 entries of
// tile blockIdx.x. Cells are walked in the permuted core's order (last other
// mode fastest); a slice's first cell fixes the starting digits. The W sums
// are added in wavefront order into one partial group.
template <int JMAX>
__global__ __launch_bounds__(1024) void k_delta_slices(SliceArgs sa) {
    extern __shared__ __attribute__((aligned(16))) unsigned char s_dyn[];
    const GramArgs &a = sa.g;
    const int no = a.nother;
    const int jn = a.jn;
    const int W = sa.W;
    int sumj = 0;
    for (int k = 0; k < no; ++k) sumj += a.jk[k];
    float *s_arow = (float *)s_dyn;
    double *s_red = (double *)(s_dyn + ((sumj * kWave * 4 + 15) / 16) * 16);
    const int lane = threadIdx.x % kWave;
    const int w = threadIdx.x / kWave;
    const int64_t tile0 = (int64_t)blockIdx.x * kWave;
    const int64_t pos = tile0 + lane;
    const bool valid = pos < a.nnz;
    // the tile's rows of the other modes, shared by the W wavefronts
    for (int k = w; k < no; k += W) {
        const int32_t i = valid ? a.oidx[k][pos] : 0;
        const int jk = a.jk[k];
        const float *r = a.fac[k] + (int64_t)i * jk;
        for (int j = 0; j < jk; ++j) s_arow[(a.aoff[k] + j) * kWave + lane] = r[j];
    }
    __syncthreads();
    const int s = blockIdx.y * W + w;
    int jk[kOther], off[kOther], dig[kOther];
    int64_t P = 1;
#pragma unroll
    for (int k = 0; k < kOther; ++k) {
        jk[k] = (k < no) ? a.jk[k] : 1;
        off[k] = (k < no) ? a.aoff[k] : 0;
        P *= jk[k];
    }
    int64_t lo, hi;
    if (sa.writer) {
        const int64_t Q = P / jk[0];
        const int mp = s / sa.sub, ss = s % sa.sub;
        lo = mp * Q + Q * ss / sa.sub;
        hi = mp * Q + Q * (ss + 1) / sa.sub;
    } else {
        lo = P * s / sa.S;
        hi = P * (s + 1) / sa.S;
    }
    {
        int64_t t = lo;
#pragma unroll
        for (int k = kOther - 1; k >= 0; --k) {
            dig[k] = (int)(t % jk[k]);
            t /= jk[k];
        }
    }
    // the writer leaves out the partner's weight (slot 0)
    const int kfirst = sa.writer ? 1 : 0;
    double acc[JMAX];
#pragma unroll
    for (int j = 0; j < JMAX; ++j) acc[j] = 0.0;
    cptr<double> g = (cptr<double>)a.gp + lo * jn;
    for (int64_t o = lo; o < hi; ++o, g += jn) {
        double wt = 1.0;
#pragma unroll
        for (int k = 0; k < kOther; ++k)
            if (k < no && k >= kfirst) wt *= (double)s_arow[(off[k] + dig[k]) * kWave + lane];
#pragma unroll
        for (int j = 0; j < JMAX; ++j)
            if (j < jn) acc[j] = __builtin_fma(g[j], wt, acc[j]);
        bool carry = true;
#pragma unroll
        for (int k = kOther - 1; k >= 0; --k) {
            if (carry && k < no) {
                if (++dig[k] == jk[k])
                    dig[k] = 0;
                else
                    carry = false;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < JMAX; ++j)
        if (j < jn) s_red[(w * jn + j) * kWave + lane] = acc[j];
    __syncthreads();
    const int64_t grp = blockIdx.y;
    for (int t = threadIdx.x; t < jn * kWave; t += blockDim.x) {
        const int j = t / kWave, l = t % kWave;
        double v = s_red[j * kWave + l];
        for (int u = 1; u < W; ++u) v += s_red[(u * jn + j) * kWave + l];
        if (tile0 + l < a.nnz) sa.dpart[(grp * jn + j) * sa.nnzp + tile0 + l] = v;
    }
}

// Row systems from the partial groups: delta = the groups summed in order
// (writer: per partner index, stored as the entry's record, then weighted by
// the partner's row), then the tile sweep of the other kernels.
template <int JMAX>
__global__ __launch_bounds__(kWave) void k_gram_slices(SliceArgs sa) {
    constexpr int EPL = (sys_entries(JMAX) + kWave - 1) / kWave;
    __shared__ double s_dl[(JMAX + 1) * kDlStride];
    __shared__ int s_row[kWave];
    const GramArgs &a = sa.g;
    const int lane = threadIdx.x;
    const int J = a.jn;
    const int RS = (J * J + 1) / 2 * 2;
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
        double d[JMAX];
#pragma unroll
        for (int j = 0; j < JMAX; ++j) d[j] = 0.0;
        if (valid) {
            const double *dp = sa.dpart + pos;
            if (!sa.writer) {
                const int G = sa.S / sa.W;
#pragma unroll 4
                for (int q = 0; q < G; ++q) {
#pragma unroll
                    for (int j = 0; j < JMAX; ++j)
                        if (j < J) d[j] += dp[((int64_t)q * J + j) * sa.nnzp];
                }
            } else {
                const int gsub = sa.sub / sa.W;
                const int jp = a.jk[0];
                const float *ap = a.fac[0] + (int64_t)a.oidx[0][pos] * jp;
                double *rec = a.cache + pos * RS;
                for (int mp = 0; mp < jp; ++mp) {
                    double t[JMAX];
#pragma unroll
                    for (int j = 0; j < JMAX; ++j) t[j] = 0.0;
#pragma unroll 4
                    for (int qs = 0; qs < gsub; ++qs) {
                        const int q = mp * gsub + qs;
#pragma unroll
                        for (int j = 0; j < JMAX; ++j)
                            if (j < J) t[j] += dp[((int64_t)q * J + j) * sa.nnzp];
                    }
                    const double wp = (double)ap[mp];
#pragma unroll
                    for (int j = 0; j < JMAX; ++j) {
                        if (j < J) {
                            rec[mp * J + j] = t[j];
                            d[j] = __builtin_fma(wp, t[j], d[j]);
                        }
                    }
                }
            }
        }
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

int slice_jmax(int J) { return J <= 4 ? 4 : J <= 8 ? 8 : J <= 16 ? 16 : 32; }

}  // namespace

static size_t delta_slices_lds(const GramArgs &g, int W) {
    int sumj = 0;
    for (int k = 0; k < g.nother; ++k) sumj += g.jk[k];
    return ((size_t)sumj * kWave * 4 + 15) / 16 * 16 + (size_t)W * g.jn * kWave * 8;
}

SlicePlan slice_plan(const Shape &s, int n, int partner, int64_t nnz, int num_cu,
                     int32_t want) {
    SlicePlan p;
    if (nnz <= 0 || want == 1 || s.ranks[n] > kMaxJ) return p;
    int64_t P = 1;
    for (int k = 0; k < s.N; ++k)
        if (k != n) P *= s.ranks[k];
    const int64_t jp = partner >= 0 ? s.ranks[partner] : 1;
    const int64_t Q = P / jp;                   // cells per partner index
    int64_t sub;                                // slices per partner index
    if (want == 0) {
        const int64_t tiles = (nnz + kWave - 1) / kWave;
        const int64_t target = (int64_t)num_cu * 32;   // eight wavefronts per SIMD
        if (tiles * 2 > target) return p;
        const int64_t total = (target + tiles - 1) / tiles;
        sub = std::min((total + jp - 1) / jp, Q / kMinSliceCells);
        if (sub >= 16) sub = sub / 16 * 16;
        if (partner < 0 && sub < 2) return p;
        sub = std::max<int64_t>(1, sub);
    } else {
        sub = std::max<int64_t>(1, std::min<int64_t>((want + jp - 1) / jp, Q));
    }
    sub = std::min<int64_t>(sub, 65535 / jp);
    p.sub = (int32_t)sub;
    p.S = (int32_t)(jp * sub);
    GramArgs g{};
    g.nother = s.N - 1;
    g.jn = s.ranks[n];
    for (int k = 0, t = 0; k < s.N; ++k)
        if (k != n) g.jk[t++] = s.ranks[k];
    int W = 16;
    while (W > 1 && (sub % W != 0 || delta_slices_lds(g, W) > 65536)) W /= 2;
    p.W = W;
    return p;
}

int64_t slice_part_doubles(int J, int64_t nnz, const SlicePlan &p) {
    return (int64_t)(p.S / p.W) * J * ((nnz + kWave - 1) / kWave * kWave);
}

hipError_t launch_delta_slices(const SliceArgs &a, hipStream_t st) {
    if (a.g.nnz <= 0) return hipSuccess;
    const int W = a.W;
    if (a.S < 1 || a.S > 65535 || a.g.jn > kMaxJ || W < 1 || W > 16 || (W & (W - 1)) ||
        a.sub % W != 0 || a.S % W != 0 || (a.writer && a.S != a.g.jk[0] * a.sub))
        return hipErrorInvalidValue;
    const size_t lds = delta_slices_lds(a.g, W);
    if (lds > 65536) return hipErrorInvalidValue;
    dim3 grid((unsigned)((a.g.nnz + kWave - 1) / kWave), (unsigned)(a.S / W)),
        block(kWave * W);
    switch (slice_jmax(a.g.jn)) {
        case 4: hipLaunchKernelGGL(k_delta_slices<4>, grid, block, lds, st, a); break;
        case 8: hipLaunchKernelGGL(k_delta_slices<8>, grid, block, lds, st, a); break;
        case 16: hipLaunchKernelGGL(k_delta_slices<16>, grid, block, lds, st, a); break;
        default: hipLaunchKernelGGL(k_delta_slices<32>, grid, block, lds, st, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_gram_slices(const SliceArgs &a, int64_t nchunks, hipStream_t st) {
    if (nchunks <= 0) return hipSuccess;
    dim3 grid((unsigned)nchunks), block(kWave);
    switch (slice_jmax(a.g.jn)) {
        case 4: hipLaunchKernelGGL(k_gram_slices<4>, grid, block, 0, st, a); break;
        case 8: hipLaunchKernelGGL(k_gram_slices<8>, grid, block, 0, st, a); break;
        case 16: hipLaunchKernelGGL(k_gram_slices<16>, grid, block, 0, st, a); break;
        default: hipLaunchKernelGGL(k_gram_slices<32>, grid, block, 0, st, a); break;
    }
    return hipGetLastError();
}

int gram_slices_blocks_per_cu(int J) {
    switch (slice_jmax(J)) {
        case 4: return blocks_per_cu(k_gram_slices<4>, 0);
        case 8: return blocks_per_cu(k_gram_slices<8>, 0);
        case 16: return blocks_per_cu(k_gram_slices<16>, 0);
        default: return blocks_per_cu(k_gram_slices<32>, 0);
    }
}

}  // namespace ptk
