// Mode-n grouping of the observed entries (the sets Omega^(n)_i of Table 2,
// which Alg. 3 visits row by row).
//
// The entries are ordered by their mode-n index with a stable least-
// significant-digit radix sort (8-bit digits): per pass, every tile of 4096
// entries counts its digits, one exclusive scan over (digit, tile) gives each
// tile's output offsets, and each tile scatters its entries in input order,
// ranking equal digits inside a wavefront with ballots. Stability makes the
// order inside a row, and hence every later floating-point sum, independent of
// the launch. The other modes' indices and the values are then gathered into
// the grouped order and the row pointers are read off the sorted keys.
#include <algorithm>

#include "ptk_internal.h"

namespace ptk {

constexpr int kRsThreads = 256;
constexpr int kRsItems = 16;
constexpr int kRsTile = kRsThreads * kRsItems;   // 4096
constexpr int kRsDigits = 256;
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;  // 2048

// --------------------------------------------------------------------------
// exclusive scan of int32 (counts < 2^31)
// --------------------------------------------------------------------------
__device__ __forceinline__ int32_t wave_incl_scan(int32_t v) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int32_t t = __shfl_up(v, off, kWave);
        if (lane >= off) v += t;
    }
    return v;
}

// Exclusive scan of v over the block (kScanThreads threads); *total receives
// the block sum.
__device__ __forceinline__ int32_t block_excl_scan(int32_t v, int32_t *s_w,
                                                   int32_t *total) {
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    const int32_t incl = wave_incl_scan(v);
    if (lane == kWave - 1) s_w[w] = incl;
    __syncthreads();
    int32_t off = 0, tot = 0;
    for (int k = 0; k < kScanThreads / kWave; ++k) {
        if (k < w) off += s_w[k];
        tot += s_w[k];
    }
    __syncthreads();
    *total = tot;
    return off + incl - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(
    const int32_t *__restrict__ in, int64_t n, int32_t *__restrict__ bsum) {
    __shared__ int32_t s_w[kScanThreads / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int32_t v = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) v += in[base + k];
    int32_t tot;
    block_excl_scan(v, s_w, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_down(
    const int32_t *in, int32_t *out, int64_t n, const int32_t *__restrict__ boff) {
    __shared__ int32_t s_w[kScanThreads / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int32_t x[kScanItems];
    int32_t v = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        x[k] = (base + k < n) ? in[base + k] : 0;
        v += x[k];
    }
    int32_t tot;
    int32_t run = block_excl_scan(v, s_w, &tot) + (boff ? boff[blockIdx.x] : 0);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = run;
        run += x[k];
    }
}

static int64_t scan_work_elems(int64_t n) {
    int64_t w = 0;
    while (n > kScanTile) {
        n = (n + kScanTile - 1) / kScanTile;
        w += n;
    }
    return w + 1;
}

// out may alias in.
static hipError_t scan_exclusive(const int32_t *in, int32_t *out, int64_t n,
                                 int32_t *work, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 1) {
        hipLaunchKernelGGL(k_scan_down, dim3(1), dim3(kScanThreads), 0, st, in,
                           out, n, (const int32_t *)nullptr);
        return hipGetLastError();
    }
    int32_t *bsum = work;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0,
                       st, in, n, bsum);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = scan_exclusive(bsum, bsum, nb, work + nb, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kScanThreads), 0, st,
                       in, out, n, (const int32_t *)bsum);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// radix sort passes
// --------------------------------------------------------------------------
__global__ __launch_bounds__(kRsThreads) void k_radix_hist(
    const int32_t *__restrict__ keys, int64_t n, int shift,
    int32_t *__restrict__ hist, int64_t ntiles) {
    __shared__ int32_t h[kRsDigits];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
#pragma unroll
    for (int k = 0; k < kRsItems; ++k) {
        const int64_t pos = base + k * kRsThreads + threadIdx.x;
        if (pos < n) atomicAdd(&h[(keys[pos] >> shift) & (kRsDigits - 1)], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kRsThreads) void k_radix_scatter(
    const int32_t *__restrict__ kin, const int32_t *__restrict__ vin,
    int32_t *__restrict__ kout, int32_t *__restrict__ vout, int64_t n, int shift,
    const int32_t *__restrict__ offs, int64_t ntiles) {
    constexpr int kWaves = kRsThreads / kWave;
    __shared__ int32_t s_base[kRsDigits];
    __shared__ int32_t s_cnt[kWaves][kRsDigits];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int w = tid / kWave;
    s_base[tid] = offs[(int64_t)tid * ntiles + blockIdx.x];
#pragma unroll
    for (int k = 0; k < kWaves; ++k) s_cnt[k][tid] = 0;
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
    for (int k = 0; k < kRsItems; ++k) {
        const int64_t pos = base + k * kRsThreads + tid;
        const bool valid = pos < n;
        const int32_t key = valid ? kin[pos] : 0;
        const int dig = (key >> shift) & (kRsDigits - 1);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (dig >> b) & 1;
            const uint64_t m = __ballot(valid && bit);
            peers &= bit ? m : ~m;
        }
        const int wrank = __popcll(peers & lt);
        if (valid && wrank == 0) s_cnt[w][dig] = __popcll(peers);
        __syncthreads();
        if (valid) {
            int32_t r = s_base[dig] + wrank;
            for (int q = 0; q < w; ++q) r += s_cnt[q][dig];
            kout[r] = key;
            vout[r] = vin ? vin[pos] : (int32_t)pos;
        }
        __syncthreads();
        int32_t add = 0;
#pragma unroll
        for (int q = 0; q < kWaves; ++q) {
            add += s_cnt[q][tid];
            s_cnt[q][tid] = 0;
        }
        s_base[tid] += add;
        __syncthreads();
    }
}

// --------------------------------------------------------------------------
// gather into grouped order; row pointers from the sorted keys
// --------------------------------------------------------------------------
struct GatherArgs {
    const int32_t *idx;
    const float *val;
    const int32_t *perm;
    int32_t *oidx;     // [N-1][nnz]
    float *vals;
    int64_t nnz;
    int32_t N, n;
};

__global__ void k_gather(GatherArgs g) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < g.nnz;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = g.perm[p];
        int t = 0;
        for (int k = 0; k < g.N; ++k) {
            if (k == g.n) continue;
            g.oidx[(int64_t)t * g.nnz + p] = g.idx[(int64_t)k * g.nnz + e];
            ++t;
        }
        g.vals[p] = g.val[e];
    }
}

// rowptr[r] = number of sorted keys below r, for r = 0..I: one thread per
// row, a binary search over the keys (balanced however the rows are spread;
// a huge mode with few entries is as fast as a dense one).
__global__ void k_rowptr(const int32_t *__restrict__ keys, int64_t nnz, int64_t I,
                         int64_t *__restrict__ rowptr) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r > I) return;
    int64_t lo = 0, hi = nnz;                 // first position with key >= r
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if ((int64_t)keys[mid] < r)
            lo = mid + 1;
        else
            hi = mid;
    }
    rowptr[r] = lo;
}

static int64_t n_tiles(int64_t nnz) { return (nnz + kRsTile - 1) / kRsTile; }

size_t sort_workspace_bytes(int64_t nnz) {
    const int64_t nt = n_tiles(nnz > 0 ? nnz : 1);
    const int64_t hist = nt * kRsDigits;
    size_t b = 0;
    b += 4 * (size_t)(nnz + 64) * 4;              // keys A/B, vals A/B
    b += (size_t)(hist + 64) * 4;                 // histogram / offsets
    b += (size_t)(scan_work_elems(hist) + 64) * 4;
    return b;
}

__global__ void k_gather_keys(const int32_t *__restrict__ src,
                              const int32_t *__restrict__ perm, int32_t *__restrict__ dst,
                              int64_t nnz) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz;
         p += (int64_t)gridDim.x * blockDim.x)
        dst[p] = src[perm[p]];
}

hipError_t build_mode_csr(const int32_t *idx, const float *val, int64_t nnz,
                          const Shape &s, int n, void *work, int64_t *rowptr,
                          int32_t *rows, int32_t *oidx, float *vals,
                          hipStream_t st, int32_t *perm_out, int sub) {
    const int64_t I = s.dims[n];
    if (nnz == 0) {
        hipLaunchKernelGGL(k_rowptr, dim3((unsigned)((I + 1 + 255) / 256)), dim3(256), 0, st,
                           rows, (int64_t)0, I, rowptr);
        return hipGetLastError();
    }
    const int64_t nt = n_tiles(nnz);
    const int64_t hist_n = nt * kRsDigits;
    int32_t *keyA = (int32_t *)work;
    int32_t *keyB = keyA + nnz + 64;
    int32_t *valA = keyB + nnz + 64;
    int32_t *valB = valA + nnz + 64;
    int32_t *hist = valB + nnz + 64;
    int32_t *swork = hist + hist_n + 64;

    const int32_t *kin = idx + (int64_t)(sub >= 0 ? sub : n) * nnz;
    const int32_t *vin = nullptr;
    int32_t *kout = keyA, *vout = valA;
    hipError_t e = hipSuccess;
    // stable passes over the 8-bit digits of keys below `extent`
    auto passes = [&](int64_t extent) -> hipError_t {
        int bits = 0;
        while ((int64_t(1) << bits) < extent) ++bits;
        const int np = bits <= 8 ? 1 : (bits + 7) / 8;
        for (int p = 0; p < np; ++p) {
            const int shift = 8 * p;
            hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nt), dim3(kRsThreads), 0, st,
                               kin, nnz, shift, hist, nt);
            hipError_t r = hipGetLastError();
            if (r != hipSuccess) return r;
            if ((r = scan_exclusive(hist, hist, hist_n, swork, st)) != hipSuccess) return r;
            hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nt), dim3(kRsThreads), 0,
                               st, kin, vin, kout, vout, nnz, shift, hist, nt);
            if ((r = hipGetLastError()) != hipSuccess) return r;
            kin = kout;
            vin = vout;
            kout = (kout == keyA) ? keyB : keyA;
            vout = (vout == valA) ? valB : valA;
        }
        return hipSuccess;
    };
    if (sub >= 0) {
        // order by the index of mode `sub` first; the stable passes over the
        // mode-n index below keep that order inside every row
        if ((e = passes(s.dims[sub])) != hipSuccess) return e;
        unsigned gb = (unsigned)std::min<int64_t>((nnz + 255) / 256, 65536);
        hipLaunchKernelGGL(k_gather_keys, dim3(gb), dim3(256), 0, st,
                           idx + (int64_t)n * nnz, vin, kout, nnz);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        kin = kout;
        kout = (kout == keyA) ? keyB : keyA;
    }
    if ((e = passes(I)) != hipSuccess) return e;
    // kin / vin hold the sorted keys and the permutation
    if ((e = hipMemcpyAsync(rows, kin, nnz * 4, hipMemcpyDeviceToDevice, st)) !=
        hipSuccess)
        return e;
    if (perm_out &&
        (e = hipMemcpyAsync(perm_out, vin, nnz * 4, hipMemcpyDeviceToDevice, st)) !=
            hipSuccess)
        return e;
    GatherArgs g;
    g.idx = idx;
    g.val = val;
    g.perm = vin;
    g.oidx = oidx;
    g.vals = vals;
    g.nnz = nnz;
    g.N = s.N;
    g.n = n;
    int64_t blocks = (nnz + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)blocks), dim3(256), 0, st, g);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rowptr, dim3((unsigned)((I + 1 + 255) / 256)), dim3(256), 0, st,
                       rows, nnz, I, rowptr);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// unit lists of the shared-index row systems
// ---------------------------------------------------------------------------
// rows may be null: runs of equal sidx only.
__device__ __forceinline__ int32_t run_flag(const int32_t *rows, const int32_t *sidx,
                                            int64_t p) {
    return p == 0 || (rows && rows[p] != rows[p - 1]) || sidx[p] != sidx[p - 1];
}

__global__ void k_run_flags(const int32_t *__restrict__ rows, const int32_t *__restrict__ sidx,
                            int64_t nnz, int32_t *__restrict__ flag) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz;
         p += (int64_t)gridDim.x * blockDim.x)
        flag[p] = run_flag(rows, sidx, p);
}

// start[r] = first position of run r; start[R] = nnz; *nruns = R.
__global__ void k_run_starts(const int32_t *__restrict__ rows, const int32_t *__restrict__ sidx,
                             int64_t nnz, const int32_t *__restrict__ rid,
                             int32_t *__restrict__ start, int32_t *__restrict__ nruns) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t f = run_flag(rows, sidx, p);
        if (f) start[rid[p]] = (int32_t)p;
        if (p == nnz - 1) {
            start[rid[p] + f] = (int32_t)nnz;
            *nruns = rid[p] + f;
        }
    }
}

// Counters of a run of len entries: q = 0..3, units of 2^q entries (none
// above cmax); q = 4, one long run, and q = 5, its tasks of at most tlen
// entries; or, for a long run of fewer than wmin entries, q = 6, one per
// entry (and no q = 4 or 5). A run of at least lmin entries (lmin > 0) is
// long and has no units.
__device__ __forceinline__ int32_t run_count(int32_t len, int q, int cmax, int32_t lmin,
                                             int32_t tlen, int32_t wmin) {
    const bool lng = lmin > 0 && len >= lmin;
    const bool narrow = len < wmin;
    if (q == 4) return (lng && !narrow) ? 1 : 0;
    if (q == 5) return (lng && !narrow) ? (len + tlen - 1) / tlen : 0;
    if (q == 6) return (lng && narrow) ? len : 0;
    if (lng || q > cmax) return 0;
    return q == cmax ? (len >> cmax) : ((len >> q) & 1);
}

constexpr int kRunCounters = 7;

__global__ void k_unit_counts(const int32_t *__restrict__ start, int32_t R, int cmax,
                              int32_t lmin, int32_t tlen, int32_t wmin,
                              int32_t *__restrict__ cnt) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < R;
         r += (int64_t)gridDim.x * blockDim.x) {
        const int32_t len = start[r + 1] - start[r];
        for (int q = 0; q < kRunCounters; ++q)
            cnt[(int64_t)q * R + r] = run_count(len, q, cmax, lmin, tlen, wmin);
    }
}

// total[q] = off[q][R-1] + the last run's counter q
__global__ void k_unit_totals(const int32_t *__restrict__ start, int32_t R, int cmax,
                              int32_t lmin, int32_t tlen, int32_t wmin,
                              const int32_t *__restrict__ off, int64_t *__restrict__ total) {
    const int q = threadIdx.x;
    if (q >= kRunCounters) return;
    const int32_t len = start[R] - start[R - 1];
    total[q] =
        (int64_t)off[(int64_t)q * R + R - 1] + run_count(len, q, cmax, lmin, tlen, wmin);
}

__global__ void k_unit_write(const int32_t *__restrict__ start, int32_t R, int cmax,
                             int32_t lmin, int32_t tlen, int32_t wmin,
                             const int32_t *__restrict__ off, const int64_t *__restrict__ base,
                             int32_t *__restrict__ units, UnitLong lg) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < R;
         r += (int64_t)gridDim.x * blockDim.x) {
        int32_t p = start[r];
        const int32_t len = start[r + 1] - p;
        if (run_count(len, 6, cmax, lmin, tlen, wmin)) {       // its entries, one by one
            int32_t *tp = lg.ntask_pos + off[6 * (int64_t)R + r];
            for (int32_t q = 0; q < len; ++q) tp[q] = p + q;
            continue;
        }
        if (run_count(len, 4, cmax, lmin, tlen, wmin)) {
            const int32_t li = off[4 * (int64_t)R + r];
            lg.run_pos[li] = p;
            const int32_t nt = run_count(len, 5, cmax, lmin, tlen, wmin);
            const int64_t o = off[5 * (int64_t)R + r];
            for (int32_t q = 0; q < nt; ++q) {
                lg.task_pos[o + q] = p + q * tlen;
                lg.task_len[o + q] = min(tlen, len - q * tlen);
                lg.task_run[o + q] = li;
            }
            continue;
        }
        for (int c = cmax; c >= 0; --c) {
            const int32_t k = run_count(len, c, cmax, lmin, tlen, wmin);
            int32_t *dst = units + base[c] + off[(int64_t)c * R + r];
            for (int32_t q = 0; q < k; ++q) {
                dst[q] = p;
                p += 1 << c;
            }
        }
    }
}

hipError_t sort_by_key(const int32_t *keys, int64_t nnz, int64_t extent, void *work,
                       int32_t *keys_out, int32_t *pos_out, hipStream_t st) {
    if (nnz <= 0) return hipSuccess;
    const int64_t nt = n_tiles(nnz);
    const int64_t hist_n = nt * kRsDigits;
    int32_t *keyA = (int32_t *)work;
    int32_t *keyB = keyA + nnz + 64;
    int32_t *valA = keyB + nnz + 64;
    int32_t *valB = valA + nnz + 64;
    int32_t *hist = valB + nnz + 64;
    int32_t *swork = hist + hist_n + 64;
    const int32_t *kin = keys;
    const int32_t *vin = nullptr;
    int32_t *kout = keyA, *vout = valA;
    int bits = 0;
    while ((int64_t(1) << bits) < extent) ++bits;
    const int np = bits <= 8 ? 1 : (bits + 7) / 8;
    hipError_t e = hipSuccess;
    for (int q = 0; q < np; ++q) {
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nt), dim3(kRsThreads), 0, st, kin, nnz,
                           8 * q, hist, nt);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = scan_exclusive(hist, hist, hist_n, swork, st)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nt), dim3(kRsThreads), 0, st, kin,
                           vin, kout, vout, nnz, 8 * q, hist, nt);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        kin = kout;
        vin = vout;
        kout = (kout == keyA) ? keyB : keyA;
        vout = (vout == valA) ? valB : valA;
    }
    if ((e = hipMemcpyAsync(keys_out, kin, nnz * 4, hipMemcpyDeviceToDevice, st)) != hipSuccess)
        return e;
    return hipMemcpyAsync(pos_out, vin, nnz * 4, hipMemcpyDeviceToDevice, st);
}

// run_pos[r] <- keys[run_pos[r]]: each run names its key value.
__global__ void k_run_keys(const int32_t *__restrict__ keys, int32_t *__restrict__ run_pos,
                           int64_t n) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x)
        run_pos[r] = keys[run_pos[r]];
}

hipError_t launch_run_keys(const int32_t *keys, const UnitLong &lg, hipStream_t st) {
    if (lg.n_long <= 0) return hipSuccess;
    const unsigned b = (unsigned)std::min<int64_t>((lg.n_long + 255) / 256, 65536);
    hipLaunchKernelGGL(k_run_keys, dim3(b), dim3(256), 0, st, keys, lg.run_pos, lg.n_long);
    return hipGetLastError();
}

// list[i] <- perm[list[i]]
__global__ void k_permute_list(const int32_t *__restrict__ perm, int32_t *__restrict__ list,
                               int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        list[i] = perm[list[i]];
}

hipError_t launch_permute_list(const int32_t *perm, int32_t *list, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const unsigned b = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_permute_list, dim3(b), dim3(256), 0, st, perm, list, n);
    return hipGetLastError();
}

int64_t units_workspace_ints(int64_t nnz) {
    // run ids, run starts, the counters of every run, the run count, totals
    // and bases, scan work
    return 2 * (nnz + 64) + kRunCounters * (nnz + 64) + 64 + scan_work_elems(nnz) + 64;
}

hipError_t build_units(const int32_t *rows, const int32_t *sidx, int64_t nnz, int emax,
                       int32_t lmin, int32_t tlen, int32_t wmin, int32_t *work, int32_t *units,
                       int64_t *count, UnitLong *lg, hipStream_t st) {
    int cmax = 0;
    while ((1 << cmax) < emax) ++cmax;
    if (cmax > 3 || (1 << cmax) != emax || tlen <= 0) return hipErrorInvalidValue;
    for (int c = 0; c <= 3; ++c) count[c] = 0;
    lg->n_long = lg->n_tasks = lg->n_ntasks = 0;
    if (wmin > 0 && (tlen < 2 || !lg->ntask_pos)) return hipErrorInvalidValue;
    if (nnz == 0) return hipSuccess;
    int32_t *rid = work;
    int32_t *start = rid + nnz + 64;
    int32_t *cnt = start + nnz + 64;
    int32_t *misc = cnt + kRunCounters * (nnz + 64);   // [0]: R; [2..]: totals, bases
    int32_t *swork = misc + 64;
    int64_t *total = (int64_t *)(misc + 2);
    int64_t *base = total + kRunCounters;
    const unsigned gb = (unsigned)std::min<int64_t>((nnz + 255) / 256, 65536);
    hipLaunchKernelGGL(k_run_flags, dim3(gb), dim3(256), 0, st, rows, sidx, nnz, rid);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = scan_exclusive(rid, rid, nnz, swork, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_run_starts, dim3(gb), dim3(256), 0, st, rows, sidx, nnz, rid, start,
                       misc);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    int32_t R = 0;
    if ((e = hipMemcpyAsync(&R, misc, 4, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    if (R <= 0 || R > nnz) return hipErrorInvalidValue;
    const unsigned rb = (unsigned)std::min<int64_t>((R + 255) / 256, 65536);
    hipLaunchKernelGGL(k_unit_counts, dim3(rb), dim3(256), 0, st, start, R, cmax, lmin, tlen,
                       wmin, cnt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    for (int q = 0; q < kRunCounters; ++q)
        if ((e = scan_exclusive(cnt + (int64_t)q * R, cnt + (int64_t)q * R, R, swork, st)) !=
            hipSuccess)
            return e;
    hipLaunchKernelGGL(k_unit_totals, dim3(1), dim3(64), 0, st, start, R, cmax, lmin, tlen,
                       wmin, cnt, total);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    int64_t ht[kRunCounters] = {};
    if ((e = hipMemcpyAsync(ht, total, 8 * kRunCounters, hipMemcpyDeviceToHost, st)) !=
        hipSuccess)
        return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    // classes in the order cmax, ..., 0
    int64_t hb[4] = {0, 0, 0, 0}, at = 0;
    for (int c = cmax; c >= 0; --c) {
        hb[c] = at;
        at += ht[c];
        count[c] = ht[c];
    }
    if (at > nnz || ht[4] > lg->cap_long || ht[5] > lg->cap_tasks || ht[6] > lg->cap_ntasks)
        return hipErrorInvalidValue;
    lg->n_long = ht[4];
    lg->n_tasks = ht[5];
    lg->n_ntasks = ht[6];
    if ((e = hipMemcpyAsync(base, hb, 8 * 4, hipMemcpyHostToDevice, st)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_unit_write, dim3(rb), dim3(256), 0, st, start, R, cmax, lmin, tlen,
                       wmin, cnt, base, units, *lg);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return hipStreamSynchronize(st);   // hb lives on this stack frame
}

// ---------------------------------------------------------------------------
// permutation helpers (position maps between the groupings of two modes)
// ---------------------------------------------------------------------------
__global__ void k_invert_perm(const int32_t *__restrict__ perm, int64_t nnz,
                              int32_t *__restrict__ inv) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nnz; i += stride)
        inv[perm[i]] = (int32_t)i;
}

__global__ void k_compose_perm(const int32_t *__restrict__ inv,
                               const int32_t *__restrict__ perm, int64_t nnz,
                               int32_t *__restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nnz; i += stride)
        out[i] = inv[perm[i]];
}

static unsigned perm_blocks(int64_t nnz) {
    int64_t b = (nnz + 255) / 256;
    return (unsigned)(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

hipError_t launch_invert_perm(const int32_t *perm, int64_t nnz, int32_t *inv,
                              hipStream_t st) {
    if (nnz <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_invert_perm, dim3(perm_blocks(nnz)), dim3(256), 0, st, perm,
                       nnz, inv);
    return hipGetLastError();
}

hipError_t launch_compose_perm(const int32_t *inv, const int32_t *perm, int64_t nnz,
                               int32_t *out, hipStream_t st) {
    if (nnz <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_compose_perm, dim3(perm_blocks(nnz)), dim3(256), 0, st, inv,
                       perm, nnz, out);
    return hipGetLastError();
}

}  // namespace ptk
