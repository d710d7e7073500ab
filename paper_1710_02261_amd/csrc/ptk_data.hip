// Steps either side of the factorisation (Sec. 4.1 and Sec. 5):
//  * reading an observed set from a COO text file (N 1-based indices and a
//    value per line), parsed by host threads;
//  * min-max normalisation of the values to [0, 1];
//  * a seeded train/test split of the entries (90/10 in the paper) with a
//    counter-based generator, and the error of the bound model over a
//    held-out entry list (test RMSE);
//  * k-means (Lloyd's iterations) over the rows of a factor matrix, the
//    concept-discovery step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <charconv>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "ptk_context.h"
#include "ptk_internal.h"

using namespace ptk;

namespace {

thread_local std::string g_err = "no error";

ptk_status gfail(ptk_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

ptk_status cfail(ptk_ctx *c, ptk_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
    return s;
}

#define DCHK(c, expr)                                                              \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess)                                                      \
            return cfail(c, e_ == hipErrorOutOfMemory ? PTK_E_NOMEM : PTK_E_HIP,  \
                         "%s: %s", #expr, hipGetErrorString(e_));                  \
    } while (0)

// ---------------------------------------------------------------------------
// COO text
// ---------------------------------------------------------------------------
bool read_file(const char *path, std::vector<char> &buf) {
    FILE *f = fopen(path, "rb");
    if (!f) return false;
    buf.clear();
    char tmp[1 << 16];
    size_t got;
    while ((got = fread(tmp, 1, sizeof tmp, f)) > 0) buf.insert(buf.end(), tmp, tmp + got);
    const bool ok = !ferror(f);
    fclose(f);
    return ok;
}

inline bool is_space(char ch) { return ch == ' ' || ch == '\t' || ch == '\r'; }

// A line is an entry when it holds any non-blank character.
inline bool blank(const char *p, const char *e) {
    for (; p < e; ++p)
        if (!is_space(*p)) return false;
    return true;
}

// Parse one entry line: N integers >= 1 (returned 0-based) and a finite
// value; nothing else but blanks.
bool parse_entry(const char *p, const char *e, int N, int64_t *ids, float *v) {
    for (int k = 0; k <= N; ++k) {
        while (p < e && is_space(*p)) ++p;
        if (p == e) return false;
        const char *q = p;
        while (q < e && !is_space(*q)) ++q;
        if (k < N) {
            int64_t x = 0;
            auto r = std::from_chars(p, q, x);
            if (r.ec != std::errc() || r.ptr != q || x < 1 || x > INT32_MAX) return false;
            ids[k] = x - 1;
        } else {
            float x = 0.0f;
            const char *s = (*p == '+') ? p + 1 : p;      // from_chars takes no '+'
            auto r = std::from_chars(s, q, x);
            if (r.ec != std::errc() || r.ptr != q || !std::isfinite(x)) return false;
            *v = x;
        }
        p = q;
    }
    return blank(p, e);
}

struct Chunk {
    const char *b, *e;
    int64_t lines = 0;           // newline-terminated or final lines
    int64_t entries = 0;
    int64_t bad_line = -1;       // first malformed line, within the chunk
    std::vector<int64_t> maxid;
};

// Cut the buffer into up to T pieces that end at line ends.
std::vector<Chunk> split_lines(const std::vector<char> &buf, int N) {
    const size_t n = buf.size();
    int T = (int)std::min<size_t>(16, std::max<size_t>(1, n >> 20));
    T = std::max(1, std::min<int>(T, (int)std::max(1u, std::thread::hardware_concurrency())));
    std::vector<Chunk> ch;
    const char *base = buf.data();
    size_t pos = 0;
    for (int t = 0; t < T && pos < n; ++t) {
        size_t end = (t == T - 1) ? n : std::max(pos, n * (t + 1) / T);
        while (end < n && base[end - 1] != '\n') ++end;
        Chunk c;
        c.b = base + pos;
        c.e = base + end;
        c.maxid.assign(N, -1);
        ch.push_back(c);
        pos = end;
    }
    return ch;
}

template <typename F>
void for_lines(const char *b, const char *e, F f) {
    while (b < e) {
        const char *nl = (const char *)memchr(b, '\n', e - b);
        const char *le = nl ? nl : e;
        f(b, le);
        b = nl ? nl + 1 : e;
    }
}

template <typename F>
void run_chunks(std::vector<Chunk> &ch, F f) {
    std::vector<std::thread> th;
    for (size_t t = 1; t < ch.size(); ++t) th.emplace_back(f, std::ref(ch[t]));
    if (!ch.empty()) f(ch[0]);
    for (auto &x : th) x.join();
}

// Count entries (and check them) per chunk; the first malformed line wins.
ptk_status scan_chunks(std::vector<Chunk> &ch, int N, const char *path) {
    run_chunks(ch, [N](Chunk &c) {
        int64_t ids[kMaxN];
        float v;
        for_lines(c.b, c.e, [&](const char *p, const char *e) {
            ++c.lines;
            if (c.bad_line >= 0 || blank(p, e)) return;
            if (!parse_entry(p, e, N, ids, &v)) {
                c.bad_line = c.lines;
                return;
            }
            ++c.entries;
            for (int k = 0; k < N; ++k) c.maxid[k] = std::max(c.maxid[k], ids[k]);
        });
    });
    int64_t before = 0;
    for (const Chunk &c : ch) {
        if (c.bad_line >= 0)
            return gfail(PTK_E_INVALID,
                         "%s line %lld: expected %d indices >= 1 and a finite value", path,
                         (long long)(before + c.bad_line), N);
        before += c.lines;
    }
    return PTK_OK;
}

}  // namespace

namespace ptk {
const char *global_error() { return g_err.c_str(); }
}  // namespace ptk

extern "C" {

ptk_status ptk_coo_scan(const char *path, int32_t N, int64_t *nnz_out, int64_t *dims_out) {
    if (!path || !nnz_out || !dims_out) return gfail(PTK_E_INVALID, "null argument");
    if (N < 1 || N > kMaxN) return gfail(PTK_E_INVALID, "N must be in [1, %d]", kMaxN);
    std::vector<char> buf;
    if (!read_file(path, buf)) return gfail(PTK_E_INVALID, "cannot read %s", path);
    std::vector<Chunk> ch = split_lines(buf, N);
    ptk_status s = scan_chunks(ch, N, path);
    if (s != PTK_OK) return s;
    int64_t nnz = 0;
    for (int k = 0; k < N; ++k) dims_out[k] = 0;
    for (const Chunk &c : ch) {
        nnz += c.entries;
        for (int k = 0; k < N; ++k) dims_out[k] = std::max(dims_out[k], c.maxid[k] + 1);
    }
    *nnz_out = nnz;
    return PTK_OK;
}

ptk_status ptk_coo_read(const char *path, int32_t N, int64_t nnz, int32_t *idx_host,
                        float *val_host) {
    if (!path || (nnz > 0 && (!idx_host || !val_host)))
        return gfail(PTK_E_INVALID, "null argument");
    if (N < 1 || N > kMaxN) return gfail(PTK_E_INVALID, "N must be in [1, %d]", kMaxN);
    std::vector<char> buf;
    if (!read_file(path, buf)) return gfail(PTK_E_INVALID, "cannot read %s", path);
    std::vector<Chunk> ch = split_lines(buf, N);
    ptk_status s = scan_chunks(ch, N, path);
    if (s != PTK_OK) return s;
    int64_t total = 0;
    std::vector<int64_t> first(ch.size());
    for (size_t t = 0; t < ch.size(); ++t) {
        first[t] = total;
        total += ch[t].entries;
    }
    if (total != nnz)
        return gfail(PTK_E_INVALID, "%s holds %lld entries, nnz = %lld", path,
                     (long long)total, (long long)nnz);
    std::vector<std::thread> th;
    auto fill = [&](size_t t) {
        int64_t pos = first[t];
        int64_t ids[kMaxN];
        float v;
        for_lines(ch[t].b, ch[t].e, [&](const char *p, const char *e) {
            if (blank(p, e)) return;
            parse_entry(p, e, N, ids, &v);          // checked by the scan
            for (int k = 0; k < N; ++k) idx_host[(int64_t)k * nnz + pos] = (int32_t)ids[k];
            val_host[pos] = v;
            ++pos;
        });
    };
    for (size_t t = 1; t < ch.size(); ++t) th.emplace_back(fill, t);
    if (!ch.empty()) fill(0);
    for (auto &x : th) x.join();
    return PTK_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// device kernels
// ---------------------------------------------------------------------------
namespace {

constexpr int kBlk = 256;
constexpr int kMinMaxBlocks = 1024;

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, kWave));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
    return v;
}

// part[2b] = min, part[2b+1] = max of block b's share
__global__ __launch_bounds__(kBlk) void k_minmax(const float *__restrict__ v, int64_t n,
                                                 double *__restrict__ part) {
    __shared__ double s_mn[kBlk / kWave], s_mx[kBlk / kWave];
    double mn = INFINITY, mx = -INFINITY;
    for (int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlk) {
        const double x = (double)v[i];
        mn = fmin(mn, x);
        mx = fmax(mx, x);
    }
    mn = wave_min(mn);
    mx = wave_max(mx);
    if (threadIdx.x % kWave == 0) {
        s_mn[threadIdx.x / kWave] = mn;
        s_mx[threadIdx.x / kWave] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlk / kWave; ++w) {
            mn = fmin(mn, s_mn[w]);
            mx = fmax(mx, s_mx[w]);
        }
        part[2 * blockIdx.x] = mn;
        part[2 * blockIdx.x + 1] = mx;
    }
}

// out[0..1] = min, max over nb block pairs (one wave)
__global__ __launch_bounds__(kWave) void k_minmax_final(const double *__restrict__ part,
                                                        int nb, double *__restrict__ out) {
    double mn = INFINITY, mx = -INFINITY;
    for (int b = threadIdx.x; b < nb; b += kWave) {
        mn = fmin(mn, part[2 * b]);
        mx = fmax(mx, part[2 * b + 1]);
    }
    mn = wave_min(mn);
    mx = wave_max(mx);
    if (threadIdx.x == 0) {
        out[0] = mn;
        out[1] = mx;
    }
}

// v <- (v - min) / (max - min) in FP64, rounded to FP32; 0 when max = min
__global__ __launch_bounds__(kBlk) void k_scale(float *__restrict__ v, int64_t n,
                                                const double *__restrict__ mm) {
    const double lo = mm[0], span = mm[1] - mm[0];
    for (int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlk)
        v[i] = span > 0.0 ? (float)(((double)v[i] - lo) / span) : 0.0f;
}

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): output number e + 1 of the
// generator seeded with `seed`, i.e. the mixing function applied to
// seed + (e + 1) * 0x9E3779B97F4A7C15 (mod 2^64).
__host__ __device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t e) {
    uint64_t z = seed + (e + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Entry e is held out when the top 53 bits of its draw, as a fraction of
// 2^53, are below the test fraction (exact in FP64).
__device__ __forceinline__ bool held_out(uint64_t seed, int64_t e, double frac) {
    return (double)(splitmix64_at(seed, (uint64_t)e) >> 11) * 0x1.0p-53 < frac;
}

constexpr int kSplitTile = 1024;

// held-out count per tile of kSplitTile entries
__global__ __launch_bounds__(kBlk) void k_split_count(int64_t nnz, double frac, uint64_t seed,
                                                      int64_t *__restrict__ tcount) {
    __shared__ int s_c[kBlk / kWave];
    const int64_t t0 = (int64_t)blockIdx.x * kSplitTile;
    int c = 0;
    for (int u = threadIdx.x; u < kSplitTile; u += kBlk) {
        const int64_t e = t0 + u;
        if (e < nnz && held_out(seed, e, frac)) ++c;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, kWave);
    if (threadIdx.x % kWave == 0) s_c[threadIdx.x / kWave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t s = 0;
        for (int w = 0; w < kBlk / kWave; ++w) s += s_c[w];
        tcount[blockIdx.x] = s;
    }
}

// exclusive scan of the tile counts in place (one workgroup, tile order);
// tcount[ntiles] receives the total
__global__ __launch_bounds__(kBlk) void k_split_scan(int64_t *__restrict__ tcount,
                                                     int64_t ntiles) {
    __shared__ int64_t s_part[kBlk];
    const int64_t per = (ntiles + kBlk - 1) / kBlk;
    const int64_t b0 = threadIdx.x * per, b1 = std::min<int64_t>(b0 + per, ntiles);
    int64_t s = 0;
    for (int64_t b = b0; b < b1; ++b) s += tcount[b];
    s_part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int t = 0; t < kBlk; ++t) {
            const int64_t x = s_part[t];
            s_part[t] = run;
            run += x;
        }
        tcount[ntiles] = run;
    }
    __syncthreads();
    int64_t run = s_part[threadIdx.x];
    for (int64_t b = b0; b < b1; ++b) {
        const int64_t x = tcount[b];
        tcount[b] = run;
        run += x;
    }
}

// Stable scatter: entries keep their order within each side.
__global__ __launch_bounds__(kBlk) void k_split_scatter(
    int64_t nnz, int N, double frac, uint64_t seed, const int32_t *__restrict__ idx,
    const float *__restrict__ val, const int64_t *__restrict__ tstart, int64_t ntest,
    int32_t *__restrict__ idx_tr, float *__restrict__ val_tr, int32_t *__restrict__ idx_te,
    float *__restrict__ val_te) {
    __shared__ int s_w[kBlk / kWave];
    __shared__ int64_t s_base;
    const int64_t t0 = (int64_t)blockIdx.x * kSplitTile;
    const int64_t ntrain = nnz - ntest;
    if (threadIdx.x == 0) s_base = tstart[blockIdx.x];
    __syncthreads();
    int64_t te_before = s_base;                   // held-out entries before this step
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    for (int u0 = 0; u0 < kSplitTile; u0 += kBlk) {
        const int64_t e = t0 + u0 + threadIdx.x;
        const bool in = e < nnz;
        const bool te = in && held_out(seed, e, frac);
        const unsigned long long bal = __ballot(te);
        const int below = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) s_w[w] = __popcll(bal);
        __syncthreads();
        int wbase = 0, step = 0;
        for (int q = 0; q < kBlk / kWave; ++q) {
            if (q < w) wbase += s_w[q];
            step += s_w[q];
        }
        if (in) {
            const int64_t rte = te_before + wbase + below;   // rank among held-out
            if (te) {
                for (int k = 0; k < N; ++k) idx_te[(int64_t)k * ntest + rte] = idx[(int64_t)k * nnz + e];
                val_te[rte] = val[e];
            } else {
                const int64_t rtr = e - rte;                  // rank among training
                for (int k = 0; k < N; ++k) idx_tr[(int64_t)k * ntrain + rtr] = idx[(int64_t)k * nnz + e];
                val_tr[rtr] = val[e];
            }
        }
        te_before += step;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// k-means over the rows of A (I x J, float32); centroids C (K x J, FP64)
// ---------------------------------------------------------------------------
// Nearest centroid per row (squared Euclidean distance in FP64, the lowest
// index among equal distances); counts the rows whose assignment changed and
// stores the distance for the inertia.
__global__ __launch_bounds__(kBlk) void k_km_assign(const float *__restrict__ A, int64_t I,
                                                    int J, const double *__restrict__ C,
                                                    int K, int32_t *__restrict__ assign,
                                                    double *__restrict__ dist,
                                                    int32_t *__restrict__ changed) {
    extern __shared__ double s_c[];
    for (int t = threadIdx.x; t < K * J; t += kBlk) s_c[t] = C[t];
    __syncthreads();
    int ch = 0;
    for (int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x; i < I;
         i += (int64_t)gridDim.x * kBlk) {
        const float *a = A + i * J;
        int best = 0;
        double bd = INFINITY;
        for (int k = 0; k < K; ++k) {
            double d = 0.0;
            for (int j = 0; j < J; ++j) {
                const double t = (double)a[j] - s_c[k * J + j];
                d = __builtin_fma(t, t, d);
            }
            if (d < bd) {
                bd = d;
                best = k;
            }
        }
        if (assign[i] != best) ++ch;
        assign[i] = best;
        dist[i] = bd;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) ch += __shfl_xor(ch, off, kWave);
    if (threadIdx.x % kWave == 0 && ch) atomicAdd(changed, ch);   // integer: exact
}

// Per-block sums of the rows of each cluster over a contiguous row range,
// rows added one at a time in order (deterministic): part[b][k][J + 1]
// (J coordinate sums, then the count). Rows are staged 64 at a time in LDS;
// lane j < J owns coordinate j, lane J the count.
__global__ __launch_bounds__(kWave) void k_km_partial(const float *__restrict__ A, int64_t I,
                                                      int J, const int32_t *__restrict__ assign,
                                                      int K, int64_t rows_per_block,
                                                      double *__restrict__ part) {
    extern __shared__ double s_acc[];             // K * (J + 1), then the staged rows
    float *s_rows = (float *)(s_acc + K * (J + 1));
    const int lane = threadIdx.x;
    const int W = J + 1;
    for (int t = lane; t < K * W; t += kWave) s_acc[t] = 0.0;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = std::min<int64_t>(r0 + rows_per_block, I);
    for (int64_t i0 = r0; i0 < r1; i0 += kWave) {
        const int nr = (int)std::min<int64_t>(kWave, r1 - i0);
        const int my_k = lane < nr ? assign[i0 + lane] : 0;
        __syncthreads();
        for (int t = lane; t < nr * J; t += kWave) s_rows[t] = A[i0 * J + t];
        __syncthreads();
        for (int r = 0; r < nr; ++r) {
            const int k = __shfl(my_k, r, kWave);
            if (lane < J) s_acc[k * W + lane] += (double)s_rows[r * J + lane];
            else if (lane == J) s_acc[k * W + J] += 1.0;
        }
    }
    __syncthreads();
    double *dst = part + (int64_t)blockIdx.x * K * W;
    for (int t = lane; t < K * W; t += kWave) dst[t] = s_acc[t];
}

// C[k] = mean of its rows (blocks summed in order); clusters without rows
// keep their centroid.
__global__ __launch_bounds__(kBlk) void k_km_update(const double *__restrict__ part, int nb,
                                                    int K, int J, double *__restrict__ C) {
    const int W = J + 1;
    for (int t = blockIdx.x * kBlk + threadIdx.x; t < K * J; t += gridDim.x * kBlk) {
        const int k = t / J, j = t % J;
        double s = 0.0, n = 0.0;
        for (int b = 0; b < nb; ++b) {
            s += part[((int64_t)b * K + k) * W + j];
            n += part[((int64_t)b * K + k) * W + J];
        }
        if (n > 0.0) C[t] = s / n;
    }
}

__global__ void k_fill_i32v(int32_t *p, int32_t v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Sum of d over n values: per-block partials over a fixed stride pattern,
// then the partials in block order (deterministic).
__global__ __launch_bounds__(kBlk) void k_sum_part(const double *__restrict__ d, int64_t n,
                                                   double *__restrict__ part) {
    __shared__ double s_p[kBlk / kWave];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlk)
        s += d[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, kWave);
    if (threadIdx.x % kWave == 0) s_p[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kBlk / kWave; ++w) t += s_p[w];
        part[blockIdx.x] = t;
    }
}

__global__ void k_sum_final(const double *__restrict__ part, int nb, double *__restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double t = 0.0;
        for (int b = 0; b < nb; ++b) t += part[b];
        out[0] = t;
    }
}

}  // namespace

namespace ptk {
uint64_t splitmix64_host(uint64_t seed, uint64_t e) { return splitmix64_at(seed, e); }
}  // namespace ptk

extern "C" {

ptk_status ptk_normalize_values(ptk_ctx *c, int64_t nnz, float *val, double *minmax_host) {
    if (!c) return gfail(PTK_E_INVALID, "null context");
    if (nnz < 0) return cfail(c, PTK_E_INVALID, "nnz < 0");
    if (nnz > 0 && !val) return cfail(c, PTK_E_INVALID, "null values");
    double *part = nullptr;
    DCHK(c, hipMalloc(&part, (2 * kMinMaxBlocks + 2) * sizeof(double)));
    double *mm = part + 2 * kMinMaxBlocks;
    const int nb = (int)std::max<int64_t>(
        1, std::min<int64_t>(kMinMaxBlocks, (nnz + kBlk - 1) / kBlk));
    hipError_t e = hipSuccess;
    if (nnz > 0) {
        hipLaunchKernelGGL(k_minmax, dim3(nb), dim3(kBlk), 0, c->st, val, nnz, part);
        hipLaunchKernelGGL(k_minmax_final, dim3(1), dim3(kWave), 0, c->st, part, nb, mm);
        hipLaunchKernelGGL(k_scale, dim3(nb), dim3(kBlk), 0, c->st, val, nnz, mm);
        e = hipGetLastError();
    }
    double h[2] = {0.0, 0.0};
    if (e == hipSuccess && nnz > 0)
        e = hipMemcpyAsync(h, mm, sizeof h, hipMemcpyDeviceToHost, c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    hipFree(part);
    DCHK(c, e);
    if (minmax_host) {
        minmax_host[0] = h[0];
        minmax_host[1] = h[1];
    }
    return PTK_OK;
}

static ptk_status split_prepare(ptk_ctx *c, int64_t nnz, double frac, uint64_t seed,
                                int64_t **tcount, int64_t *ntest) {
    const int64_t ntiles = (nnz + kSplitTile - 1) / kSplitTile;
    DCHK(c, hipMalloc(tcount, (ntiles + 1) * sizeof(int64_t)));
    hipLaunchKernelGGL(k_split_count, dim3((unsigned)ntiles), dim3(kBlk), 0, c->st, nnz, frac,
                       seed, *tcount);
    hipLaunchKernelGGL(k_split_scan, dim3(1), dim3(kBlk), 0, c->st, *tcount, ntiles);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(ntest, *tcount + ntiles, sizeof(int64_t), hipMemcpyDeviceToHost,
                           c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    if (e != hipSuccess) {
        hipFree(*tcount);
        *tcount = nullptr;
        DCHK(c, e);
    }
    return PTK_OK;
}

ptk_status ptk_split_count(ptk_ctx *c, int64_t nnz, double test_fraction, uint64_t seed,
                           int64_t *ntest_host) {
    if (!c) return gfail(PTK_E_INVALID, "null context");
    if (nnz < 0 || !ntest_host) return cfail(c, PTK_E_INVALID, "nnz < 0 or null output");
    if (!(test_fraction >= 0.0 && test_fraction <= 1.0))
        return cfail(c, PTK_E_INVALID, "test_fraction must be in [0, 1]");
    *ntest_host = 0;
    if (nnz == 0) return PTK_OK;
    int64_t *tcount = nullptr;
    ptk_status s = split_prepare(c, nnz, test_fraction, seed, &tcount, ntest_host);
    hipFree(tcount);
    return s;
}

ptk_status ptk_split_entries(ptk_ctx *c, int32_t N, int64_t nnz, const int32_t *idx,
                             const float *val, double test_fraction, uint64_t seed,
                             int64_t ntest, int32_t *idx_train, float *val_train,
                             int32_t *idx_test, float *val_test) {
    if (!c) return gfail(PTK_E_INVALID, "null context");
    if (N < 1 || N > kMaxN) return cfail(c, PTK_E_INVALID, "N must be in [1, %d]", kMaxN);
    if (nnz < 0) return cfail(c, PTK_E_INVALID, "nnz < 0");
    if (!(test_fraction >= 0.0 && test_fraction <= 1.0))
        return cfail(c, PTK_E_INVALID, "test_fraction must be in [0, 1]");
    if (nnz == 0) return ntest == 0 ? PTK_OK : cfail(c, PTK_E_INVALID, "ntest mismatch");
    if (!idx || !val || (ntest < nnz && (!idx_train || !val_train)) ||
        (ntest > 0 && (!idx_test || !val_test)))
        return cfail(c, PTK_E_INVALID, "null buffer");
    int64_t *tcount = nullptr, have = 0;
    ptk_status s = split_prepare(c, nnz, test_fraction, seed, &tcount, &have);
    if (s != PTK_OK) return s;
    if (have != ntest) {
        hipFree(tcount);
        return cfail(c, PTK_E_INVALID, "ntest = %lld, but the split holds out %lld",
                     (long long)ntest, (long long)have);
    }
    const int64_t ntiles = (nnz + kSplitTile - 1) / kSplitTile;
    hipLaunchKernelGGL(k_split_scatter, dim3((unsigned)ntiles), dim3(kBlk), 0, c->st, nnz, N,
                       test_fraction, seed, idx, val, tcount, ntest, idx_train, val_train,
                       idx_test, val_test);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    hipFree(tcount);
    DCHK(c, e);
    return PTK_OK;
}

ptk_status ptk_kmeans(ptk_ctx *c, int32_t n, int32_t K, int32_t iters, double *centroids,
                      int32_t *assign, double *result_host) {
    if (!c) return gfail(PTK_E_INVALID, "null context");
    if (n < 0 || n >= c->s.N) return cfail(c, PTK_E_INVALID, "mode %d out of range", n);
    if (!c->core) return cfail(c, PTK_E_STATE, "no model bound (ptk_bind_model)");
    const int J = c->s.ranks[n];
    const int64_t I = c->s.dims[n];
    if (K < 1 || (int64_t)K * (J + 1) * 8 > 32768)
        return cfail(c, PTK_E_INVALID, "K must be in [1, %d] for J = %d", 32768 / (8 * (J + 1)),
                     J);
    if (iters < 0) return cfail(c, PTK_E_INVALID, "iters < 0");
    if (!centroids || !assign) return cfail(c, PTK_E_INVALID, "null buffer");
    const float *A = c->fac[n];
    const int64_t nb = std::max<int64_t>(1, std::min<int64_t>(1024, (I + 63) / 64));
    const int64_t rpb = (I + nb - 1) / nb;
    const int ab = (int)std::max<int64_t>(1, std::min<int64_t>(4096, (I + kBlk - 1) / kBlk));
    double *work = nullptr;
    const size_t part_d = (size_t)nb * K * (J + 1);
    DCHK(c, hipMalloc(&work, (part_d + I + 1) * sizeof(double) + 2 * sizeof(int32_t) + 64));
    double *part = work, *dist = work + part_d, *inert = dist + I;
    int32_t *changed = (int32_t *)(inert + 1);
    const size_t lds_c = (size_t)K * J * 8;
    const size_t lds_p = (size_t)K * (J + 1) * 8 + (size_t)kWave * J * 4;
    hipError_t e = hipSuccess;
    hipLaunchKernelGGL(k_fill_i32v, dim3((unsigned)((I + 255) / 256)), dim3(256), 0, c->st,
                       assign, -1, I);
    for (int t = 0; t <= iters && e == hipSuccess; ++t) {
        hipLaunchKernelGGL(k_fill_i32v, dim3(1), dim3(64), 0, c->st, changed, 0, (int64_t)1);
        hipLaunchKernelGGL(k_km_assign, dim3(ab), dim3(kBlk), lds_c, c->st, A, I, J, centroids,
                           K, assign, dist, changed);
        if (t < iters) {
            hipLaunchKernelGGL(k_km_partial, dim3((unsigned)nb), dim3(kWave), lds_p, c->st, A,
                               I, J, assign, K, rpb, part);
            hipLaunchKernelGGL(k_km_update, dim3((unsigned)((K * J + kBlk - 1) / kBlk)),
                               dim3(kBlk), 0, c->st, part, (int)nb, K, J, centroids);
        }
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        // the per-block partials reuse the head of part (nb * K * (J + 1) >= 1024
        // doubles is not guaranteed, so at most that many blocks)
        const int sb = (int)std::max<int64_t>(
            1, std::min<int64_t>(std::min<int64_t>(1024, (int64_t)part_d),
                                 (I + kBlk - 1) / kBlk));
        hipLaunchKernelGGL(k_sum_part, dim3(sb), dim3(kBlk), 0, c->st, dist, I, part);
        hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(64), 0, c->st, part, sb, inert);
        e = hipGetLastError();
    }
    double h = 0.0;
    int32_t ch = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&h, inert, sizeof h, hipMemcpyDeviceToHost, c->st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&ch, changed, sizeof ch, hipMemcpyDeviceToHost, c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    hipFree(work);
    DCHK(c, e);
    if (result_host) {
        result_host[0] = h;
        result_host[1] = (double)ch;
    }
    return PTK_OK;
}

}  // extern "C"
