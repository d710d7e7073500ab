// Row systems from a sparse core (the Approx variant, Alg. 4 with Sec. 3.3):
// after the removals most cells of G are zero, and delta (eq. "delta") only
// needs the non-zero ones:
//     delta_j = sum over non-zero cells beta with beta_n = j of
//               G_beta * prod_{k != n} a^(k)_{i_k beta_k}.
// The dense kernels run the contraction chain: about one instruction per
// core cell (an FMA whose core operand is an SGPR), whatever its value. Here
// a non-zero cell costs its last factor value (a register-indexed move and
// a widening), one product and one FMA, plus the scalar work of reading its
// record, so it pays only once few cells are left; every issued instruction,
// scalar or vector, takes an issue slot of the wavefront.
//
// Cell lists (ptk_sparse.h): k_sparse_count / k_sparse_fill build them from
// the bound core on the device, one workgroup per (mode, j), at the start of
// every iteration (inside a captured graph), and set the per-mode switch
// use[n] = (non-zero cells <= limit * cells).
//
// k_gram_sparse<N, J, P>: P entries per lane, tiles of 64 P entries. The
// lanes' factor rows of the other modes stay in VGPRs and are read with the
// wavefront-uniform register indices of the records. The product over the
// leading slots is kept and redone only from the slot the record names
// (always formed in slot order, so the result does not depend on which
// products were kept). Records come through the scalar cache one ahead of
// their use: the next record's load is issued after the wait for the
// current one. Then the same sweep into the packed row systems as the dense
// kernels (ptk_device.h). Both the dense and the sparse kernel are
// launched; each reads use[n] and the one not chosen returns at once, so the
// switch needs no host round trip.
#include "ptk_device.h"
#include "ptk_sparse.h"

namespace ptk {

namespace {

// Other-mode indices of the r-th cell (C order over the other modes) with
// beta_n = j: slot digits packed 8 bits each (slot 0 lowest); returns the
// cell's index in the C-order core.
__device__ __forceinline__ int64_t sparse_cell(int N, int n, int J, int64_t r, int j,
                                               uint32_t *packed) {
    int dig[kMaxN];
    int64_t t = r;
    for (int k = N - 1; k >= 0; --k) {
        if (k == n) {
            dig[k] = j;
            continue;
        }
        dig[k] = (int)(t % J);
        t /= J;
    }
    int64_t idx = 0;
    uint32_t p = 0;
    int slot = 0;
    for (int k = 0; k < N; ++k) {
        idx = idx * J + dig[k];
        if (k != n) p |= (uint32_t)dig[k] << (8 * slot++);
    }
    *packed = p;
    return idx;
}

}  // namespace

// counts[n * J + j] = non-zero cells of mode n with beta_n = j
__global__ __launch_bounds__(256) void k_sparse_count(const float *__restrict__ G,
                                                      SparseArgs s) {
    __shared__ int32_t s_cnt[4];
    const int n = blockIdx.x / s.J, j = blockIdx.x % s.J;
    const int64_t per = s.cells / s.J;
    int32_t c = 0;
    for (int64_t r = threadIdx.x; r < per; r += blockDim.x) {
        uint32_t pk;
        c += G[sparse_cell(s.N, n, s.J, r, j, &pk)] != 0.0f;
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) c += __shfl_xor(c, off, kWave);
    if (threadIdx.x % kWave == 0) s_cnt[threadIdx.x / kWave] = c;
    __syncthreads();
    if (threadIdx.x == 0) s.count[blockIdx.x] = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
}

// The records of (n, j) in order; cstart, the empty record and use[] from
// the counts.
__global__ __launch_bounds__(256) void k_sparse_fill(const float *__restrict__ G,
                                                     SparseArgs s) {
    __shared__ int32_t s_base;
    __shared__ int32_t s_wave[4];
    __shared__ uint32_t s_wlast[4];          // each wave's last listed digits
    __shared__ uint32_t s_last;              // the last listed digits so far
    __shared__ int32_t s_any;                // any cell listed so far
    const int N = s.N, J = s.J, NO = N - 1;
    const int n = blockIdx.x / J, j = blockIdx.x % J;
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    const int64_t per = s.cells / J;
    int32_t *cstart = s.cstart + (int64_t)n * (J + 1);
    uint32_t *rec = s.recs + (int64_t)n * s.rec * 4;
    if (threadIdx.x == 0) {
        int32_t b = 0, tot = 0;
        for (int q = 0; q < J; ++q) {
            if (q < j) b += s.count[n * J + q];
            tot += s.count[n * J + q];
        }
        s_base = b;
        s_any = 0;
        s_last = 0;
        cstart[j] = b;
        if (j == J - 1) {
            cstart[J] = tot;
            rec[(int64_t)tot * 4 + 0] = 0;   // the empty record after the last
            rec[(int64_t)tot * 4 + 1] = 0;
            rec[(int64_t)tot * 4 + 2] = (uint32_t)((NO - 1) * J);
            rec[(int64_t)tot * 4 + 3] = (uint32_t)(NO - 1) << 24;
            s.use[n] = (double)tot <= s.limit * (double)s.cells ? 1 : 0;
        }
    }
    __syncthreads();
    for (int64_t r0 = 0; r0 < per; r0 += blockDim.x) {
        const int64_t r = r0 + threadIdx.x;
        uint32_t pk = 0;
        float v = 0.0f;
        if (r < per) v = G[sparse_cell(N, n, J, r, j, &pk)];
        const bool nz = r < per && v != 0.0f;
        const unsigned long long m = __ballot(nz);
        const unsigned long long lower = m & ((1ull << lane) - 1ull);
        // digits of the listed cell before this one in list order
        const int pl = lower ? 63 - __clzll(lower) : 0;
        const uint32_t pk_lane = __shfl(pk, pl, kWave);
        const int last_lane = m ? 63 - __clzll(m) : 0;
        const uint32_t pk_last = __shfl(pk, last_lane, kWave);
        if (lane == 0) {
            s_wave[wid] = (int32_t)__popcll(m);
            if (m) s_wlast[wid] = pk_last;
        }
        __syncthreads();
        int32_t before = 0, total = 0;
        for (int q = 0; q < 4; ++q) {
            if (q < wid) before += s_wave[q];
            total += s_wave[q];
        }
        if (nz) {
            bool have = lower != 0;
            uint32_t prevpk = pk_lane;
            for (int q = wid - 1; q >= 0 && !have; --q)
                if (s_wave[q]) {
                    have = true;
                    prevpk = s_wlast[q];
                }
            if (!have && s_any) {
                have = true;
                prevpk = s_last;
            }
            int lvl = 0;
            if (have) {
                const uint32_t diff = pk ^ prevpk;
                lvl = diff ? (int)(__builtin_ctz(diff) >> 3) : NO - 1;
                if (lvl > NO - 1) lvl = NO - 1;
            }
            uint32_t lead = 0;
            for (int l = 0; l < NO - 1; ++l)
                lead |= (uint32_t)(l * J + (int)((pk >> (8 * l)) & 0xffu)) << (8 * l);
            const int64_t at = s_base + before + (int32_t)__popcll(lower);
            const double g = (double)v;
            const unsigned long long gb = (unsigned long long)__double_as_longlong(g);
            rec[at * 4 + 0] = (uint32_t)gb;
            rec[at * 4 + 1] = (uint32_t)(gb >> 32);
            rec[at * 4 + 2] = (uint32_t)((NO - 1) * J + (int)((pk >> (8 * (NO - 1))) & 0xffu));
            rec[at * 4 + 3] = lead | ((uint32_t)lvl << 24);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            s_base += total;
            for (int q = 3; q >= 0; --q)
                if (s_wave[q]) {
                    s_last = s_wlast[q];
                    s_any = 1;
                    break;
                }
        }
        __syncthreads();
    }
}

hipError_t launch_sparse_lists(const float *G, const SparseArgs &s, hipStream_t st) {
    const unsigned blocks = (unsigned)(s.N * s.J);
    hipLaunchKernelGGL(k_sparse_count, dim3(blocks), dim3(256), 0, st, G, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sparse_fill, dim3(blocks), dim3(256), 0, st, G, s);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// the row-system kernel
// ---------------------------------------------------------------------------
template <int N, int J, int P>
__global__ __launch_bounds__(kWave) void k_gram_sparse(GramArgs a, SparseMode sm) {
    if (!*sm.use) return;                    // the dense kernel has this mode
    constexpr int NO = N - 1;
    constexpr int NP = NO > 1 ? NO - 1 : 1;  // kept products of leading slots
    constexpr int E = sys_entries(J);
    constexpr int EPL = (E + kWave - 1) / kWave;
    static_assert(NO >= 2 && NO <= 4, "records hold up to three leading slots");
    static_assert(P == 1 || P == 2, "one or two entries per lane");
    __shared__ double s_dl[(J + 1) * kDlStride];
    __shared__ int s_row[kWave];
    cptr<uint32_t> rec = (cptr<uint32_t>)sm.recs;
    cptr<int32_t> cstart = (cptr<int32_t>)sm.cstart;

    const int lane = threadIdx.x;
    const int64_t chunk = blockIdx.x;
    const int64_t cs = chunk * a.chunk;
    const int64_t ce = min(cs + a.chunk, a.nnz);

    SysLane<EPL> sl;
    sl.init(lane, J);
    int cur = -1;
    for (int64_t base = cs; base < ce; base += P * kWave) {
        // one array per entry: each stays in VGPRs (a two-dimensional one
        // would go to scratch)
        float rv0[NO * J], rv1[NO * J];
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const int64_t pos = base + q * kWave + lane;
            const bool valid = pos < ce;
#pragma unroll
            for (int k = 0; k < NO; ++k) {
                const int32_t i = valid ? a.oidx[k][pos] : 0;
                const float *r = a.fac[k] + (int64_t)i * J;
#pragma unroll
                for (int m = 0; m < J; ++m) {
                    if (q == 0) rv0[k * J + m] = r[m];
                    else rv1[k * J + m] = r[m];
                }
            }
        }
        // the rows are in registers before the record loop (no waits on
        // their loads inside it)
#pragma unroll
        for (int i = 0; i < NO * J; ++i) {
            asm volatile("" : "+v"(rv0[i]));
            if (P == 2) asm volatile("" : "+v"(rv1[i]));
        }
        auto rowv = [&](int q, uint32_t i) -> double {
            return (double)(q == 0 ? rv0[i] : rv1[i]);
        };
        double d[P][J];
        double pre[P][NP];
        int32_t c = cstart[0];
        cptr<uint32_t> rp = rec + 4 * (int64_t)c;
        uint32_t n0 = rp[0], n1 = rp[1], n2 = rp[2], n3 = rp[3];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            double acc[P];
#pragma unroll
            for (int q = 0; q < P; ++q) acc[q] = 0.0;
            const int32_t cend = cstart[j + 1];
            for (; c < cend; ++c, rp += 4) {
                // take this record (waits for its loads) before the next
                // record's loads are issued
                asm volatile("" : "+s"(n0), "+s"(n1), "+s"(n2), "+s"(n3)::"memory");
                const uint32_t gl = n0, gh = n1, ix = n2, lead = n3;
                n0 = rp[4];
                n1 = rp[5];
                n2 = rp[6];
                n3 = rp[7];
                const double g =
                    __longlong_as_double((long long)(((unsigned long long)gh << 32) | gl));
                const uint32_t lvl = lead >> 24;
                if (lvl < (uint32_t)(NO - 1)) {
#pragma unroll
                    for (int l = 0; l < NO - 1; ++l) {
                        if ((uint32_t)l >= lvl) {
                            const uint32_t li = (lead >> (8 * l)) & 0xffu;
#pragma unroll
                            for (int q = 0; q < P; ++q) {
                                const double v = rowv(q, li);
                                pre[q][l] = l == 0 ? v : pre[q][l > 0 ? l - 1 : 0] * v;
                            }
                        }
                    }
                }
#pragma unroll
                for (int q = 0; q < P; ++q)
                    acc[q] = __builtin_fma(g, pre[q][NO - 2] * rowv(q, ix), acc[q]);
            }
#pragma unroll
            for (int q = 0; q < P; ++q) d[q][j] = acc[q];
        }
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const int64_t pos = base + q * kWave + lane;
            const bool valid = pos < ce;
            const int nb = (int)max((int64_t)0, min((int64_t)kWave, ce - base - q * kWave));
            if (nb == 0) break;                  // uniform
            if (a.dstore && valid) {
#pragma unroll
                for (int j = 0; j < J; ++j) a.dstore[(int64_t)j * a.nnz + pos] = d[q][j];
            }
            const int rw = valid ? (a.rows ? a.rows[pos] : 0) : 0;
            if (a.kbase && valid) {          // deltas of least-squares rows
                const int64_t kb = a.kbase[rw];
                if (kb != kNoKeep) {
#pragma unroll
                    for (int j = 0; j < J; ++j) a.keep[(kb + pos) * J + j] = d[q][j];
                }
            }
#pragma unroll
            for (int j = 0; j < J; ++j) s_dl[j * kDlStride + lane] = d[q][j];
            s_dl[J * kDlStride + lane] = valid ? (double)a.val[pos] : 0.0;
            s_row[lane] = rw;
            __syncthreads();
            sweep_tile<EPL>(a, sl, s_dl, s_row, nb, cur, chunk, cs, ce);
            __syncthreads();
        }
    }
    if (cur >= 0) flush_row<EPL>(a, sl, cur, chunk, cs, ce);
}

// the shapes of the Approx kernels
#define PTK_SPARSE_SHAPES(X)                                                    \
    X(3, 3) X(3, 4) X(3, 5) X(3, 8) X(3, 10) X(3, 16) X(4, 3) X(4, 5) X(4, 8) \
    X(4, 10) X(5, 3) X(5, 5) X(5, 8)

// entries per lane: two share every record's scalar work
constexpr int kSpEntries = 2;

bool sparse_available(int N, int J) {
#define PTK_X(n_, j_) if (N == n_ && J == j_) return true;
    PTK_SPARSE_SHAPES(PTK_X)
#undef PTK_X
    return false;
}

hipError_t launch_gram_sparse(const GramArgs &a, int N, int J, const SparseMode &sm,
                              int64_t nchunks, hipStream_t st) {
    if (nchunks <= 0) return hipSuccess;
#define PTK_X(n_, j_)                                                                 \
    if (N == n_ && J == j_) {                                                         \
        hipLaunchKernelGGL((k_gram_sparse<n_, j_, kSpEntries>), dim3((unsigned)nchunks), \
                           dim3(kWave), 0, st, a, sm);                                \
        return hipGetLastError();                                                     \
    }
    PTK_SPARSE_SHAPES(PTK_X)
#undef PTK_X
    return hipErrorInvalidValue;
}

}  // namespace ptk
