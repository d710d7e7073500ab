// Approx variant of the ALS sweep (Alg. 4, Sec. 3.3): the partial
// reconstruction error of every core cell (eq. "recon_partial") and the
// removal of the cells with the largest values.
//
// With r = xhat - x and w(alpha, beta) = prod_n a^(n)_{i_n beta_n}, the
// definition sum_alpha (x - xhat)^2 - (x - xhat + t)^2, t = G_beta w, becomes
//     R(beta) = 2 G_beta S1(beta) - G_beta^2 S2(beta),
//     S1 = sum_alpha r w,   S2 = sum_alpha w^2,
// two sums over the entries of Kronecker products of factor rows.
//
// The sums are linear in the entries, and the entries are grouped by the
// rows of one mode g: with T_i(beta') the sum over the entries of row i of
// r (resp. 1) times the product of the other modes' factor elements at
// beta' (and its square for S2),
//     S1(beta) = sum_i a^(g)_{i beta_g} T1_i(beta'),
//     S2(beta) = sum_i (a^(g)_{i beta_g})^2 T2_i(beta'),
// so each entry costs J^(N-1) products instead of J^N, and a row is folded
// in with J multiply-adds when it ends (rows split between slices need no
// merge: each piece is folded in on its own).
//
// Two forms compute the same S1, S2 (up to rounding order): the per-cell
// groups below (any order) and the row sums further down (orders 4 and 5).
//
// Per-cell groups: a wavefront owns 64 cells beta' of T: lane l takes a
// value p of the last two other modes, the wavefront fixes the others (the
// third-last through one index k, the ones before through its lead group),
// and it accumulates the J values of beta_g for each of them. It walks a
// slice of the entries, 64 at a time: each lane stages one entry's
// residual-weighted leading product in LDS (the same for the whole
// wavefront, read back as one broadcast per entry), the wavefront then
// copies the 64 entries' rows of the last two other modes into LDS with
// contiguous loads, and every lane reads its two elements per entry from
// there and accumulates. Sums are FP64; the slices are reduced in a fixed
// order.
#include "ptk_approx.h"
#include "ptk_device.h"

namespace ptk {

#define PTK_APPROX_SHAPES(X) PTK_FAST_SHAPES_LIST(X)

// the same shapes as the fast row-system kernels
#define PTK_FAST_SHAPES_LIST(X) \
    X(3, 3) X(3, 4) X(3, 5) X(3, 8) X(3, 10) X(3, 16) \
    X(4, 3) X(4, 5) X(4, 8) X(4, 10) \
    X(5, 3) X(5, 5) X(5, 8)

__host__ __device__ inline int64_t ipow_rt(int64_t b, int e) {
    int64_t r = 1;
    for (int k = 0; k < e; ++k) r *= b;
    return r;
}

bool approx_available(int N, int J) {
#define PTK_X(n_, j_) if (N == n_ && J == j_) return true;
    PTK_APPROX_SHAPES(PTK_X)
#undef PTK_X
    return false;
}

// ---------------------------------------------------------------------------
// residuals xhat - x (FP64) over one mode's grouping
// ---------------------------------------------------------------------------
template <int N, int J, int U>
__global__ __launch_bounds__(kWave) void k_residual(EntryArgs a) {
    constexpr int NO = N - 1;
    constexpr int NOUT = NO - U;
    __shared__ float s_aout[(NOUT > 0 ? NOUT : 1) * J * kWave];
    const int lane = threadIdx.x;
    for (int64_t base = (int64_t)blockIdx.x * kWave; base < a.m;
         base += (int64_t)gridDim.x * kWave) {
        const int64_t pos = base + lane;
        const bool valid = pos < a.m;
        double ain[U][J];
        load_rows_fast<NO, J, U, double>(a, pos, valid, s_aout, lane, ain);
        __syncthreads();
        double d[J];
        delta_fast<NO, J, U, double>(a.gp, s_aout, lane, ain, d);
        __syncthreads();
        if (valid) {
            const float *own = a.own + (int64_t)a.own_idx[pos] * J;
            double xh = 0.0;
#pragma unroll
            for (int j = 0; j < J; ++j) xh = __builtin_fma((double)own[j], d[j], xh);
            a.partial[pos] = xh - (double)a.val[pos];
        }
    }
}

hipError_t launch_residual(const EntryArgs &a, const Shape &s, int64_t nblocks,
                           hipStream_t st) {
    if (a.m <= 0 || nblocks <= 0) return hipSuccess;
    const int J = s.ranks[0];
#define PTK_X(n_, j_)                                                               \
    if (s.N == n_ && J == j_) {                                                     \
        hipLaunchKernelGGL((k_residual<n_, j_, fast_depth(n_, j_)>), dim3((unsigned)nblocks), \
                           dim3(kWave), 0, st, a);                                  \
        return hipGetLastError();                                                   \
    }
    PTK_APPROX_SHAPES(PTK_X)
#undef PTK_X
    return hipErrorInvalidValue;
}

// The same residuals from deltas the last mode's row-system kernel stored
// ([J][nnz], its grouped order): xhat = delta . a_new, J multiply-adds.
template <int J>
__global__ void k_resid_from_delta(const double *__restrict__ delta,
                                   const float *__restrict__ fac,
                                   const int32_t *__restrict__ rows,
                                   const float *__restrict__ val, int64_t nnz,
                                   double *__restrict__ resid) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nnz) return;
    const float *own = fac + (int64_t)rows[p] * J;
    double xh = 0.0;
#pragma unroll
    for (int j = 0; j < J; ++j) xh = __builtin_fma((double)own[j], delta[(int64_t)j * nnz + p], xh);
    resid[p] = xh - (double)val[p];
}

// Residuals from kept deltas and, in the same pass, the row-sum form's
// per-entry weights uw[e] = (r a[k], a[k]^2), a the entry's row of the
// third-last other mode. A wavefront forms the residuals of 64 entries
// (lane = entry) and stages them with the entries' rows in LDS, then writes
// their 2J weights each as one contiguous run of 64 x 2J doubles (lane =
// consecutive output).
template <int J>
__global__ __launch_bounds__(kWave) void k_resid_uw_from_delta(
    const double *__restrict__ delta, const float *__restrict__ fac,
    const int32_t *__restrict__ rows, const float *__restrict__ val,
    const float *__restrict__ fac3, const int32_t *__restrict__ idx3, int64_t nnz,
    double *__restrict__ resid, double *__restrict__ uw) {
    __shared__ double s_r[kWave];
    __shared__ float s_a[kWave * J];
    const int lane = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kWave;
    const int64_t p = base + lane;
    double r = 0.0;
    if (p < nnz) {
        const float *own = fac + (int64_t)rows[p] * J;
        const float *a3 = fac3 + (int64_t)idx3[p] * J;
        double xh = 0.0;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            xh = __builtin_fma((double)own[j], delta[(int64_t)j * nnz + p], xh);
            s_a[lane * J + j] = a3[j];
        }
        r = xh - (double)val[p];
        resid[p] = r;
    }
    s_r[lane] = r;
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 2 * J; ++t) {
        const int o = t * kWave + lane;            // output within the run
        const int e = o / (2 * J), kk = o % (2 * J);
        if (base + e < nnz) {
            const int k = kk < J ? kk : kk - J;
            const double a = (double)s_a[e * J + k];
            uw[base * 2 * J + o] = kk < J ? s_r[e] * a : a * a;
        }
    }
}

hipError_t launch_resid_uw_from_delta(const double *delta, const float *fac,
                                      const int32_t *rows, const float *val,
                                      const float *fac3, const int32_t *idx3, int64_t nnz,
                                      int J, double *resid, double *uw, hipStream_t st) {
    if (nnz <= 0) return hipSuccess;
    const dim3 grid((unsigned)((nnz + kWave - 1) / kWave)), block(kWave);
    switch (J) {
#define PTK_X(j_)                                                                          \
    case j_:                                                                               \
        hipLaunchKernelGGL(k_resid_uw_from_delta<j_>, grid, block, 0, st, delta, fac, rows,  \
                           val, fac3, idx3, nnz, resid, uw);                               \
        return hipGetLastError();
        PTK_X(3) PTK_X(5) PTK_X(8) PTK_X(10)
#undef PTK_X
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_resid_from_delta(const double *delta, const float *fac, const int32_t *rows,
                                   const float *val, int64_t nnz, int J, double *resid,
                                   hipStream_t st) {
    if (nnz <= 0) return hipSuccess;
    const dim3 grid((unsigned)((nnz + 255) / 256)), block(256);
    switch (J) {
#define PTK_X(j_)                                                                          \
    case j_:                                                                               \
        hipLaunchKernelGGL(k_resid_from_delta<j_>, grid, block, 0, st, delta, fac, rows, val, \
                           nnz, resid);                                                    \
        return hipGetLastError();
        PTK_X(3) PTK_X(4) PTK_X(5) PTK_X(8) PTK_X(10) PTK_X(16)
#undef PTK_X
    default:
        return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// S1, S2 per slice of entries
// ---------------------------------------------------------------------------
constexpr int kApproxChunk = kWave;   // entries staged per step

// Third-last-mode values per wavefront of the partial-error kernel: each
// lane then updates KG cells per staged entry from one pair of loads.
constexpr int kk_per_wave(int N, int J) { return (N - 1 >= 3 && J % 2 == 0) ? 2 : 1; }

template <int N, int J>
__global__ __launch_bounds__(kWave) void k_partial_error(ApproxArgs a) {
    constexpr int NP = N - 1;             // modes of T (all but g)
    constexpr int P = J * J;
    constexpr int NPG = (P + kWave - 1) / kWave;
    // values of the third-last other mode per wavefront (KG of them) and the
    // number of such groups
    constexpr int KG = kk_per_wave(N, J);
    constexpr int KS = NP >= 3 ? J / KG : 1;
    constexpr int NLG = NP >= 4 ? ipow(J, NP - 3) : 1;
    constexpr int CELLS = ipow(J, N);
    constexpr int CH = kApproxChunk;
    typedef double double2v __attribute__((ext_vector_type(2)));
    __shared__ double2v s_uw[CH][KG];     // (r q, q^2) per staged entry and kk
    __shared__ int32_t s_ia[CH], s_ib[CH], s_row[CH];
    __shared__ float s_va[CH * J], s_vb[CH * J];   // rows of the last two modes
    const int lane = threadIdx.x;
    int b = blockIdx.x;
    const int pg = b % NPG;
    b /= NPG;
    const int kk0 = (b % KS) * KG;        // first third-last value of this wave
    b /= KS;
    const int lg = b % NLG;
    const int sl = b / NLG;
    const int p = pg * kWave + lane;
    const bool act = p < P;
    const int m1 = act ? p / J : 0, m2 = act ? p % J : 0;
    int pre[NP > 3 ? NP - 3 : 1];
    {
        int t = lg;
#pragma unroll
        for (int k = NP - 4; k >= 0; --k) {
            pre[k] = t % J;
            t /= J;
        }
    }
    double S1[KG][J], S2[KG][J];
#pragma unroll
    for (int i = 0; i < KG; ++i)
#pragma unroll
        for (int k = 0; k < J; ++k) S1[i][k] = S2[i][k] = 0.0;
    double t1[KG], t2[KG];                // T1, T2 of the current row, this lane's cells
#pragma unroll
    for (int i = 0; i < KG; ++i) t1[i] = t2[i] = 0.0;
    int cur = -1;
    auto fold = [&](int row) {            // S += a^(g)_row (x) T_row
        cptr<float> ag = (cptr<float>)a.fac_g + (int64_t)row * J;
#pragma unroll
        for (int k = 0; k < J; ++k) {
            const double x = (double)ag[k];
#pragma unroll
            for (int i = 0; i < KG; ++i) {
                S1[i][k] = __builtin_fma(x, t1[i], S1[i][k]);
                S2[i][k] = __builtin_fma(x * x, t2[i], S2[i][k]);
            }
        }
    };
    const int64_t e0 = (int64_t)sl * a.slice;
    const int64_t e1 = min(e0 + a.slice, a.nnz);
    const float *fa = a.fac[NP - 2], *fb = a.fac[NP - 1];
    for (int64_t base = e0; base < e1; base += CH) {
        const int nb = (int)min((int64_t)CH, e1 - base);
        // stage: lane t takes entry base + t
        {
            const bool ok = lane < nb;
            const int64_t e = base + lane;
            double q0 = 0.0, r = 0.0;
            if (ok) {
                q0 = 1.0;
#pragma unroll
                for (int k = 0; k < NP - 3; ++k)
                    q0 *= (double)a.fac[k][(int64_t)a.idx[k][e] * J + pre[k]];
                r = a.resid[e];
            }
#pragma unroll
            for (int i = 0; i < KG; ++i) {
                double q = q0;
                if (NP >= 3 && ok)
                    q *= (double)a.fac[NP - 3][(int64_t)a.idx[NP - 3][e] * J + kk0 + i];
                s_uw[lane][i] = double2v{r * q, q * q};
            }
            s_ia[lane] = ok ? a.idx[NP - 2][e] : 0;
            s_ib[lane] = ok ? a.idx[NP - 1][e] : 0;
            s_row[lane] = ok ? a.rows[e] : -1;
        }
        __syncthreads();
        // the staged entries' rows of the last two other modes
        for (int t = lane; t < CH * J; t += kWave) {
            const int u = t / J, j = t % J;
            s_va[t] = fa[(int64_t)s_ia[u] * J + j];
            s_vb[t] = fb[(int64_t)s_ib[u] * J + j];
        }
        __syncthreads();
#pragma unroll 8
        for (int u = 0; u < CH; ++u) {
            if (u < nb) {                 // uniform
                const int row = s_row[u];
                if (row != cur) {         // uniform
                    if (cur >= 0) fold(cur);
                    cur = row;
#pragma unroll
                    for (int i = 0; i < KG; ++i) t1[i] = t2[i] = 0.0;
                }
                const double v = (double)s_va[u * J + m1] * (double)s_vb[u * J + m2];
                const double v2 = v * v;
#pragma unroll
                for (int i = 0; i < KG; ++i) {
                    const double2v uw = s_uw[u][i];
                    t1[i] = __builtin_fma(uw.x, v, t1[i]);
                    t2[i] = __builtin_fma(uw.y, v2, t2[i]);
                }
            }
        }
        __syncthreads();
    }
    if (cur >= 0) fold(cur);
    if (act) {
#pragma unroll
        for (int i = 0; i < KG; ++i) {
            // C-order cell of (beta_g = k, the other modes' digits)
            int64_t rest = 0;
            int t = 0;
#pragma unroll
            for (int mode = 0; mode < N; ++mode) {
                if (mode == a.g) continue;
                const int d = (t < NP - 3)    ? pre[t]
                              : (t == NP - 3) ? kk0 + i
                              : (t == NP - 2) ? m1
                                              : m2;
                rest = rest * J + d;
                ++t;
            }
            // insert beta_g at position g: cell = hi * J^(N-g) + beta_g * J^(N-1-g) + lo
            const int64_t sg = ipow_rt(J, N - 1 - a.g);
            const int64_t hi = rest / sg, lo = rest % sg;
            double *o1 = a.part + (int64_t)sl * 2 * CELLS;
            double *o2 = o1 + CELLS;
#pragma unroll
            for (int k = 0; k < J; ++k) {
                const int64_t cell = (hi * J + k) * sg + lo;
                o1[cell] = S1[i][k];
                o2[cell] = S2[i][k];
            }
        }
    }
}

int32_t approx_slices(const Shape &s, int64_t nnz, int num_cu) {
    const int J = s.ranks[0];
    const int NP = s.N - 1;
    int64_t waves_per_slice = (int64_t)((J * J + kWave - 1) / kWave);
    if (NP >= 3) waves_per_slice *= J / kk_per_wave(s.N, J);
    for (int k = 4; k <= NP; ++k) waves_per_slice *= J;
    // about 16 wavefronts per CU in all, slices of at least 256 entries
    int64_t sl = ((int64_t)16 * num_cu + waves_per_slice - 1) / waves_per_slice;
    sl = std::min<int64_t>(sl, (nnz + 255) / 256);
    return (int32_t)std::max<int64_t>(1, sl);
}

int64_t approx_part_doubles(const Shape &s, int32_t nslices) {
    int64_t cells = 1;
    for (int k = 0; k < s.N; ++k) cells *= s.ranks[k];
    return (int64_t)nslices * 2 * cells;
}

hipError_t launch_partial_error(const ApproxArgs &a, const Shape &s, hipStream_t st) {
    const int J = s.ranks[0];
#define PTK_X(n_, j_)                                                            \
    if (s.N == n_ && J == j_) {                                                  \
        const int64_t blocks = (int64_t)((j_ * j_ + kWave - 1) / kWave) *        \
                               (n_ - 1 >= 3 ? j_ / kk_per_wave(n_, j_) : 1) *   \
                               (n_ - 1 >= 4 ? ipow(j_, n_ - 4) : 1) * a.nslices; \
        hipLaunchKernelGGL((k_partial_error<n_, j_>), dim3((unsigned)blocks),     \
                           dim3(kWave), 0, st, a);                               \
        return hipGetLastError();                                                \
    }
    PTK_APPROX_SHAPES(PTK_X)
#undef PTK_X
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Row-sum form (orders 4 and 5): the same sums S1, S2 in three kernels.
//
// The cells beta' of T factor into (lead modes, third-last mode k, last two
// modes p). Every lane owns one p and all J values of k, so that per entry
// the 2J values r a[k] and a[k]^2 of the third-last mode's row are the same
// for the whole wavefront: they are read once per entry through the scalar
// cache (precomputed per entry by k_approx_uw) and each feeds one FMA per
// lane, as the core values do in the row-system kernels. The lane holds T1,
// T2 of its J cells for the current row; at the end of a row piece it
// stores them to that piece's slot, and k_row_fold then forms
// S(beta) = sum over slots a^(g)_{row, beta_g} T_slot(beta') per range of
// slots. Slots: slot i for the piece of row i that holds its first entry,
// slot rows + s for the first piece of slice s when its row began in an
// earlier slice.
// ---------------------------------------------------------------------------
template <int J>
__global__ void k_approx_uw(const double *__restrict__ resid, const float *__restrict__ fac3,
                            const int32_t *__restrict__ idx3, int64_t nnz,
                            double *__restrict__ uw) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (entry, k)
    if (t >= nnz * J) return;
    const int64_t e = t / J;
    const int k = (int)(t % J);
    const double a = (double)fac3[(int64_t)idx3[e] * J + k];
    uw[e * 2 * J + k] = resid[e] * a;
    uw[e * 2 * J + J + k] = a * a;
}

constexpr int kXcds = 8;                 // XCDs of the MI355X

// Pairs p of the last two other modes per lane of the row-sum kernel (two
// when J*J exceeds a wavefront: every weight read then feeds two FMAs per
// lane), and the wavefronts that cover the J*J pairs.
constexpr int rs_ppl(int J) { return J * J > kWave ? 2 : 1; }
constexpr int rs_groups(int J) { return (J * J + kWave * rs_ppl(J) - 1) / (kWave * rs_ppl(J)); }

template <int N, int J>
__global__ __launch_bounds__(kWave) void k_row_sums(RowSumArgs a) {
    constexpr int NP = N - 1;             // other modes, NP >= 3
    constexpr int P = J * J;
    constexpr int PPL = rs_ppl(J);
    constexpr int NPG = rs_groups(J);
    constexpr int NLG = ipow(J, NP - 3);
    constexpr int NT = ipow(J, NP);
    __shared__ float s_va[kWave * J], s_vb[kWave * J];
    __shared__ double s_q[kWave];
    __shared__ int32_t s_ia[kWave], s_ib[kWave], s_row[kWave];
    const int lane = threadIdx.x;
    // workgroups go to the 8 XCDs in turn (block b on XCD b % 8): the
    // wavefronts of one slice take blocks 8 apart, so that they share one
    // XCD's L2 for the slice's weights and factor rows (nslices % 8 == 0)
    const int x = blockIdx.x % kXcds;
    int b = blockIdx.x / kXcds;
    const int pg = b % NPG;
    b /= NPG;
    const int lg = b % NLG;
    const int sl = (b / NLG) * kXcds + x;
    const int64_t e0 = (int64_t)sl * a.slice;
    const int64_t e1 = min(e0 + a.slice, a.nnz);
    if (e0 >= e1) return;                 // uniform
    int p[PPL], m1[PPL], m2[PPL];
    bool act[PPL];
#pragma unroll
    for (int i = 0; i < PPL; ++i) {
        p[i] = (pg * PPL + i) * kWave + lane;
        act[i] = p[i] < P;
        m1[i] = act[i] ? p[i] / J : 0;
        m2[i] = act[i] ? p[i] % J : 0;
    }
    int pre[NP > 3 ? NP - 3 : 1];
    {
        int t = lg;
#pragma unroll
        for (int k = NP - 4; k >= 0; --k) {
            pre[k] = t % J;
            t /= J;
        }
    }
    double T1[PPL][J], T2[PPL][J];
#pragma unroll
    for (int i = 0; i < PPL; ++i)
#pragma unroll
        for (int k = 0; k < J; ++k) T1[i][k] = T2[i][k] = 0.0;
    // the lane's sums of the current row piece to its slot
    auto store = [&](int64_t sl_) {
#pragma unroll
        for (int i = 0; i < PPL; ++i) {
            if (!act[i]) continue;
            double *o = a.tbuf + sl_ * 2 * NT + (int64_t)lg * J * P + p[i];
#pragma unroll
            for (int k = 0; k < J; ++k) {
                o[k * P] = T1[i][k];
                o[NT + k * P] = T2[i][k];
            }
        }
    };
    int cur = -1, myrow = -1;
    int64_t slot = 0;
    const float *fa = a.fac[NP - 2], *fb = a.fac[NP - 1];
    // the weights of a tile are 8J lines of 128 bytes; the tile after the one
    // being staged is touched with vector loads so that its scalar loads hit
    // L2 instead of waiting on HBM (the values are folded into pf, which is
    // consumed by a store that never happens, nnz being >= 0)
    constexpr int kLines = 8 * J;
    const unsigned char *uw_bytes = (const unsigned char *)a.uw;
    const int64_t uw_end = a.nnz * 2 * J * 8;
    uint32_t pf = 0;
    for (int64_t base = e0; base < e1; base += kWave) {
        const int nb = (int)min((int64_t)kWave, e1 - base);
        for (int t = lane; t < kLines; t += kWave) {
            const int64_t off = (base + kWave) * 2 * J * 8 + (int64_t)t * 128;
            if (base + kWave < e1 && off < uw_end) pf += *(const uint32_t *)(uw_bytes + off);
        }
        {
            const bool ok = lane < nb;
            const int64_t e = base + lane;
            double q = 1.0;
            if (ok) {
#pragma unroll
                for (int k = 0; k < NP - 3; ++k)
                    q *= (double)a.fac[k][(int64_t)a.idx[k][e] * J + pre[k]];
            }
            s_q[lane] = q;
            s_ia[lane] = ok ? a.idx[NP - 2][e] : 0;
            s_ib[lane] = ok ? a.idx[NP - 1][e] : 0;
            myrow = ok ? a.rows[e] : -1;
            s_row[lane] = myrow;
        }
        __syncthreads();
        for (int t = lane; t < kWave * J; t += kWave) {
            const int u = t / J, j = t % J;
            s_va[t] = fa[(int64_t)s_ia[u] * J + j];
            s_vb[t] = fb[(int64_t)s_ib[u] * J + j];
        }
        // the tile's row changes as one scalar mask (bit u: entry u starts
        // a row piece), so the entry loop tests a bit instead of waiting on
        // an LDS read per entry
        const int prevrow = lane == 0 ? cur : s_row[lane > 0 ? lane - 1 : 0];
        const uint64_t change = __ballot(lane < nb && myrow != prevrow);
        __syncthreads();
        for (int u = 0; u < nb; ++u) {
            // the entry's weights first: all their scalar loads in flight
            // before the LDS reads, so that one wait covers both
            cptr<double> w = (cptr<double>)(a.uw + (base + u) * 2 * J);
            double wv[2 * J];
#pragma unroll
            for (int k = 0; k < 2 * J; ++k) wv[k] = w[k];
            if ((change >> u) & 1) {
                const int row = __builtin_amdgcn_readlane(myrow, u);
                if (cur >= 0) store(slot);
                cur = row;
                const int64_t e = base + u;
                slot = (e == e0 && e0 > 0 && a.rows[e0 - 1] == row) ? a.nrows + sl : row;
#pragma unroll
                for (int i = 0; i < PPL; ++i)
#pragma unroll
                    for (int k = 0; k < J; ++k) T1[i][k] = T2[i][k] = 0.0;
            }
            double v[PPL], v2[PPL];
#pragma unroll
            for (int i = 0; i < PPL; ++i) {
                v[i] = (double)s_va[u * J + m1[i]] * (double)s_vb[u * J + m2[i]];
                if constexpr (NP > 3) v[i] *= s_q[u];
                v2[i] = v[i] * v[i];
            }
#pragma unroll
            for (int k = 0; k < J; ++k)
#pragma unroll
                for (int i = 0; i < PPL; ++i) {
                    T1[i][k] = __builtin_fma(wv[k], v[i], T1[i][k]);
                    T2[i][k] = __builtin_fma(wv[J + k], v2[i], T2[i][k]);
                }
        }
        __syncthreads();
    }
    if (cur >= 0) store(slot);
    if (a.nnz < 0) a.tbuf[lane] = (double)pf;
}

// part[r][0..1][cell] = S1, S2 over the slots of range r (fixed order).
template <int N, int J>
__global__ __launch_bounds__(256) void k_row_fold(RowSumArgs a) {
    constexpr int NT = ipow(J, N - 1);
    constexpr int CELLS = NT * J;
    const int rest = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    const int64_t s0 = (int64_t)r * a.fold_per;
    const int64_t s1 = min(s0 + a.fold_per, a.nslots);
    double S1[J], S2[J];
#pragma unroll
    for (int k = 0; k < J; ++k) S1[k] = S2[k] = 0.0;
    if (rest < NT) {
        // slots never written (empty rows, slices that start a row) are read
        // but replaced by zero; no branch, so several slots' loads overlap
#pragma unroll 4
        for (int64_t q = s0; q < s1; ++q) {
            int64_t row = 0;
            bool valid;
            if (q < a.nrows) {
                row = q;
                valid = a.rowptr[row + 1] > a.rowptr[row];
            } else {
                const int64_t e = (q - a.nrows) * a.slice;
                valid = e > 0 && e < a.nnz && a.rows[e - 1] == a.rows[e];
                row = valid ? a.rows[e] : 0;
            }
            const double t1v = a.tbuf[q * 2 * NT + rest];
            const double t2v = a.tbuf[q * 2 * NT + NT + rest];
            const double t1 = valid ? t1v : 0.0, t2 = valid ? t2v : 0.0;
            cptr<float> ag = (cptr<float>)(a.fac_g + row * J);
#pragma unroll
            for (int k = 0; k < J; ++k) {
                const double x = (double)ag[k];
                S1[k] = __builtin_fma(x, t1, S1[k]);
                S2[k] = __builtin_fma(x * x, t2, S2[k]);
            }
        }
        // C-order cell of (beta_g = k, beta' = rest): beta_g inserted at mode g
        const int64_t sg = ipow_rt(J, N - 1 - a.g);
        const int64_t hi = rest / sg, lo = rest % sg;
        double *o1 = a.part + (int64_t)r * 2 * CELLS;
        double *o2 = o1 + CELLS;
#pragma unroll
        for (int k = 0; k < J; ++k) {
            const int64_t cell = (hi * J + k) * sg + lo;
            o1[cell] = S1[k];
            o2[cell] = S2[k];
        }
    }
}

// the Approx shapes of orders 4 and 5
#define PTK_ROWSUM_SHAPES(X) X(4, 3) X(4, 5) X(4, 8) X(4, 10) X(5, 3) X(5, 5) X(5, 8)

bool row_sums_available(int N, int J) {
#define PTK_X(n_, j_) if (N == n_ && J == j_) return true;
    PTK_ROWSUM_SHAPES(PTK_X)
#undef PTK_X
    return false;
}

int64_t row_sums_slices(const Shape &s, int64_t nnz, int num_cu) {
    const int J = s.ranks[0];
    int64_t waves_per_slice = rs_groups(J);
    for (int k = 4; k <= s.N - 1; ++k) waves_per_slice *= J;
    // about 16 wavefronts per CU in all, slices of at least 256 entries
    int64_t sl = ((int64_t)16 * num_cu + waves_per_slice - 1) / waves_per_slice;
    sl = std::min<int64_t>(sl, (nnz + 255) / 256);
    sl = std::max<int64_t>(1, sl);
    return (sl + kXcds - 1) / kXcds * kXcds;     // whole rounds of the XCDs
}

int64_t row_sums_tbuf_doubles(const Shape &s, int g, int64_t nslices) {
    return (s.dims[g] + nslices) * 2 * ipow_rt(s.ranks[0], s.N - 1);
}

hipError_t launch_row_sums(const RowSumArgs &a, const Shape &s, hipStream_t st) {
    const int J = s.ranks[0];
#define PTK_X(n_, j_)                                                                   \
    if (s.N == n_ && J == j_) {                                                         \
        if (a.nnz > 0) {                                                                \
            hipError_t e = hipSuccess;                                                  \
            if (!a.uw_ready) {                                                          \
                const int64_t t = a.nnz * j_;                                           \
                hipLaunchKernelGGL((k_approx_uw<j_>), dim3((unsigned)((t + 255) / 256)), \
                                   dim3(256), 0, st, a.resid, a.fac[n_ - 4],            \
                                   a.idx[n_ - 4], a.nnz, a.uw);                         \
                if ((e = hipGetLastError()) != hipSuccess) return e;                    \
            }                                                                           \
            const int64_t blocks = (int64_t)rs_groups(j_) * ipow(j_, n_ - 4) * a.nslices; \
            hipLaunchKernelGGL((k_row_sums<n_, j_>), dim3((unsigned)blocks), dim3(kWave), \
                               0, st, a);                                               \
            if ((e = hipGetLastError()) != hipSuccess) return e;                        \
        }                                                                               \
        const int nt = ipow(j_, n_ - 1);                                                \
        hipLaunchKernelGGL((k_row_fold<n_, j_>),                                        \
                           dim3((unsigned)((nt + 255) / 256), (unsigned)a.nfold),       \
                           dim3(256), 0, st, a);                                        \
        return hipGetLastError();                                                       \
    }
    PTK_ROWSUM_SHAPES(PTK_X)
#undef PTK_X
    return hipErrorInvalidValue;
}

// R(beta) = 2 G S1 - G^2 S2, slices summed in order; 0 (positive) for cells
// that are not entries of the core.
__global__ void k_partial_reduce(const double *__restrict__ part, int32_t nslices,
                                 const float *__restrict__ G, int64_t cells,
                                 double *__restrict__ R) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells) return;
    double s1 = 0.0, s2 = 0.0;
    for (int32_t sl = 0; sl < nslices; ++sl) {
        s1 += part[((int64_t)sl * 2) * cells + c];
        s2 += part[((int64_t)sl * 2 + 1) * cells + c];
    }
    const double g = (double)G[c];
    const double r = g == 0.0 ? 0.0 : 2.0 * g * s1 - g * g * s2;
    R[c] = r + 0.0;                    // -0 -> +0
}

hipError_t launch_partial_reduce(const double *part, int32_t nslices, const float *G,
                                 int64_t cells, double *R, hipStream_t st) {
    hipLaunchKernelGGL(k_partial_reduce, dim3((unsigned)((cells + 255) / 256)), dim3(256),
                       0, st, part, nslices, G, cells, R);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// removal: one workgroup, radix select of the k-th largest R
// ---------------------------------------------------------------------------
// Order-preserving key of a double (larger value -> larger key).
__device__ __forceinline__ unsigned long long order_key(double v) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    return (u >> 63) ? ~u : (u | (1ull << 63));
}

constexpr int kSelThreads = 1024;

__global__ __launch_bounds__(kSelThreads) void k_approx_select(
    const double *__restrict__ R, float *__restrict__ G, int64_t cells, double p,
    int32_t *__restrict__ removed) {
    __shared__ int hist[256];
    __shared__ int s_wcnt[kSelThreads / kWave], s_woff[kSelThreads / kWave];
    __shared__ unsigned long long s_nz;
    __shared__ int s_digit;
    __shared__ long long s_rem;
    const int tid = threadIdx.x;
    if (tid == 0) s_nz = 0;
    __syncthreads();
    unsigned long long mine = 0;
    for (int64_t c = tid; c < cells; c += kSelThreads) mine += G[c] != 0.0f;
    atomicAdd(&s_nz, mine);
    __syncthreads();
    const long long k = (long long)floor(p * (double)s_nz);
    if (k <= 0) {
        if (tid == 0) *removed = 0;
        return;
    }
    // MSB-first radix select over 8 digits: prefix = key of the k-th largest
    unsigned long long prefix = 0, mask = 0;
    long long remaining = k;
    for (int pos = 7; pos >= 0; --pos) {
        for (int d = tid; d < 256; d += kSelThreads) hist[d] = 0;
        __syncthreads();
        for (int64_t c = tid; c < cells; c += kSelThreads) {
            if (G[c] == 0.0f) continue;
            const unsigned long long key = order_key(R[c]);
            if ((key & mask) == prefix) atomicAdd(&hist[(key >> (8 * pos)) & 255], 1);
        }
        __syncthreads();
        if (tid == 0) {
            long long cum = 0;
            int d = 255;
            for (; d > 0; --d) {
                if (cum + hist[d] >= remaining) break;
                cum += hist[d];
            }
            s_digit = d;
            s_rem = remaining - cum;
        }
        __syncthreads();
        prefix |= (unsigned long long)s_digit << (8 * pos);
        mask |= 0xFFull << (8 * pos);
        remaining = s_rem;
        __syncthreads();
    }
    // keys above the threshold go; of the keys equal to it, the first
    // `remaining` in cell order
    const int wid = tid / kWave, lid = tid % kWave;
    long long running = 0;
    for (int64_t base = 0; base < cells; base += kSelThreads) {
        const int64_t c = base + tid;
        bool gt = false, eq = false;
        if (c < cells && G[c] != 0.0f) {
            const unsigned long long key = order_key(R[c]);
            gt = key > prefix;
            eq = key == prefix;
        }
        const unsigned long long bal = __ballot(eq);
        const int below = __popcll(bal & ((1ull << lid) - 1ull));
        if (lid == 0) s_wcnt[wid] = __popcll(bal);
        __syncthreads();
        if (tid == 0) {
            int acc = 0;
            for (int w = 0; w < kSelThreads / kWave; ++w) {
                s_woff[w] = acc;
                acc += s_wcnt[w];
            }
        }
        __syncthreads();
        const long long rank = running + s_woff[wid] + below;
        if (gt || (eq && rank < remaining)) G[c] = 0.0f;
        running += s_woff[kSelThreads / kWave - 1] + s_wcnt[kSelThreads / kWave - 1];
        __syncthreads();
    }
    if (tid == 0) *removed = (int32_t)k;
}

hipError_t launch_approx_select(const double *R, float *G, int64_t cells, double p,
                                int32_t *removed, hipStream_t st) {
    hipLaunchKernelGGL(k_approx_select, dim3(1), dim3(kSelThreads), 0, st, R, G, cells,
                       p, removed);
    return hipGetLastError();
}

}  // namespace ptk
