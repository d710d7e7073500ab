// Row solves of the row-wise ALS (Sec. 3.2, eq. "rowupdate"), FP64.
//
// a_i = c_i (B_i + lambda I)^{-1} is computed as the solution of the
// symmetric positive definite system (B_i + lambda I) a_i^T = c_i^T by a
// Cholesky factorisation and two triangular solves (Golub & Van Loan,
// Alg. 4.2.1) instead of the explicit inverse of Alg. 3.
//
// Accuracy check. With M = B_i + lambda I and D = diag(M), the forward error
// of the Cholesky solve grows with the condition of the scaled matrix
// S = D^-1/2 M D^-1/2. Each kernel computes tr(S^-1) = sum_k M_kk (M^-1)_kk
// from the factor, (M^-1)_kk = ||L^-1 e_k||^2 (about J^3/6 more multiply-adds
// per row); cond(S) lies within a factor J of it either way. A row whose
// factorisation breaks down, or whose tr(S^-1) exceeds the limit, is not
// written: it is flagged (rflag[i] = 1) for the least-squares solve of
// ptk_resolve.hip, which works from the entries and needs no formed B_i.
#include "ptk_internal.h"

namespace ptk {

// Merge the partial systems of rows that cross work-range boundaries:
// split[3*s + {0,1,2}] = (row, first range, last range). The first range
// holds the row's head in its tail slot, every later range its head slot.
// A block of 1024 threads serves one row: 64 entries of the packed system at
// a time, the ranges dealt round-robin to 16 groups whose sums are combined in
// a fixed order (deterministic for any range count). The loop is unrolled by
// 16 so that a long row (thousands of ranges) keeps 16 loads in flight per
// lane.
constexpr int kMergeGroups = 16;

__global__ __launch_bounds__(kWave * kMergeGroups) void k_merge(
    const double *__restrict__ part, const int32_t *__restrict__ split, int E,
    double *__restrict__ bbuf) {
    __shared__ double s_acc[kMergeGroups][kWave];
    const int s = blockIdx.x;
    const int row = split[3 * s + 0];
    const int c0 = split[3 * s + 1];
    const int c1 = split[3 * s + 2];
    const int lane = threadIdx.x % kWave;
    const int grp = threadIdx.x / kWave;
    for (int e0 = 0; e0 < E; e0 += kWave) {
        const int e = e0 + lane;
        double acc = 0.0;
        if (e < E) {
            if (grp == 0) acc = part[((int64_t)c0 * 2 + 1) * E + e];
#pragma unroll 16
            for (int c = c0 + 1 + grp; c <= c1; c += kMergeGroups)
                acc += part[((int64_t)c * 2 + 0) * E + e];
        }
        s_acc[grp][lane] = acc;
        __syncthreads();
        if (grp == 0 && e < E) {
            double t = s_acc[0][lane];
#pragma unroll
            for (int q = 1; q < kMergeGroups; ++q) t += s_acc[q][lane];
            bbuf[(int64_t)row * E + e] = t;
        }
        __syncthreads();
    }
}

hipError_t launch_merge(const double *part, const int32_t *split, int32_t nsplit,
                        int E, double *bbuf, hipStream_t st) {
    if (nsplit <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_merge, dim3(nsplit), dim3(kWave * kMergeGroups), 0, st, part,
                       split, E, bbuf);
    return hipGetLastError();
}

// Packed Cholesky in place: L(i, j), j <= i, overwrites B(j, i). One thread
// per row; the packed system and a J-vector of work space live in LDS, one
// column per thread.
__global__ void k_solve(const double *__restrict__ bbuf,
                        const int64_t *__restrict__ rowptr, int64_t I, int J,
                        double lambda, float *__restrict__ A, SolveFlags f) {
    extern __shared__ double s_sys[];
    const int bs = blockDim.x;
    const int64_t i = (int64_t)blockIdx.x * bs + threadIdx.x;
    if (i >= I) return;
    float *arow = A + i * J;
    const int64_t cnt = rowptr[i + 1] - rowptr[i];
    if (cnt == 0) {                        // no entry: B = 0, c = 0 -> a = 0
        for (int p = 0; p < J; ++p) arow[p] = 0.0f;
        f.rflag[i] = 0;
        return;
    }
    const int T = J * (J + 1) / 2;
    const int E = T + J;
    double *m = s_sys + threadIdx.x;       // entry k at m[k * bs]
    const double *src = bbuf + i * E;
    for (int k = 0; k < E; ++k) m[k * bs] = src[k];
    for (int p = 0; p < J; ++p) m[tri_pos(p, p, J) * bs] += lambda;

    bool ok = true;
    for (int r = 0; r < J && ok; ++r) {
        for (int c = 0; c <= r; ++c) {
            double s = m[tri_pos(c, r, J) * bs];
            for (int k = 0; k < c; ++k)
                s -= m[tri_pos(k, r, J) * bs] * m[tri_pos(k, c, J) * bs];
            if (c == r) {
                if (!(s > 0.0)) {
                    ok = false;
                    break;
                }
                m[tri_pos(r, r, J) * bs] = sqrt(s);
            } else {
                m[tri_pos(c, r, J) * bs] = s / m[tri_pos(c, c, J) * bs];
            }
        }
    }
    // tr(S^-1) = sum_k M_kk ||L^-1 e_k||^2, M_kk = sum_{q <= k} L_kq^2
    double tr = 0.0;
    if (ok) {
        double *y = m + (size_t)E * bs;    // work space, J entries
        for (int k = 0; k < J; ++k) {
            double mkk = 0.0;
            for (int q = 0; q <= k; ++q) {
                const double l = m[tri_pos(q, k, J) * bs];
                mkk += l * l;
            }
            y[k * bs] = 1.0 / m[tri_pos(k, k, J) * bs];
            double ss = y[k * bs] * y[k * bs];
            for (int r = k + 1; r < J; ++r) {
                double t = 0.0;
                for (int q = k; q < r; ++q) t += m[tri_pos(q, r, J) * bs] * y[q * bs];
                y[r * bs] = -t / m[tri_pos(r, r, J) * bs];
                ss += y[r * bs] * y[r * bs];
            }
            tr += mkk * ss;
        }
    }
    const bool flag = !ok || !(tr <= f.cond_limit);
    f.rflag[i] = flag;
    if (flag) return;
    double *y = m + T * bs;                // rhs c, overwritten by y then a
    for (int r = 0; r < J; ++r) {          // L y = c
        double s = y[r * bs];
        for (int k = 0; k < r; ++k) s -= m[tri_pos(k, r, J) * bs] * y[k * bs];
        y[r * bs] = s / m[tri_pos(r, r, J) * bs];
    }
    for (int r = J - 1; r >= 0; --r) {     // L^T a = y
        double s = y[r * bs];
        for (int k = r + 1; k < J; ++k) s -= m[tri_pos(r, k, J) * bs] * y[k * bs];
        y[r * bs] = s / m[tri_pos(r, r, J) * bs];
    }
    for (int p = 0; p < J; ++p) arow[p] = (float)y[p * bs];
}

// The same solve with a group of G lanes per row (G = 4, 8 or 16 >= J,
// 64/G rows per wavefront): lane l keeps row l of B + lambda I in registers.
// Cholesky column by column (the diagonal and the new column are broadcast
// within the group, 1 / L_kk kept in every lane), then L y = c with each y_r
// broadcast, then L^T a = y with a group reduction per step. For the
// condition estimate lane l forms column l of L^-1 (the rows of L broadcast
// from their lanes). FP64; same flagging and empty-row rule as k_solve.
template <int J>
__global__ __launch_bounds__(256) void k_solve_grp(const double *__restrict__ bbuf,
                                                   const int64_t *__restrict__ rowptr,
                                                   int64_t I, double lambda,
                                                   float *__restrict__ A, SolveFlags f) {
    constexpr int G = J <= 4 ? 4 : (J <= 8 ? 8 : 16);
    constexpr int T = J * (J + 1) / 2;
    constexpr int E = T + J;
    const int l = threadIdx.x % G;
    const int64_t i = (int64_t)blockIdx.x * (blockDim.x / G) + threadIdx.x / G;
    const bool have = i < I;
    const int64_t cnt = have ? rowptr[i + 1] - rowptr[i] : 0;
    const bool empty = have && cnt == 0;
    const bool live = have && !empty;          // uniform within the group
    if (!live) {
        // nothing to solve; the group leaves together, so no shuffle below
        // reads its lanes
        if (empty && l < J) A[i * J + l] = 0.0f;   // no entry: B = 0, c = 0 -> a = 0
        if (empty && l == 0) f.rflag[i] = 0;
        return;
    }
    double b[J];
    double c = 0.0;
#pragma unroll
    for (int k = 0; k < J; ++k) b[k] = 0.0;
    if (l < J) {
        const double *sys = bbuf + i * E;
#pragma unroll
        for (int k = 0; k < J; ++k)
            b[k] = sys[l <= k ? tri_pos(l, k, J) : tri_pos(k, l, J)];
        c = sys[T + l];
#pragma unroll
        for (int k = 0; k < J; ++k)
            if (k == l) b[k] += lambda;
    }
    bool ok = true;
    double rinv[J];                            // 1 / L_kk, the same in every lane
#pragma unroll
    for (int k = 0; k < J; ++k) {
        const double d = __shfl(b[k], k, G);   // updated B_kk
        ok = ok && d > 0.0;
        const double lkk = sqrt(d > 0.0 ? d : 1.0);
        rinv[k] = 1.0 / lkk;
        const double mine = (l == k) ? lkk : b[k] * rinv[k];   // L_lk (l >= k)
        b[k] = mine;
#pragma unroll
        for (int j = k + 1; j < J; ++j) {
            const double ljk = __shfl(mine, j, G);
            if (l > k) b[j] = __builtin_fma(-mine, ljk, b[j]);
        }
    }
    // tr(S^-1): lane l solves L y = e_l (y_r = 0 for r < l) and adds
    // M_ll ||y||^2, M_ll = sum_{q <= l} L_lq^2
    double ss = 0.0, mll = 0.0;
    {
        double y[J];
#pragma unroll
        for (int r = 0; r < J; ++r) {
            double t = 0.0;
#pragma unroll
            for (int q = 0; q < r; ++q) t = __builtin_fma(__shfl(b[q], r, G), y[q], t);
            y[r] = (r < l) ? 0.0 : (r == l ? rinv[r] : -t * rinv[r]);
            ss = __builtin_fma(y[r], y[r], ss);
        }
#pragma unroll
        for (int q = 0; q < J; ++q)
            if (q <= l) mll = __builtin_fma(b[q], b[q], mll);
    }
    double tr = (l < J) ? mll * ss : 0.0;
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) tr += __shfl_xor(tr, off, G);
    // L y = c
    double y = c;
#pragma unroll
    for (int r = 0; r < J; ++r) {
        const double yr = __shfl(y, r, G) * rinv[r];
        if (l == r) y = yr;
        if (l > r) y = __builtin_fma(-b[r], yr, y);
    }
    // L^T a = y, a_r = (y_r - sum_{k > r} L_kr a_k) / L_rr
    double a = 0.0;
#pragma unroll
    for (int r = J - 1; r >= 0; --r) {
        double t = (l > r && l < J) ? b[r] * a : 0.0;
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) t += __shfl_xor(t, off, G);
        const double ar = (__shfl(y, r, G) - t) * rinv[r];
        if (l == r) a = ar;
    }
    const bool flag = !ok || !(tr <= f.cond_limit);      // uniform within the group
    if (l == 0) f.rflag[i] = flag;
    if (!flag && l < J) A[i * J + l] = (float)a;
}

// One row per lane for J <= 11: the packed system (J(J+1)/2 + J doubles)
// lives in the lane's registers, with every index known at compile time, so
// the factorisation, the condition estimate and both substitutions are plain
// FMA chains with no exchange between lanes; 64 rows per wavefront run side by
// side. The upper triangle is overwritten by L^T (Cholesky, right-looking; the
// diagonal keeps the pivots L_kk^2); same results, flagging and empty-row
// rule as k_solve.
template <int J>
__global__ __launch_bounds__(kWave) void k_solve_row(const double *__restrict__ bbuf,
                                                     const int64_t *__restrict__ rowptr,
                                                     int64_t I, double lambda,
                                                     float *__restrict__ A, SolveFlags f) {
    constexpr int T = J * (J + 1) / 2;
    constexpr int E = T + J;
    const int64_t i = (int64_t)blockIdx.x * kWave + threadIdx.x;
    if (i >= I) return;
    float *arow = A + i * J;
    const int64_t cnt = rowptr[i + 1] - rowptr[i];
    if (cnt == 0) {                            // no entry: B = 0, c = 0 -> a = 0
#pragma unroll
        for (int k = 0; k < J; ++k) arow[k] = 0.0f;
        f.rflag[i] = 0;
        return;
    }
    const double *sys = bbuf + i * E;
    double m[T], y[J];
#pragma unroll
    for (int t = 0; t < T; ++t) m[t] = sys[t];
#pragma unroll
    for (int k = 0; k < J; ++k) y[k] = sys[T + k];
#pragma unroll
    for (int k = 0; k < J; ++k) m[tri_pos(k, k, J)] += lambda;
    bool ok = true;
    double rinv[J];
#pragma unroll
    for (int k = 0; k < J; ++k) {
        const double d = m[tri_pos(k, k, J)];
        ok = ok && d > 0.0;
        const double lkk = sqrt(d > 0.0 ? d : 1.0);
        rinv[k] = 1.0 / lkk;
#pragma unroll
        for (int j = k + 1; j < J; ++j) m[tri_pos(k, j, J)] *= rinv[k];   // L_jk
#pragma unroll
        for (int j = k + 1; j < J; ++j) {
#pragma unroll
            for (int q = j; q < J; ++q)
                m[tri_pos(j, q, J)] =
                    __builtin_fma(-m[tri_pos(k, j, J)], m[tri_pos(k, q, J)], m[tri_pos(j, q, J)]);
        }
    }
    // tr(S^-1) = sum_k M_kk ||L^-1 e_k||^2 with M_kk = L_kk^2 + sum_{q<k} L_kq^2
    double tr = 0.0;
#pragma unroll
    for (int k = 0; k < J; ++k) {
        double mkk = m[tri_pos(k, k, J)];
#pragma unroll
        for (int q = 0; q < k; ++q)
            mkk = __builtin_fma(m[tri_pos(q, k, J)], m[tri_pos(q, k, J)], mkk);
        double z[J];
        z[k] = rinv[k];
        double ss = z[k] * z[k];
#pragma unroll
        for (int r = k + 1; r < J; ++r) {
            double t = 0.0;
#pragma unroll
            for (int q = k; q < r; ++q) t = __builtin_fma(m[tri_pos(q, r, J)], z[q], t);
            z[r] = -t * rinv[r];
            ss = __builtin_fma(z[r], z[r], ss);
        }
        tr = __builtin_fma(mkk, ss, tr);
    }
    const bool flag = !ok || !(tr <= f.cond_limit);
    f.rflag[i] = flag;
    if (flag) return;
    // L y = c, then L^T a = y (L_rk at (k, r) of the upper triangle)
#pragma unroll
    for (int r = 0; r < J; ++r) {
#pragma unroll
        for (int k = 0; k < r; ++k) y[r] = __builtin_fma(-m[tri_pos(k, r, J)], y[k], y[r]);
        y[r] *= rinv[r];
    }
#pragma unroll
    for (int r = J - 1; r >= 0; --r) {
#pragma unroll
        for (int k = r + 1; k < J; ++k) y[r] = __builtin_fma(-m[tri_pos(r, k, J)], y[k], y[r]);
        y[r] *= rinv[r];
    }
#pragma unroll
    for (int k = 0; k < J; ++k) arow[k] = (float)y[k];
}

hipError_t launch_solve(const double *bbuf, const int64_t *rowptr, int64_t I,
                        int J, double lambda, float *A, const SolveFlags &f,
                        hipStream_t st) {
    if (I <= 0) return hipSuccess;
#define PTK_SOLVE_ROW(j_)                                                           \
    if (J == j_) {                                                                  \
        hipLaunchKernelGGL(k_solve_row<j_>, dim3((unsigned)((I + kWave - 1) / kWave)), \
                           dim3(kWave), 0, st, bbuf, rowptr, I, lambda, A, f);      \
        return hipGetLastError();                                                   \
    }
    PTK_SOLVE_ROW(3) PTK_SOLVE_ROW(4) PTK_SOLVE_ROW(5) PTK_SOLVE_ROW(7) PTK_SOLVE_ROW(8)
    PTK_SOLVE_ROW(9) PTK_SOLVE_ROW(10) PTK_SOLVE_ROW(11)
#undef PTK_SOLVE_ROW
#define PTK_SOLVE_GRP(j_)                                                           \
    if (J == j_) {                                                                  \
        constexpr int G = j_ <= 4 ? 4 : (j_ <= 8 ? 8 : 16);                         \
        const int64_t rows_per_block = 256 / G;                                     \
        hipLaunchKernelGGL(k_solve_grp<j_>,                                         \
                           dim3((unsigned)((I + rows_per_block - 1) / rows_per_block)), \
                           dim3(256), 0, st, bbuf, rowptr, I, lambda, A, f);        \
        return hipGetLastError();                                                   \
    }
    PTK_SOLVE_GRP(16)
#undef PTK_SOLVE_GRP
    const int E = sys_entries(J) + J;       // the system and a work vector
    int bs = 64;
    while (bs > 8 && (size_t)E * bs * 8 > 64 * 1024) bs /= 2;
    const size_t lds = (size_t)E * bs * 8;
    hipLaunchKernelGGL(k_solve, dim3((unsigned)((I + bs - 1) / bs)), dim3(bs), lds,
                       st, bbuf, rowptr, I, J, lambda, A, f);
    return hipGetLastError();
}

// Error of the last mode's update from its row systems: for the entries of
// row i, sum (x - a_i^T delta)^2 = sum x^2 - 2 a_i^T c_i + a_i^T B_i a_i, so
// the squared error of eq. "reconfull" after the sweep is
//     sum_Omega x^2 + sum_i (a_i^T B_i a_i - 2 a_i^T c_i)
// with a_i the stored (float32) row. A row solved by the least-squares path
// with its own error term (rflag[i] == kLsOwnError) adds rsse[i] instead:
// the same term, summed from its entries' deltas. (Heavy flagged rows keep the identity, evaluated with
// their accurate a_i.) Per-block partial sums, FP64.
__global__ __launch_bounds__(256) void k_row_sse(const double *__restrict__ bbuf,
                                                 const int64_t *__restrict__ rowptr,
                                                 const float *__restrict__ A,
                                                 int64_t I, int J,
                                                 const uint8_t *__restrict__ rflag,
                                                 const double *__restrict__ rsse,
                                                 double *__restrict__ partial) {
    __shared__ double s_part[256 / kWave];
    const int T = J * (J + 1) / 2;
    const int E = T + J;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < I;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (rowptr[i] == rowptr[i + 1]) continue;
        if (rflag && rflag[i] == kLsOwnError) {
            acc += rsse[i];
            continue;
        }
        const double *sys = bbuf + i * E;
        const float *a = A + i * J;
        double q = 0.0;
        for (int p = 0; p < J; ++p) {
            const double ap = (double)a[p];
            double r = 0.0;
            for (int qq = p + 1; qq < J; ++qq)
                r = __builtin_fma(sys[tri_pos(p, qq, J)], (double)a[qq], r);
            q += ap * (sys[tri_pos(p, p, J)] * ap + 2.0 * r - 2.0 * sys[T + p]);
        }
        acc += q;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, kWave);
    if ((threadIdx.x % kWave) == 0) s_part[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0)
        partial[blockIdx.x] = (s_part[0] + s_part[1]) + (s_part[2] + s_part[3]);
}

// The same sum with a group of lanes per row (the grouping of k_solve_grp):
// lane l takes row l of B_i and c_i, and adds a_l (B_i a)_l - 2 a_l c_l.
template <int J>
__global__ __launch_bounds__(256) void k_row_sse_grp(const double *__restrict__ bbuf,
                                                     const int64_t *__restrict__ rowptr,
                                                     const float *__restrict__ A,
                                                     int64_t I,
                                                     const uint8_t *__restrict__ rflag,
                                                     const double *__restrict__ rsse,
                                                     double *__restrict__ partial) {
    constexpr int G = J <= 4 ? 4 : (J <= 8 ? 8 : 16);
    constexpr int T = J * (J + 1) / 2;
    constexpr int E = T + J;
    __shared__ double s_part[256 / kWave];
    const int l = threadIdx.x % G;
    const int64_t stride = (int64_t)gridDim.x * (256 / G);
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * (256 / G) + threadIdx.x / G; i < I; i += stride) {
        if (l >= J || rowptr[i] == rowptr[i + 1]) continue;
        if (rflag && rflag[i] == kLsOwnError) {
            if (l == 0) acc += rsse[i];
            continue;
        }
        const double *sys = bbuf + i * E;
        const float *a = A + i * J;
        double r = 0.0;
#pragma unroll
        for (int k = 0; k < J; ++k)
            r = __builtin_fma(sys[l <= k ? tri_pos(l, k, J) : tri_pos(k, l, J)],
                              (double)a[k], r);
        acc += (double)a[l] * (r - 2.0 * sys[T + l]);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, kWave);
    if ((threadIdx.x % kWave) == 0) s_part[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0)
        partial[blockIdx.x] = (s_part[0] + s_part[1]) + (s_part[2] + s_part[3]);
}

hipError_t launch_row_sse(const double *bbuf, const int64_t *rowptr, const float *A,
                          int64_t I, int J, const uint8_t *rflag, const double *rsse,
                          double *partial, int nblocks, hipStream_t st) {
#define PTK_SSE_GRP(j_)                                                                  \
    if (J == j_) {                                                                       \
        hipLaunchKernelGGL(k_row_sse_grp<j_>, dim3(nblocks), dim3(256), 0, st, bbuf, rowptr, \
                           A, I, rflag, rsse, partial);                                  \
        return hipGetLastError();                                                        \
    }
    PTK_SSE_GRP(3) PTK_SSE_GRP(4) PTK_SSE_GRP(5) PTK_SSE_GRP(7) PTK_SSE_GRP(8)
    PTK_SSE_GRP(9) PTK_SSE_GRP(10) PTK_SSE_GRP(11) PTK_SSE_GRP(16)
#undef PTK_SSE_GRP
    hipLaunchKernelGGL(k_row_sse, dim3(nblocks), dim3(256), 0, st, bbuf, rowptr, A, I, J,
                       rflag, rsse, partial);
    return hipGetLastError();
}

}  // namespace ptk
