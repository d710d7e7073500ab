// Least-squares row solves for the rows that the Cholesky kernels hand over
// (Sec. 3.2, eq. "rowupdate", Theorem 1), FP64.
//
// eq. "rowupdate" is the normal-equation form of the row's regularised least
// squares problem
//     min_a  sum_alpha (x_alpha - a^T delta_alpha)^2 + lambda ||a||^2,
// i.e. of the stacked system [sqrt(lambda) I ; Delta] a ~ [0 ; x]. Forming
// B_i = Delta^T Delta squares the conditioning: once ||B_i|| * 2^-52 is near
// lambda the FP64 factorisation of B_i + lambda I is wrong or breaks down,
// although the minimiser is unique and well defined. The solve kernels flag
// such rows (breakdown, or a large scaled condition estimate); this kernel
// solves them from the entries instead: it recomputes every entry's delta in
// FP64 and builds the QR factorisation of the stacked system with Householder
// reflections (Golub & Van Loan, Sec. 5.2), 64 entries at a time, then
// back-substitutes. |R_jj| never falls below sqrt(lambda), so every row is
// solved.
//
// Layout of the triangle: lane q of a wavefront holds column q of [R | z]
// (column jn is z) in registers; lane l holds the delta row and value of one
// entry of the chunk. Each reflection needs one wavefront sum per column.
//
// Light rows (at most kLsLight entries) take one wavefront each; heavy rows
// take all W wavefronts of a workgroup, each reducing every W-th chunk into
// its own triangle, merged in wavefront order (the rows of a triangle are fed
// to the next one as entries). Results do not depend on the order in which
// rows were flagged.
#include "ptk_device.h"

namespace ptk {

namespace {

// Sum over the wavefront; the butterfly gives every lane the same bits.
__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Reflect one chunk of rows [d | x] (one per lane, zero rows allowed) into
// the triangle rc (column-distributed, see above).
template <int JMAX>
__device__ __forceinline__ void ls_merge(double (&rc)[JMAX], double (&d)[JMAX], double &x,
                                         int jn, int lane) {
#pragma unroll
    for (int j = 0; j < JMAX; ++j) {
        if (j >= jn) break;
        const double dj = d[j];
        const double sig = wsum(dj * dj);
        if (sig == 0.0) continue;              // nothing to annihilate in column j
        const double alpha = __shfl(rc[j], j, kWave);
        const double mu = sqrt(alpha * alpha + sig);
        const double beta = alpha >= 0.0 ? -mu : mu;
        const double v0 = alpha - beta;        // |alpha| + mu: no cancellation
        const double vtv = v0 * v0 + sig;
#pragma unroll
        for (int q = j + 1; q < JMAX; ++q) {
            if (q >= jn) break;
            const double s = wsum(dj * d[q]);
            const double rjq = __shfl(rc[j], q, kWave);
            const double f = 2.0 * (v0 * rjq + s) / vtv;
            if (lane == q) rc[j] = rjq - f * v0;
            d[q] = __builtin_fma(-f, dj, d[q]);
        }
        {
            const double s = wsum(dj * x);
            const double rjz = __shfl(rc[j], jn, kWave);
            const double f = 2.0 * (v0 * rjz + s) / vtv;
            if (lane == jn) rc[j] = rjz - f * v0;
            x = __builtin_fma(-f, dj, x);
        }
        if (lane == j) rc[j] = beta;
        d[j] = 0.0;
    }
}

// R a = z; lane q < jn returns a_q.
template <int JMAX>
__device__ __forceinline__ double ls_back(const double (&rc)[JMAX], int jn, int lane) {
    double aq = 0.0;
#pragma unroll
    for (int j = JMAX - 1; j >= 0; --j) {
        if (j >= jn) continue;
        const double t = wsum((lane > j && lane < jn) ? rc[j] * aq : 0.0);
        const double zj = __shfl(rc[j], jn, kWave);
        const double rjj = __shfl(rc[j], j, kWave);
        const double aj = (zj - t) / rjj;
        if (lane == j) aq = aj;
    }
    return aq;
}

// delta (FP64) and value of entry pos of the row, or zeros past its end.
template <int JMAX>
__device__ __forceinline__ void chunk_rows(const ResolveArgs &a, int64_t pos, int64_t end,
                                           float *arow, int lane, double (&d)[JMAX],
                                           double &x) {
    const bool valid = pos < end;
    load_rows_generic<JMAX>(a, pos, valid, arow, lane);   // lane-private LDS
    delta_generic<JMAX>(a, arow, lane, d);
#pragma unroll
    for (int j = 0; j < JMAX; ++j)
        if (!valid || j >= a.jn) d[j] = 0.0;
    x = valid ? (double)a.val[pos] : 0.0;
}

// Initial triangle of one wavefront: sqrt(lambda) I (or 0 for the helpers of
// a heavy row), z = 0.
template <int JMAX>
__device__ __forceinline__ void ls_init(double (&rc)[JMAX], double diag, int jn, int lane) {
#pragma unroll
    for (int p = 0; p < JMAX; ++p) rc[p] = (p == lane && lane < jn) ? diag : 0.0;
}

// Write the stored (float) row, count the result; returns the stored value
// of a_lane as a double (0 past jn), or NaN in every lane if not finite.
__device__ __forceinline__ double ls_store(const ResolveArgs &a, int64_t i, double aq,
                                           int lane, int64_t cnt) {
    const bool fin = (lane >= a.jn) || isfinite(aq);
    const bool all = __all(fin);
    if (lane == 0) {
        atomicAdd(&a.stats[all ? 1 : 0], 1);
        atomicMax(&a.stats[2], (int32_t)(cnt < INT32_MAX ? cnt : INT32_MAX));
    }
    if (!all) return __builtin_nan("");
    const float af = (float)aq;
    if (lane < a.jn) a.A[i * a.jn + lane] = af;
    return lane < a.jn ? (double)af : 0.0;
}

// Sum over the chunks c = first, first + step, ... of the row of p (p - 2x),
// p = a^T delta with a_j held by lane j (af).
template <int JMAX>
__device__ __forceinline__ double ls_error(const ResolveArgs &a, int64_t r0, int64_t r1,
                                           int64_t first, int64_t step, double af,
                                           float *arow, int lane) {
    double acc = 0.0;
    for (int64_t c0 = r0 + first * kWave; c0 < r1; c0 += step * kWave) {
        double d[JMAX], x;
        chunk_rows<JMAX>(a, c0 + lane, r1, arow, lane, d, x);
        double p = 0.0;
#pragma unroll
        for (int j = 0; j < JMAX; ++j)
            if (j < a.jn) p = __builtin_fma(__shfl(af, j, kWave), d[j], p);
        acc += wsum(p * (p - 2.0 * x));
    }
    return acc;
}

}  // namespace

// W wavefronts per workgroup; dynamic LDS: W * (sum_k J_k) * 64 floats of
// factor rows, then W * JMAX * (JMAX + 1) doubles of triangles, then W + 1
// doubles of partial errors.
template <int JMAX, int W>
__global__ __launch_bounds__(kWave *W) void k_resolve(ResolveArgs a) {
    extern __shared__ __attribute__((aligned(16))) unsigned char s_dyn[];
    int sumj = 0;
    for (int k = 0; k < a.nother; ++k) sumj += a.jk[k];
    const int lane = threadIdx.x % kWave;
    const int w = threadIdx.x / kWave;
    float *arow = (float *)s_dyn + (size_t)w * sumj * kWave;
    double *s_tri = (double *)(s_dyn + (((size_t)W * sumj * kWave * 4 + 15) / 16) * 16);
    double *s_err = s_tri + (size_t)W * JMAX * (JMAX + 1);
    const double sl = sqrt(a.lambda);
    const int jn = a.jn;

    // heavy rows: one workgroup per row
    const int nheavy = a.cnt[1];
    for (int h = blockIdx.x; h < nheavy; h += gridDim.x) {
        const int64_t i = a.list[a.cap - 1 - h];
        const int64_t r0 = a.rowptr[i], r1 = a.rowptr[i + 1];
        double rc[JMAX];
        ls_init<JMAX>(rc, w == 0 ? sl : 0.0, jn, lane);
        for (int64_t c0 = r0 + (int64_t)w * kWave; c0 < r1; c0 += (int64_t)W * kWave) {
            double d[JMAX], x;
            chunk_rows<JMAX>(a, c0 + lane, r1, arow, lane, d, x);
            ls_merge<JMAX>(rc, d, x, jn, lane);
        }
        // helpers hand their triangles over, row p of [R | z] at s_tri[w][p][*]
        double *mine = s_tri + (size_t)w * JMAX * (JMAX + 1);
        if (w > 0 && lane <= jn) {
#pragma unroll
            for (int p = 0; p < JMAX; ++p)
                if (p < jn) mine[p * (JMAX + 1) + lane] = rc[p];
        }
        __syncthreads();
        double aq = 0.0;
        if (w == 0) {
            for (int v = 1; v < W; ++v) {
                const double *t = s_tri + (size_t)v * JMAX * (JMAX + 1);
                double d[JMAX], x = 0.0;
#pragma unroll
                for (int q = 0; q < JMAX; ++q)
                    d[q] = (lane < jn && q < jn) ? t[lane * (JMAX + 1) + q] : 0.0;
                if (lane < jn) x = t[lane * (JMAX + 1) + jn];
                ls_merge<JMAX>(rc, d, x, jn, lane);
            }
            aq = ls_back<JMAX>(rc, jn, lane);
            const double af = ls_store(a, i, aq, lane, r1 - r0);
            if (lane < JMAX) s_tri[lane] = af;        // hand the stored row over
        }
        __syncthreads();
        if (a.rsse) {
            const double af = lane < JMAX ? s_tri[lane] : 0.0;
            double e = 0.0;
            if (!isnan(af) && !isnan(s_tri[0]))
                e = ls_error<JMAX>(a, r0, r1, w, W, af, arow, lane);
            else
                e = __builtin_nan("");
            if (lane == 0) s_err[w] = e;
            __syncthreads();
            if (threadIdx.x == 0) {
                double t = 0.0;
                for (int v = 0; v < W; ++v) t += s_err[v];
                a.rsse[i] = t;
            }
        }
        __syncthreads();
    }

    // light rows: one wavefront per row
    const int nlight = a.cnt[0];
    for (int t = blockIdx.x * W + w; t < nlight; t += gridDim.x * W) {
        const int64_t i = a.list[t];
        const int64_t r0 = a.rowptr[i], r1 = a.rowptr[i + 1];
        double rc[JMAX];
        ls_init<JMAX>(rc, sl, jn, lane);
        for (int64_t c0 = r0; c0 < r1; c0 += kWave) {
            double d[JMAX], x;
            chunk_rows<JMAX>(a, c0 + lane, r1, arow, lane, d, x);
            ls_merge<JMAX>(rc, d, x, jn, lane);
        }
        const double aq = ls_back<JMAX>(rc, jn, lane);
        const double af = ls_store(a, i, aq, lane, r1 - r0);
        if (a.rsse) {
            const double e = isnan(__shfl(af, 0, kWave))
                                 ? __builtin_nan("")
                                 : ls_error<JMAX>(a, r0, r1, 0, 1, af, arow, lane);
            if (lane == 0) a.rsse[i] = e;
        }
    }
}

namespace {

template <int JMAX, int W>
size_t resolve_lds(int sumj) {
    return (((size_t)W * sumj * kWave * 4 + 15) / 16) * 16 +
           (size_t)W * JMAX * (JMAX + 1) * 8 + (W + 1) * 8;
}

template <int JMAX>
hipError_t launch_resolve_j(const ResolveArgs &a, int num_cu, hipStream_t st) {
    int sumj = 0;
    for (int k = 0; k < a.nother; ++k) sumj += a.jk[k];
    const dim3 grid((unsigned)(2 * num_cu));
    const size_t l4 = resolve_lds<JMAX, 4>(sumj), l2 = resolve_lds<JMAX, 2>(sumj),
                 l1 = resolve_lds<JMAX, 1>(sumj);
    if (l4 <= 64 * 1024)
        hipLaunchKernelGGL((k_resolve<JMAX, 4>), grid, dim3(4 * kWave), l4, st, a);
    else if (l2 <= 64 * 1024)
        hipLaunchKernelGGL((k_resolve<JMAX, 2>), grid, dim3(2 * kWave), l2, st, a);
    else
        hipLaunchKernelGGL((k_resolve<JMAX, 1>), grid, dim3(kWave), l1, st, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_resolve(const ResolveArgs &a, int num_cu, hipStream_t st) {
    const int jn = a.jn;
    if (jn <= 4) return launch_resolve_j<4>(a, num_cu, st);
    if (jn <= 8) return launch_resolve_j<8>(a, num_cu, st);
    if (jn <= 16) return launch_resolve_j<16>(a, num_cu, st);
    return launch_resolve_j<32>(a, num_cu, st);
}

}  // namespace ptk
