// Final step of Alg. 2 (Sec. 3.1): A^(n) = Q^(n) R^(n), A^(n) <- Q^(n),
// G <- G x_n R^(n), in FP64.
//
// The thin QR of the tall-skinny I x J factor is taken by shifted
// CholeskyQR3 (Fukaya, Kannan, Nakatsukasa, Yamamoto and Yanagisawa, 2020):
// a first pass factors W + s I = R_0^T R_0, W = A^T A, with the shift
// s = 11 (I J + J (J + 1)) u ||A||_F^2 (u = 2^-53, ||A||_F^2 = trace W), and
// Q_0 = A R_0^{-1} is then well enough conditioned for CholeskyQR2 (Fukaya
// et al., 2014): W = Q^T Q = R^T R, Q = Q R^{-1}, twice; R = R_2 R_1 R_0.
// The shift keeps the first Cholesky factorisation defined up to
// cond(A) of about 1/u instead of 1/sqrt(u); the two unshifted passes make
// Q orthonormal to working precision. Cholesky factors have a positive
// diagonal, so this is the unique thin QR with diag(R) > 0 when A has full
// column rank. The Gram sums are deterministic two-level reductions.
#include "ptk_internal.h"

namespace ptk {

constexpr int kQrThreads = 256;
constexpr int kQrRows = 64;          // rows staged in LDS per step
constexpr int kQrBlocks = 512;

// Per-block partial of the packed upper triangle of X^T X (X is fp32 or fp64).
template <typename T>
__global__ __launch_bounds__(kQrThreads) void k_colgram(const T *__restrict__ X,
                                                        int64_t I, int J,
                                                        double *__restrict__ part) {
    __shared__ double s_x[kQrRows * kMaxJ];
    const int Tn = J * (J + 1) / 2;
    // entries owned by this thread: t, t + 256, t + 512 (J <= 32 -> Tn <= 528)
    double acc[3] = {0.0, 0.0, 0.0};
    int pp[3], qq[3];
    for (int u = 0; u < 3; ++u) {
        int e = threadIdx.x + u * kQrThreads;
        pp[u] = qq[u] = -1;
        if (e < Tn) {
            int p = 0;
            while (e >= J - p) {
                e -= J - p;
                ++p;
            }
            pp[u] = p;
            qq[u] = p + e;
        }
    }
    const int64_t per = (I + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * per;
    const int64_t r1 = min(I, r0 + per);
    for (int64_t base = r0; base < r1; base += kQrRows) {
        const int nr = (int)min((int64_t)kQrRows, r1 - base);
        __syncthreads();
        for (int t = threadIdx.x; t < nr * J; t += kQrThreads)
            s_x[t] = (double)X[base * J + t];
        __syncthreads();
        for (int u = 0; u < 3; ++u) {
            if (pp[u] < 0) continue;
            double a = acc[u];
            for (int r = 0; r < nr; ++r)
                a = __builtin_fma(s_x[r * J + pp[u]], s_x[r * J + qq[u]], a);
            acc[u] = a;
        }
    }
    for (int u = 0; u < 3; ++u) {
        const int e = threadIdx.x + u * kQrThreads;
        if (e < Tn) part[(int64_t)blockIdx.x * Tn + e] = acc[u];
    }
}

// Sum the block partials in order, factor W = R^T R; R (J x J, row-major,
// upper) goes to R_out. If Rprev is given, R_out = R * Rprev and Rcur keeps R.
// With shift_frac > 0, shift_frac * trace(W) is added to the diagonal first.
__global__ __launch_bounds__(64) void k_chol_small(const double *__restrict__ part,
                                                   int nparts, int J, double shift_frac,
                                                   double *__restrict__ Rcur,
                                                   const double *__restrict__ Rprev,
                                                   double *__restrict__ Rout,
                                                   int32_t *__restrict__ bad) {
    __shared__ double W[kMaxJ * kMaxJ];
    __shared__ double R[kMaxJ * kMaxJ];
    const int Tn = J * (J + 1) / 2;
    for (int e = threadIdx.x; e < Tn; e += blockDim.x) {
        double s = 0.0;
        for (int b = 0; b < nparts; ++b) s += part[(int64_t)b * Tn + e];
        int p = 0, r = e;
        while (r >= J - p) {
            r -= J - p;
            ++p;
        }
        W[p * J + p + r] = s;      // upper triangle, row-major
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (shift_frac > 0.0) {
            double tr = 0.0;
            for (int i = 0; i < J; ++i) tr += W[i * J + i];
            for (int i = 0; i < J; ++i) W[i * J + i] += shift_frac * tr;
        }
        // W = R^T R, R upper: R[i][j] for j >= i
        bool ok = true;
        for (int i = 0; i < J * J; ++i) R[i] = 0.0;
        for (int i = 0; i < J && ok; ++i) {
            double d = W[i * J + i];
            for (int k = 0; k < i; ++k) d -= R[k * J + i] * R[k * J + i];
            if (!(d > 0.0)) {
                ok = false;
                break;
            }
            d = sqrt(d);
            R[i * J + i] = d;
            for (int j = i + 1; j < J; ++j) {
                double s = W[i * J + j];
                for (int k = 0; k < i; ++k) s -= R[k * J + i] * R[k * J + j];
                R[i * J + j] = s / d;
            }
        }
        if (!ok) {
            atomicAdd(bad, 1);
            for (int i = 0; i < J * J; ++i) R[i] = (i % (J + 1) == 0) ? 1.0 : 0.0;
        }
        for (int i = 0; i < J * J; ++i) Rcur[i] = R[i];
        if (Rprev) {
            for (int i = 0; i < J; ++i)
                for (int j = 0; j < J; ++j) {
                    double s = 0.0;
                    for (int k = 0; k < J; ++k) s += R[i * J + k] * Rprev[k * J + j];
                    Rout[i * J + j] = s;
                }
        }
    }
}

// Q = X R^{-1} row by row: q R = x  (forward substitution on R^T).
template <typename T>
__global__ void k_right_solve(const T *__restrict__ X, int64_t I, int J,
                              const double *__restrict__ R, double *__restrict__ Q,
                              float *__restrict__ Qf) {
    __shared__ double s_r[kMaxJ * kMaxJ];
    for (int t = threadIdx.x; t < J * J; t += blockDim.x) s_r[t] = R[t];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= I) return;
    double q[kMaxJ];
#pragma unroll
    for (int j = 0; j < kMaxJ; ++j) {
        if (j >= J) break;
        double s = (double)X[i * J + j];
        for (int k = 0; k < j; ++k) s -= q[k] * s_r[k * J + j];
        q[j] = s / s_r[j * J + j];
    }
#pragma unroll
    for (int j = 0; j < kMaxJ; ++j) {
        if (j >= J) break;
        if (Q) Q[i * J + j] = q[j];
        if (Qf) Qf[i * J + j] = (float)q[j];
    }
}

size_t qr_workspace_bytes(int64_t I, int J) {
    const int Tn = J * (J + 1) / 2;
    return (size_t)2 * I * J * 8 + (size_t)kQrBlocks * Tn * 8 + 4 * kMaxJ * kMaxJ * 8 +
           1024;
}

hipError_t launch_thin_qr(float *A, int64_t I, int J, void *work, double *R,
                          int32_t *bad, hipStream_t st) {
    const int Tn = J * (J + 1) / 2;
    double *Q0 = (double *)work;
    double *Q1 = Q0 + I * J;
    double *part = Q1 + I * J;
    double *R0 = part + (size_t)kQrBlocks * Tn;
    double *R1 = R0 + kMaxJ * kMaxJ;
    double *R10 = R1 + kMaxJ * kMaxJ;
    double *R2 = R10 + kMaxJ * kMaxJ;
    int64_t nb64 = (I + kQrRows - 1) / kQrRows;
    int blocks = (int)(nb64 < kQrBlocks ? nb64 : kQrBlocks);
    if (blocks < 1) blocks = 1;
    const unsigned rs_blocks = (unsigned)((I + 255) / 256);
    const double shift = 11.0 * ((double)I * J + (double)J * (J + 1)) * 0x1p-53;
    // shifted pass: W = A^T A, W + s I = R0^T R0, Q0 = A R0^{-1}
    hipLaunchKernelGGL(k_colgram<float>, dim3(blocks), dim3(kQrThreads), 0, st, A, I,
                       J, part);
    hipLaunchKernelGGL(k_chol_small, dim3(1), dim3(64), 0, st, part, blocks, J, shift, R0,
                       (const double *)nullptr, (double *)nullptr, bad);
    hipLaunchKernelGGL(k_right_solve<float>, dim3(rs_blocks), dim3(256), 0, st, A, I,
                       J, R0, Q0, (float *)nullptr);
    // CholeskyQR2 on Q0: R1 (R10 = R1 R0), Q1 = Q0 R1^{-1}; R2 (R = R2 R10),
    // Q = Q1 R2^{-1} written to A
    hipLaunchKernelGGL(k_colgram<double>, dim3(blocks), dim3(kQrThreads), 0, st, Q0,
                       I, J, part);
    hipLaunchKernelGGL(k_chol_small, dim3(1), dim3(64), 0, st, part, blocks, J, 0.0, R1,
                       R0, R10, bad);
    hipLaunchKernelGGL(k_right_solve<double>, dim3(rs_blocks), dim3(256), 0, st, Q0,
                       I, J, R1, Q1, (float *)nullptr);
    hipLaunchKernelGGL(k_colgram<double>, dim3(blocks), dim3(kQrThreads), 0, st, Q1,
                       I, J, part);
    hipLaunchKernelGGL(k_chol_small, dim3(1), dim3(64), 0, st, part, blocks, J, 0.0, R2,
                       R10, R, bad);
    hipLaunchKernelGGL(k_right_solve<double>, dim3(rs_blocks), dim3(256), 0, st, Q1,
                       I, J, R2, (double *)nullptr, A);
    return hipGetLastError();
}

// G' = G x_n R: G'[.., j, ..] = sum_k R[j][k] G[.., k, ..] (FP64 core).
struct NmodeArgs {
    int32_t N, n;
    int32_t J[kMaxN];
    int64_t S, inner;
};

__global__ void k_nmode(const double *__restrict__ Gin, double *__restrict__ Gout,
                        NmodeArgs a, const double *__restrict__ R) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.S) return;
    const int Jn = a.J[a.n];
    const int j = (int)((s / a.inner) % Jn);
    const int64_t base = s - (int64_t)j * a.inner;
    double acc = 0.0;
    for (int k = 0; k < Jn; ++k) acc += R[j * Jn + k] * Gin[base + (int64_t)k * a.inner];
    Gout[s] = acc;
}

__global__ void k_f32_to_f64(const float *__restrict__ x, double *__restrict__ y,
                             int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = (double)x[i];
}
__global__ void k_f64_to_f32(const double *__restrict__ x, float *__restrict__ y,
                             int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = (float)x[i];
}

// G (float) <- G x_1 R^(1) ... x_N R^(N); Rs holds the N factors packed
// (kMaxJ^2 apart); work holds 2 * S doubles.
hipError_t launch_core_mode_product(const float *G, float *Gout, const Shape &s,
                                    int n_unused, const double *Rs,
                                    hipStream_t st) {
    (void)n_unused;
    int64_t S = 1;
    for (int k = 0; k < s.N; ++k) S *= s.ranks[k];
    double *g0 = (double *)(Rs + (size_t)kMaxN * kMaxJ * kMaxJ);
    double *g1 = g0 + S;
    const unsigned blocks = (unsigned)((S + 255) / 256);
    hipLaunchKernelGGL(k_f32_to_f64, dim3(blocks), dim3(256), 0, st, G, g0, S);
    for (int n = 0; n < s.N; ++n) {
        NmodeArgs a;
        a.N = s.N;
        a.n = n;
        a.S = S;
        a.inner = 1;
        for (int k = 0; k < s.N; ++k) a.J[k] = s.ranks[k];
        for (int k = n + 1; k < s.N; ++k) a.inner *= s.ranks[k];
        hipLaunchKernelGGL(k_nmode, dim3(blocks), dim3(256), 0, st, g0, g1, a,
                           Rs + (size_t)n * kMaxJ * kMaxJ);
        double *t = g0;
        g0 = g1;
        g1 = t;
    }
    hipLaunchKernelGGL(k_f64_to_f32, dim3(blocks), dim3(256), 0, st, g0, Gout, S);
    return hipGetLastError();
}

}  // namespace ptk
