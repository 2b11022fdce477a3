// kernels_nw.hip -- the hyper-parameter step of one side (paper: Algorithm 1,
// "sample hyper-parameters ... based on U / V"; Section 2: Normal-Wishart
// hyperpriors on the shared Gaussian prior of the rows).
//
// One workgroup, FP64.  From the per-chunk sums of x_i and x_i x_i^T:
//   xbar = sum x / n,  S = sum x x^T - n xbar xbar^T
//   beta* = beta0 + n, nu* = nu0 + n, mu* = (beta0 mu0 + n xbar) / beta*
//   P = W0^{-1} + S + (beta0 n / beta*)(xbar - mu0)(xbar - mu0)^T
//   W* = P^{-1} = L^{-T} L^{-1} with L L^T = P
//   L_W = chol(W*);  A lower with A_kk = sqrt(chi2(nu* - k)), A_kl ~ N(0,1)
//   Lambda = (L_W A)(L_W A)^T  (Bartlett decomposition)
//   mu = mu* + chol(beta* Lambda)^{-T} z
// and Lambda mu, plus FP32 copies for the mixed-precision row kernels.
// The K x K work matrices live in LDS for K <= 64 and in a global scratch
// buffer (L2-resident) above that.
#include <algorithm>

#include "common.hpp"
#include "rng.hpp"

namespace bpmf {

namespace {

constexpr int NW_THREADS = 256;

// In-place right-looking Cholesky of the lower triangle of A (stride K).
__device__ void block_cholesky(double *A, int K, int *flag)
{
    const int tid = threadIdx.x;
    for (int k = 0; k < K; ++k) {
        if (tid == 0) {
            double d = A[k * K + k];
            if (!(d > 0.0) || !isfinite(d)) {
                *flag = 1;
                d = 1.0;
            }
            A[k * K + k] = sqrt(d);
        }
        __syncthreads();
        const double dk = A[k * K + k];
        for (int i = k + 1 + tid; i < K; i += NW_THREADS) A[i * K + k] /= dk;
        __syncthreads();
        const int mrem = K - k - 1;
        for (int ii = tid >> 4; ii < mrem; ii += NW_THREADS / 16) {
            const int i = k + 1 + ii;
            const double lik = A[i * K + k];
            for (int jj = tid & 15; jj <= ii; jj += 16) {
                const int j = k + 1 + jj;
                A[i * K + j] = fma(-lik, A[j * K + k], A[i * K + j]);
            }
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(NW_THREADS) void nw_kernel(const double *partials, int n_chunks,
                                                        int64_t n, int K, const double *mu0,
                                                        double beta0, double nu0,
                                                        const double *W0inv, DrawSrc draws,
                                                        double *scratch, HyperDev hyp,
                                                        int use_lds)
{
    extern __shared__ double lds[];
    __shared__ int s_flag;
    const int tid = threadIdx.x;
    const int KK = K * K;
    double *base = use_lds ? lds : scratch;
    double *M1 = base;
    double *M2 = M1 + KK;
    double *xbar = M2 + KK;          // K
    double *sums = xbar + K;         // K + K(K+1)/2
    double *chi2 = sums + K + K * (K + 1) / 2;  // K
    double *zb = chi2 + K;           // K(K-1)/2 (at least 1)
    double *zm = zb + max(1, K * (K - 1) / 2);  // K
    double *dvec = zm + K;           // K
    const int E = K + K * (K + 1) / 2;
    const double dn = (double)n;
    const double bstar = beta0 + dn, nstar = nu0 + dn;

    if (tid == 0) s_flag = 0;
    // 1. fixed-order reduction of the chunk partials
    for (int e = tid; e < E; e += NW_THREADS) {
        double s = 0.0;
        for (int c = 0; c < n_chunks; ++c) s += partials[(int64_t)c * E + e];
        sums[e] = s;
    }
    // draws
    if (draws.tape_nw) {
        for (int k = tid; k < K; k += NW_THREADS) chi2[k] = draws.tape_nw[k];
        for (int q = tid; q < K * (K - 1) / 2; q += NW_THREADS) zb[q] = draws.tape_nw[K + q];
        for (int q = tid; q < K; q += NW_THREADS) zm[q] = draws.tape_nw[K + K * (K - 1) / 2 + q];
    } else {
        const uint32_t h = half_sweep_index(draws);
        for (int k = tid; k < K; k += NW_THREADS)
            chi2[k] = 2.0 * gamma_mt(draws.seed, h, (uint32_t)k, 0.5 * (nstar - (double)k));
        for (int q = tid; q < K * (K - 1) / 2; q += NW_THREADS)
            zb[q] = stream_normal_f64(draws.seed, h, 1u, (uint32_t)q);
        for (int q = tid; q < K; q += NW_THREADS) zm[q] = stream_normal_f64(draws.seed, h, 2u, (uint32_t)q);
    }
    __syncthreads();
    for (int a = tid; a < K; a += NW_THREADS) xbar[a] = n > 0 ? sums[a] / dn : 0.0;
    __syncthreads();
    // 2. P = W0^{-1} + S + coef (xbar - mu0)(xbar - mu0)^T, both triangles
    const double coef = beta0 * dn / bstar;
    for (int e = tid; e < KK; e += NW_THREADS) {
        const int a = e / K, c = e - a * K;
        const int hi = a > c ? a : c, lo = a > c ? c : a;
        const double sxx = sums[K + hi * (hi + 1) / 2 + lo];
        const double S = sxx - dn * xbar[a] * xbar[c];
        M1[e] = W0inv[e] + S + coef * (xbar[a] - mu0[a]) * (xbar[c] - mu0[c]);
    }
    __syncthreads();
    // 3. L = chol(P)
    block_cholesky(M1, K, &s_flag);
    // 4. M2 = L^{-1}, column c by forward substitution (one thread per column)
    for (int c = tid; c < K; c += NW_THREADS) {
        for (int i = 0; i < c; ++i) M2[i * K + c] = 0.0;
        M2[c * K + c] = 1.0 / M1[c * K + c];
        for (int i = c + 1; i < K; ++i) {
            double s = 0.0;
            for (int m = c; m < i; ++m) s = fma(M1[i * K + m], M2[m * K + c], s);
            M2[i * K + c] = -s / M1[i * K + i];
        }
    }
    __syncthreads();
    // 5. W* = L^{-T} L^{-1}
    for (int e = tid; e < KK; e += NW_THREADS) {
        const int a = e / K, c = e - a * K;
        const int m0 = a > c ? a : c;
        double s = 0.0;
        for (int m = m0; m < K; ++m) s = fma(M2[m * K + a], M2[m * K + c], s);
        M1[e] = s;
    }
    __syncthreads();
    // 6. L_W = chol(W*)
    block_cholesky(M1, K, &s_flag);
    // 7. T = L_W A (lower)
    for (int e = tid; e < KK; e += NW_THREADS) {
        const int a = e / K, c = e - a * K;
        double s = 0.0;
        for (int m = c; m <= a; ++m) {
            const double Amc = (m == c) ? sqrt(chi2[c]) : zb[m * (m - 1) / 2 + c];
            s = fma(M1[a * K + m], Amc, s);
        }
        M2[e] = (c <= a) ? s : 0.0;
    }
    __syncthreads();
    // 8. Lambda = T T^T
    for (int e = tid; e < KK; e += NW_THREADS) {
        const int a = e / K, c = e - a * K;
        const int m1 = a < c ? a : c;
        double s = 0.0;
        for (int m = 0; m <= m1; ++m) s = fma(M2[a * K + m], M2[c * K + m], s);
        M1[e] = s;
        hyp.Lambda[e] = s;
        hyp.Lambda_f[e] = (float)s;
    }
    __syncthreads();
    // 9. chol(beta* Lambda) and mu = mu* + Lc^{-T} z
    for (int e = tid; e < KK; e += NW_THREADS) M2[e] = bstar * M1[e];
    __syncthreads();
    block_cholesky(M2, K, &s_flag);
    if (tid == 0) {
        // backward substitution Lc^T d = z
        for (int k = K - 1; k >= 0; --k) {
            double s = zm[k];
            for (int m = k + 1; m < K; ++m) s = fma(-M2[m * K + k], dvec[m], s);
            dvec[k] = s / M2[k * K + k];
        }
    }
    __syncthreads();
    for (int a = tid; a < K; a += NW_THREADS) {
        const double mus = (beta0 * mu0[a] + dn * xbar[a]) / bstar;
        hyp.mu[a] = mus + dvec[a];
    }
    __syncthreads();
    for (int a = tid; a < K; a += NW_THREADS) {
        double s = 0.0;
        for (int c = 0; c < K; ++c) s = fma(M1[a * K + c], hyp.mu[c], s);
        hyp.Lmu[a] = s;
        hyp.Lmu_f[a] = (float)s;
    }
}

}  // namespace

hipError_t prepare_nw(int K)
{
    if (K > 64) return hipSuccess;
    return hipFuncSetAttribute((const void *)nw_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(nw_scratch_doubles(K) * sizeof(double)));
}

size_t nw_scratch_doubles(int K)
{
    return (size_t)2 * K * K + K + K + K * (K + 1) / 2 + K + (size_t)std::max(1, K * (K - 1) / 2) + K + K;
}

hipError_t launch_nw(const double *partials, int n_chunks, int64_t n, int K, const double *mu0,
                     double beta0, double nu0, const double *W0inv, DrawSrc draws,
                     double *scratch, HyperDev hyp, int use_lds, hipStream_t s)
{
    size_t lds = use_lds ? nw_scratch_doubles(K) * sizeof(double) : 0;
    hipLaunchKernelGGL(nw_kernel, dim3(1), dim3(NW_THREADS), lds, s, partials, n_chunks, n, K,
                       mu0, beta0, nu0, W0inv, draws, scratch, hyp, use_lds);
    return hipGetLastError();
}

}  // namespace bpmf
