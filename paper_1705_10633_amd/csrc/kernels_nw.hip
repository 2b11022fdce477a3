// kernels_nw.hip -- the hyper-parameter step of one side (paper: Algorithm 1,
// "sample hyper-parameters ... based on U / V"; Section 2: Normal-Wishart
// hyperpriors on the shared Gaussian prior of the rows).
//
// From the sums of x_i and x_i x_i^T over the n rows of the side, FP64:
//   xbar = sum x / n,  S = sum x x^T - n xbar xbar^T
//   beta* = beta0 + n, nu* = nu0 + n, mu* = (beta0 mu0 + n xbar) / beta*
//   P = W0^{-1} + S + (beta0 n / beta*)(xbar - mu0)(xbar - mu0)^T,  W* = P^{-1}
//   Lambda = (L_W A)(L_W A)^T with L_W = chol(W*) and the Bartlett factor A
//   (A_kk = sqrt(chi2(nu* - k)), A_kl ~ N(0,1) below the diagonal)
//   mu = mu* + chol(beta* Lambda)^{-T} z.
// Two identities keep this to one factorisation and two triangular solves:
//  * with P = R R^T, R upper triangular with positive diagonal (a Cholesky
//    factorisation that starts from the last pivot), R^{-T} is lower
//    triangular with positive diagonal and R^{-T} R^{-1} = W*, so it is
//    chol(W*); T = L_W A is then the solution of R^T T = A;
//  * T is lower triangular with positive diagonal and T T^T = Lambda, so
//    chol(beta* Lambda) = sqrt(beta*) T and the mean draw solves
//    T^T d = z / sqrt(beta*).
// One workgroup; the K x K work matrices live in LDS for K <= 64 and in a
// global scratch buffer (L2-resident) above that.
#include <algorithm>

#include "common.hpp"
#include "rng.hpp"

namespace bpmf {

namespace {

constexpr int NW_THREADS = 256;

// sums[e] = sum over chunks of partials[c][e]: 8 threads per entry over fixed
// chunk ranges, combined by a fixed xor tree.
__global__ __launch_bounds__(256) void stats_reduce_kernel(const double *partials, int n_chunks,
                                                           int E, double *sums)
{
    const int e = blockIdx.x * 32 + (threadIdx.x >> 3);
    const int part = threadIdx.x & 7;
    double s = 0.0;
    if (e < E) {
        // four independent accumulators (fixed assignment c % 4), combined in order
        const int c0 = n_chunks * part / 8, c1 = n_chunks * (part + 1) / 8;
        double s4[4] = {0.0, 0.0, 0.0, 0.0};
        int c = c0;
        for (; c + 4 <= c1; c += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) s4[u] += partials[(int64_t)(c + u) * E + e];
        }
        for (int u = 0; c < c1; ++c, ++u) s4[u] += partials[(int64_t)c * E + e];
        s = (s4[0] + s4[1]) + (s4[2] + s4[3]);
    }
    s += __shfl_xor(s, 4, 8);
    s += __shfl_xor(s, 2, 8);
    s += __shfl_xor(s, 1, 8);
    if (part == 0 && e < E) sums[e] = s;
}

template <bool USE_LDS>
__global__ __launch_bounds__(NW_THREADS) void nw_kernel(const double *sums, int64_t n, int K,
                                                        const double *mu0, double beta0, double nu0,
                                                        const double *W0inv, DrawSrc draws,
                                                        double *scratch, HyperDev hyp,
                                                        DevState *state)
{
    extern __shared__ double lds[];
    __shared__ int s_flag;
    const int tid = threadIdx.x;
    const int KK = K * K;
    double *base = USE_LDS ? lds : scratch;
    double *M1 = base;                    // P, then R (upper) / Lambda
    double *M2 = M1 + KK;                 // T (lower)
    double *xbar = M2 + KK;               // K
    double *rd = xbar + K;                // K: diagonal of R
    double *chi2 = rd + K;                // K
    double *zb = chi2 + K;                // K(K-1)/2 (at least 1)
    double *zm = zb + max(1, K * (K - 1) / 2);  // K
    double *dvec = zm + K;                // K
    double *dout = dvec + K;              // K
    const double dn = (double)n;
    const double bstar = beta0 + dn, nstar = nu0 + dn;

    if (tid == 0) s_flag = 0;
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
    for (int a = tid; a < K; a += NW_THREADS) xbar[a] = n > 0 ? sums[a] / dn : 0.0;
    __syncthreads();
    // P = W0^{-1} + S + coef (xbar - mu0)(xbar - mu0)^T (both triangles)
    const double coef = beta0 * dn / bstar;
    for (int e = tid; e < KK; e += NW_THREADS) {
        const int a = e / K, c = e - a * K;
        const int hi = a > c ? a : c, lo = a > c ? c : a;
        const double sxx = sums[K + hi * (hi + 1) / 2 + lo];
        const double S = sxx - dn * xbar[a] * xbar[c];
        M1[e] = W0inv[e] + S + coef * (xbar[a] - mu0[a]) * (xbar[c] - mu0[c]);
    }
    // P = R R^T from the last pivot up.  Step k reads column k of the
    // remaining block from the lower positions (k, i), i < k, writes
    // R_ik = P_ki / R_kk to the upper position (i, k) and updates the leading
    // block's lower triangle; those positions are disjoint, so one barrier
    // per step suffices.
    for (int k = K - 1; k >= 0; --k) {
        __syncthreads();
        double akk = M1[k * K + k];
        if (!(akk > 0.0) || !isfinite(akk)) {
            if (tid == 0) s_flag = 1;
            akk = 1.0;
        }
        const double rkk = sqrt(akk);
        const double inv = 1.0 / rkk;
        const double inv2 = 1.0 / akk;
        if (tid == 0) rd[k] = rkk;
        for (int i = tid; i < k; i += NW_THREADS) M1[i * K + k] = M1[k * K + i] * inv;
        for (int ii = tid >> 4; ii < k; ii += NW_THREADS / 16) {
            const double pki = M1[k * K + ii] * inv2;
            for (int jj = tid & 15; jj <= ii; jj += 16) M1[ii * K + jj] = fma(-pki, M1[k * K + jj], M1[ii * K + jj]);
        }
    }
    __syncthreads();
    // T: R^T T = A (both lower triangular), right-looking: step m fixes row m
    // of T and removes its contribution from the rows below.  M2 starts as A.
    for (int e = tid; e < KK; e += NW_THREADS) {
        const int i = e / K, c = e - i * K;
        M2[e] = (c > i) ? 0.0 : ((i == c) ? sqrt(chi2[c]) : zb[i * (i - 1) / 2 + c]);
    }
    for (int m = 0; m < K; ++m) {
        __syncthreads();
        const double irm = 1.0 / rd[m];
        // rows i > m, columns c <= m: M2[i][c] -= R_mi T_mc, with T_mc = M2[m][c] / R_mm
        const int rows = K - 1 - m, cols = m + 1;
        for (int e = tid; e < rows * cols; e += NW_THREADS) {
            const int ii = e / cols, c = e - ii * cols;
            const int i = m + 1 + ii;
            M2[i * K + c] = fma(-M1[m * K + i], M2[m * K + c] * irm, M2[i * K + c]);
        }
        __syncthreads();
        for (int c = tid; c <= m; c += NW_THREADS) M2[m * K + c] *= irm;
    }
    __syncthreads();
    // Lambda = T T^T in 4x4 register tiles (T[a][m] = 0 for m > a)
    {
        const int nb = (K + 3) / 4;
        for (int tb = tid; tb < nb * nb; tb += NW_THREADS) {
            const int ba = tb / nb, bc = tb - ba * nb;
            double acc[4][4] = {};
            const int mmax = min(K, 4 * min(ba, bc) + 4);
            for (int m = 0; m < mmax; ++m) {
                double ta[4], tc[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int a = 4 * ba + q, c = 4 * bc + q;
                    ta[q] = a < K ? M2[a * K + m] : 0.0;
                    tc[q] = c < K ? M2[c * K + m] : 0.0;
                }
#pragma unroll
                for (int x = 0; x < 4; ++x)
#pragma unroll
                    for (int y = 0; y < 4; ++y) acc[x][y] = fma(ta[x], tc[y], acc[x][y]);
            }
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) {
                    const int a = 4 * ba + x, c = 4 * bc + y;
                    if (a < K && c < K) {
                        M1[a * K + c] = acc[x][y];
                        hyp.Lambda[a * K + c] = acc[x][y];
                        hyp.Lambda_f[a * K + c] = (float)acc[x][y];
                    }
                }
        }
    }
    // mean: T^T d = z / sqrt(beta*), column-oriented backward substitution
    const double isb = 1.0 / sqrt(bstar);
    for (int a = tid; a < K; a += NW_THREADS) dvec[a] = zm[a] * isb;
    for (int k = K - 1; k >= 0; --k) {
        __syncthreads();
        const double dk = dvec[k] / M2[k * K + k];
        if (tid == 0) dout[k] = dk;
        for (int i = tid; i < k; i += NW_THREADS) dvec[i] = fma(-M2[k * K + i], dk, dvec[i]);
    }
    __syncthreads();
    for (int a = tid; a < K; a += NW_THREADS) {
        const double mus = (beta0 * mu0[a] + dn * xbar[a]) / bstar;
        hyp.mu[a] = mus + dout[a];
        dvec[a] = mus + dout[a];
    }
    __syncthreads();
    for (int a = tid; a < K; a += NW_THREADS) {
        double s = 0.0;
        for (int c = 0; c < K; ++c) s = fma(M1[a * K + c], dvec[c], s);
        hyp.Lmu[a] = s;
        hyp.Lmu_f[a] = (float)s;
    }
    if (tid == 0 && s_flag) atomicAdd((unsigned long long *)&state->nonfinite_rows, 1ull);
}

}  // namespace

size_t nw_scratch_doubles(int K)
{
    return (size_t)2 * K * K + 4 * (size_t)K + (size_t)std::max(1, K * (K - 1) / 2) + 3 * (size_t)K;
}

hipError_t prepare_nw(int K)
{
    if (K > 64) return hipSuccess;
    return hipFuncSetAttribute((const void *)nw_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(nw_scratch_doubles(K) * sizeof(double)));
}

hipError_t launch_stats_reduce(const double *partials, int n_chunks, int K, double *sums, hipStream_t s)
{
    const int E = K + K * (K + 1) / 2;
    hipLaunchKernelGGL(stats_reduce_kernel, dim3((unsigned)((E + 31) / 32)), dim3(256), 0, s, partials,
                       n_chunks, E, sums);
    return hipGetLastError();
}

hipError_t launch_nw(const double *sums, int64_t n, int K, const double *mu0, double beta0, double nu0,
                     const double *W0inv, DrawSrc draws, double *scratch, HyperDev hyp, int use_lds,
                     DevState *state, hipStream_t s)
{
    size_t lds = use_lds ? nw_scratch_doubles(K) * sizeof(double) : 0;
    if (use_lds)
        hipLaunchKernelGGL(nw_kernel<true>, dim3(1), dim3(NW_THREADS), lds, s, sums, n, K, mu0, beta0, nu0,
                           W0inv, draws, scratch, hyp, state);
    else
        hipLaunchKernelGGL(nw_kernel<false>, dim3(1), dim3(NW_THREADS), 0, s, sums, n, K, mu0, beta0, nu0,
                           W0inv, draws, scratch, hyp, state);
    return hipGetLastError();
}

}  // namespace bpmf
