// kernels_foldin.hip -- fold-in of new users against stored posterior samples.
//
// For request r and stored sample s (movie factors V_s, user hypers
// Lambda_s, mu_s) the new user's row conditional is the same Gaussian as a
// Gibbs row update (paper: Section 2, Algorithm 1) with z = 0, i.e. its mean
//   m_s = (Lambda_s + alpha sum_j v_j v_j^T)^{-1} (Lambda_s mu_s + alpha sum_j (r_j - rbar) v_j),
// computed with the same wavefront building blocks as the sampler's FP32
// path (FP32 gathers, Gram on FP32 matrix cores, FP32 Cholesky).  One
// wavefront per (request, sample); each writes m_s . v_q for its request's
// query columns.  A pair whose FP32 pivot fails is recomputed in FP64 by a
// second kernel, and a third averages the S partials in sample order.
// Nothing a wavefront computes depends on the other requests of the batch.
#include <algorithm>
#include <mutex>

#include "common.hpp"
#include "rowsolve.hpp"

namespace bpmf {

namespace {

template <int KP>
__global__ __launch_bounds__(64) void foldin_kernel(int S, int K, int64_t N, float alpha, float rbar,
                                                    const float *Vs, const double *Lam,
                                                    const double *mu, const int64_t *req_ptr,
                                                    const int32_t *cols, const float *vals,
                                                    const int64_t *q_ptr, const int32_t *q_cols,
                                                    float *partial, int64_t n_queries)
{
    using SH = RowShape<KP>;
    __shared__ __attribute__((aligned(16))) float u[SH::UNION];
    __shared__ __attribute__((aligned(16))) float rv[64];
    __shared__ __attribute__((aligned(16))) float colbuf[3 * KP];
    __shared__ int sidx[16];
    const int lane = threadIdx.x;
    const int64_t r = blockIdx.x / S;
    const int s = (int)(blockIdx.x - r * S);
    const float *V = Vs + (int64_t)s * N * K;
    const double *L = Lam + (int64_t)s * K * K;
    const double *m0 = mu + (int64_t)s * K;
    const int64_t s0 = req_ptr[r], s1 = req_ptr[r + 1];

    floatx16 acc[SH::NTILE];
#pragma unroll
    for (int t = 0; t < SH::NTILE; ++t)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[t][e] = 0.0f;
    float bacc = 0.0f;
    gram_f32<KP>(cols + s0, vals + s0, s1 - s0, V, K, rbar, u, rv, sidx, acc, bacc);

    float *tri = u;
    store_precision<KP>(tri, acc, K, alpha, [=](int rr, int cc) { return (float)L[rr * K + cc]; });
    const int ri = lane % KP;
    float bb = 0.0f;
    if (ri < K) {
        double lm = 0.0;
        for (int c = 0; c < K; ++c) lm = fma(L[ri * K + c], m0[c], lm);
        bb = fmaf(alpha, bacc, (float)lm);
    }
    __syncthreads();
    bool fail;
    const float m = chol_solve<KP>(tri, colbuf, K, bb, 0.0f, fail);
    if (lane < KP) colbuf[lane] = (ri < K) ? (fail ? __builtin_nanf("") : m) : 0.0f;
    __syncthreads();
    const int64_t q0 = q_ptr[r], q1 = q_ptr[r + 1];
    for (int64_t q = q0 + lane; q < q1; q += 64) {
        const float *v = V + (int64_t)q_cols[q] * K;
        float p = 0.0f;
        for (int i = 0; i < K; ++i) p = fmaf(colbuf[i], v[i], p);
        partial[(int64_t)s * n_queries + q] = p;
    }
}

// FP64 recompute of the (request, sample) pairs whose FP32 Cholesky pivot
// failed (the same rule as the sampler's rows: a pivot that is not finite or
// not above 64 K 2^-24 max_k P_kk).  foldin_kernel writes NaN partial
// predictions for such a pair, so a pair is recomputed when its request has
// query columns (otherwise there is nothing to predict) and the partial of
// its first query is NaN.  Each block scans a slice of the pairs into an LDS
// list, then recomputes its listed pairs one after the other: the Gram of
// the FP32 sample rows in FP64, P = Lambda_s + alpha G in LDS, a
// right-looking Cholesky across the block, the two triangular solves (z = 0)
// and the query dot products, all in FP64.  With no failed pair the launch
// only reads one partial per pair.
constexpr int FF_THREADS = 256;
constexpr int FF_CH = 16;

__global__ __launch_bounds__(FF_THREADS) void foldin_f64_kernel(int S, int K, int64_t N, double alpha, double rbar,
                                                                const float *Vs, const double *Lam, const double *mu,
                                                                int64_t n_req, const int64_t *req_ptr,
                                                                const int32_t *cols, const float *vals,
                                                                const int64_t *q_ptr, const int32_t *q_cols,
                                                                float *partial, int64_t n_queries)
{
    __shared__ double P[64 * 64];
    __shared__ double stage[FF_CH * 64];
    __shared__ double rv[FF_CH];
    __shared__ double bv[64];
    __shared__ int sidx[FF_CH];
    __shared__ int64_t list[FF_THREADS];
    __shared__ int nlist, bad;
    const int tid = threadIdx.x;
    const int64_t npair = n_req * S;
    for (int64_t base = (int64_t)blockIdx.x * FF_THREADS; base < npair; base += (int64_t)gridDim.x * FF_THREADS) {
        if (tid == 0) nlist = 0;
        __syncthreads();
        const int64_t pr = base + tid;
        if (pr < npair) {
            const int64_t r = pr / S;
            const int s = (int)(pr - r * S);
            const int64_t q0 = q_ptr[r];
            if (q_ptr[r + 1] > q0 && isnan(partial[(int64_t)s * n_queries + q0])) list[atomicAdd(&nlist, 1)] = pr;
        }
        __syncthreads();
        const int cnt = nlist;
        for (int it = 0; it < cnt; ++it) {
            const int64_t r = list[it] / S;
            const int s = (int)(list[it] - r * S);
            const float *V = Vs + (int64_t)s * N * K;
            const double *L = Lam + (int64_t)s * K * K;
            const int64_t s0 = req_ptr[r], s1 = req_ptr[r + 1];
            // entries e = tid + 256 m of the full K x K Gram (K <= 64: m < 16)
            double acc[16];
#pragma unroll
            for (int m = 0; m < 16; ++m) acc[m] = 0.0;
            double bacc = 0.0;
            for (int64_t c0 = s0; c0 < s1; c0 += FF_CH) {
                const int n = (int)min((int64_t)FF_CH, s1 - c0);
                if (tid < n) {
                    sidx[tid] = cols[c0 + tid];
                    rv[tid] = (double)vals[c0 + tid] - rbar;
                }
                __syncthreads();
                for (int e = tid; e < n * K; e += FF_THREADS) {
                    const int q = e / K, f = e - q * K;
                    stage[q * 64 + f] = (double)V[(int64_t)sidx[q] * K + f];
                }
                __syncthreads();
#pragma unroll
                for (int m = 0; m < 16; ++m) {
                    const int e = tid + FF_THREADS * m;
                    if (e < K * K) {
                        const int i = e / K, j = e - i * K;
                        for (int q = 0; q < n; ++q) acc[m] = fma(stage[q * 64 + i], stage[q * 64 + j], acc[m]);
                    }
                }
                if (tid < K)
                    for (int q = 0; q < n; ++q) bacc = fma(rv[q], stage[q * 64 + tid], bacc);
                __syncthreads();
            }
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                const int e = tid + FF_THREADS * m;
                if (e < K * K) P[e] = fma(alpha, acc[m], L[e]);
            }
            if (tid < K) {
                const double *m0 = mu + (int64_t)s * K;
                double lm = 0.0;
                for (int c = 0; c < K; ++c) lm = fma(L[tid * K + c], m0[c], lm);
                bv[tid] = fma(alpha, bacc, lm);
            }
            if (tid == 0) bad = 0;
            __syncthreads();
            // right-looking Cholesky of the lower triangle, in place
            for (int k = 0; k < K; ++k) {
                if (tid == 0) {
                    double d = P[k * K + k];
                    if (!(d > 0.0) || !isfinite(d)) {
                        bad = 1;
                        d = 1.0;
                    }
                    P[k * K + k] = sqrt(d);
                }
                __syncthreads();
                const double dk = P[k * K + k];
                for (int i = k + 1 + tid; i < K; i += FF_THREADS) P[i * K + k] /= dk;
                __syncthreads();
                for (int e = tid; e < (K - k - 1) * (K - k - 1); e += FF_THREADS) {
                    const int i = k + 1 + e / (K - k - 1), j = k + 1 + e % (K - k - 1);
                    if (j <= i) P[i * K + j] = fma(-P[i * K + k], P[j * K + k], P[i * K + j]);
                }
                __syncthreads();
            }
            // m = L^{-T} L^{-1} b
            for (int k = 0; k < K; ++k) {
                const double yk = bv[k] / P[k * K + k];
                __syncthreads();
                for (int i = k + 1 + tid; i < K; i += FF_THREADS) bv[i] = fma(-P[i * K + k], yk, bv[i]);
                if (tid == 0) bv[k] = yk;
                __syncthreads();
            }
            for (int k = K - 1; k >= 0; --k) {
                const double xk = bv[k] / P[k * K + k];
                __syncthreads();
                for (int i = tid; i < k; i += FF_THREADS) bv[i] = fma(-P[k * K + i], xk, bv[i]);
                if (tid == 0) bv[k] = xk;
                __syncthreads();
            }
            const bool nan_out = bad != 0;
            for (int64_t q = q_ptr[r] + tid; q < q_ptr[r + 1]; q += FF_THREADS) {
                const float *v = V + (int64_t)q_cols[q] * K;
                double p = 0.0;
                for (int i = 0; i < K; ++i) p = fma(bv[i], (double)v[i], p);
                partial[(int64_t)s * n_queries + q] = nan_out ? __builtin_nanf("") : (float)p;
            }
            __syncthreads();
        }
        __syncthreads();
    }
}

__global__ void foldin_reduce_kernel(int S, float rbar, const float *partial, int64_t n_queries,
                                     float *out)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_queries) return;
    float acc = 0.0f;
    for (int s = 0; s < S; ++s) acc += partial[(int64_t)s * n_queries + q];
    out[q] = rbar + acc / (float)S;
}

}  // namespace

// Device-resident partials for bpmf_foldin_noalloc: a file-scope array, one
// copy per GPU, held until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is a stand-in, not a device
// address); it looks up each device's address once, with that device
// current, and passes that.
constexpr int64_t kNoallocPartials = int64_t(1) << 20;  // floats (4 MiB)
static __device__ __align__(256) float scratch[kNoallocPartials];

int64_t foldin_noalloc_max_partials() { return kNoallocPartials; }

hipError_t foldin_noalloc_scratch(float **out)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static float *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = (float *)p;
    }
    *out = addr[dev];
    return hipSuccess;
}

hipError_t launch_foldin(int S, int K, int64_t N, double alpha, double rbar, const float *Vs,
                         const double *Lam, const double *mu, int64_t n_req, const int64_t *req_ptr,
                         const int32_t *cols, const float *vals, const int64_t *q_ptr,
                         const int32_t *q_cols, int64_t n_queries, float *partial, float *out,
                         hipStream_t st)
{
    if (n_req <= 0) return hipSuccess;
    const dim3 grid((unsigned)(n_req * S)), block(64);
    const float fa = (float)alpha, fr = (float)rbar;
    if (K <= 32)
        hipLaunchKernelGGL(foldin_kernel<32>, grid, block, 0, st, S, K, N, fa, fr, Vs, Lam, mu,
                           req_ptr, cols, vals, q_ptr, q_cols, partial, n_queries);
    else if (K <= 64)
        hipLaunchKernelGGL(foldin_kernel<64>, grid, block, 0, st, S, K, N, fa, fr, Vs, Lam, mu,
                           req_ptr, cols, vals, q_ptr, q_cols, partial, n_queries);
    else
        return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n_queries <= 0) return e;
    const int64_t pair_blocks = (n_req * S + FF_THREADS - 1) / FF_THREADS;
    hipLaunchKernelGGL(foldin_f64_kernel, dim3((unsigned)std::min<int64_t>(pair_blocks, 1024)), dim3(FF_THREADS), 0, st,
                       S, K, N, alpha, rbar, Vs, Lam, mu, n_req, req_ptr, cols, vals, q_ptr, q_cols, partial,
                       n_queries);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(foldin_reduce_kernel, dim3((unsigned)((n_queries + 255) / 256)), dim3(256), 0,
                       st, S, fr, partial, n_queries, out);
    return hipGetLastError();
}

}  // namespace bpmf
