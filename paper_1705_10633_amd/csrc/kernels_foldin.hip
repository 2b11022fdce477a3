// kernels_foldin.hip -- fold-in of new users against stored posterior samples.
//
// For request r and stored sample s (movie factors V_s, user hypers
// Lambda_s, mu_s) the new user's row conditional is the same Gaussian as a
// Gibbs row update (paper: Section 2, Algorithm 1) with z = 0, i.e. its mean
//   m_s = (Lambda_s + alpha sum_j v_j v_j^T)^{-1} (Lambda_s mu_s + alpha sum_j (r_j - rbar) v_j),
// computed with the same wavefront building blocks as the sampler's FP32
// path (FP32 gathers, Gram on FP32 matrix cores, FP32 Cholesky).  One
// wavefront per (request, sample); each writes m_s . v_q for its request's
// query columns, and a second kernel averages the S partials in sample order.
// Nothing a wavefront computes depends on the other requests of the batch.
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
    hipLaunchKernelGGL(foldin_reduce_kernel, dim3((unsigned)((n_queries + 255) / 256)), dim3(256), 0,
                       st, S, fr, partial, n_queries, out);
    return hipGetLastError();
}

}  // namespace bpmf
