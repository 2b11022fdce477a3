// kernels_mixed.hip -- mixed-precision row update, one wavefront per row.
//
// Same conditional as the FP64 path (paper: Section 2 and Algorithm 1; the
// Cholesky-instead-of-inverse choice of Section 3.1):
//   P = Lambda + alpha G,  G = sum_{j in Omega_i} v_j v_j^T,
//   b = Lambda mu + alpha sum_j (r_ij - rbar) v_j,  x_i = L^{-T}(L^{-1} b + z_i).
//
// gfx950 mapping (K padded to KP = 32 or 64 with an identity block):
//  * gather: each lane fetches 16-byte pieces of 4 rated rows; BF16 mode reads
//    the BF16 copy of the other side (row stride KP), FP32 mode the FP32 master;
//  * Gram on v_mfma_f32_32x32x16_bf16 (BF16) or v_mfma_f32_32x32x2_f32 (FP32),
//    lower 32x32 tiles only, FP32 accumulation;
//  * FP32 Cholesky and solves with one matrix row per lane;
//  * a row whose pivot is not finite or not above 64 K 2^-24 max_k P_kk is not
//    written; it is appended to a list that the FP64 kernel recomputes.
#include "common.hpp"
#include "rng.hpp"
#include "rowsolve.hpp"

namespace bpmf {

namespace {

template <int KP, bool BF16>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 4))) void rows_mixed_kernel(SideArgs a, int K, float alpha, float rbar,
                                                        HyperDev hyp, DrawSrc draws,
                                                        int32_t *fb_list, DevState *state,
                                                        int side)
{
    using S = RowShape<KP>;
    __shared__ __attribute__((aligned(16))) float u[S::UNION];
    __shared__ __attribute__((aligned(16))) float rv[64];
    __shared__ __attribute__((aligned(16))) float colbuf[3 * KP];
    __shared__ int sidx[16];

    const int lane = threadIdx.x;
    const int4 rt = a.rowtab[blockIdx.x];
    const int row = rt.x;
    const int64_t s0 = (int64_t)(((uint64_t)(uint32_t)rt.w << 32) | (uint32_t)rt.z), s1 = s0 + rt.y;
    const float *vals = (const float *)a.val;

    floatx16 acc[S::NTILE];
#pragma unroll
    for (int t = 0; t < S::NTILE; ++t)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[t][e] = 0.0f;
    float bacc = 0.0f;

    if constexpr (BF16)
        gram_bf16<KP>(a.idx + s0, vals + s0, s1 - s0, a.other_bf16, a.shadow_stride, (int32_t)a.n_other,
                      rbar, (char *)u, (uint32_t *)rv, acc, bacc);
    else
        gram_f32<KP>(a.idx + s0, vals + s0, s1 - s0, (const float *)a.other, K, rbar, u, rv,
                     sidx, acc, bacc);

    float *tri = u;
    store_precision_tri<KP>(tri, acc, alpha, hyp.Lambda_tri);
    const int ri = lane % KP;
    // unconditional load and a multiplicative mask: as a select, the load
    // would be moved behind a branch with its own wait
    const float bb = fmaf(alpha, bacc, hyp.Lmu_f[ri < K ? ri : 0]) * (ri < K ? 1.0f : 0.0f);

    float z;
    if (draws.tape_rows) {
        z = (ri < K) ? (float)draws.tape_rows[(int64_t)row * K + ri] : 0.0f;
    } else {
        const uint32_t h = half_sweep_index(draws);
        if (lane < KP / 2) {
            float z0, z1;
            box_muller_f32(philox4x32_10(ctr4((uint32_t)lane, (uint32_t)row, h, 0u), draws.seed), z0, z1);
            colbuf[2 * lane] = z0;
            colbuf[2 * lane + 1] = z1;
        }
        __syncthreads();
        z = (ri < K) ? colbuf[ri] : 0.0f;
    }
    __syncthreads();

    bool fail;
    const float x = chol_solve<KP>(tri, colbuf, K, bb, z, fail);
    if (!fail) {
        float *X = (float *)a.X;
        if (lane < KP && ri < K) X[(int64_t)row * K + ri] = x;
        if (a.X_bf16 && lane < KP)
            a.X_bf16[(int64_t)row * a.shadow_stride + ri] = ri < K ? f32_to_bf16_rne(x) : (uint16_t)0;
    } else if (lane == 0) {
        const int pos = atomicAdd(&state->fb_count[side], 1);
        fb_list[pos] = row;
    }
}

// Rows with many ratings (the head of the rating-count order): the gathers
// and the Gram are split over HW wavefronts, each taking a contiguous slice
// of the row's ratings; the partial Gram tiles and right-hand sides are
// summed in a fixed tree through LDS (so the result does not depend on
// timing), and wavefront 0 forms P, factors and samples as in
// rows_mixed_kernel.  One wavefront per row would leave a row with thousands
// of ratings running long after the rest of the launch has finished (the
// load imbalance of heavy items, paper Section 3.2).
constexpr int HW = 8;

template <int KP, bool BF16>
__global__ __launch_bounds__(64 * HW) void rows_heavy_kernel(SideArgs a, int K, float alpha, float rbar,
                                                             HyperDev hyp, DrawSrc draws, int32_t *fb_list,
                                                             DevState *state, int side)
{
    using S = RowShape<KP>;
    constexpr int TE = S::NTILE * 16;  // accumulator floats per lane
    __shared__ __attribute__((aligned(16))) float u[HW][S::UNION];
    __shared__ __attribute__((aligned(16))) float rv[HW][64];
    __shared__ __attribute__((aligned(16))) float red[HW / 2][TE * 64];
    __shared__ float bred[HW / 2][64];
    __shared__ __attribute__((aligned(16))) float colbuf[3 * KP];
    __shared__ int sidx[HW][16];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row = a.order[blockIdx.x];
    const int64_t s0 = a.ptr[row], n = a.ptr[row + 1] - s0;
    const int64_t b0 = s0 + n * wave / HW, b1 = s0 + n * (wave + 1) / HW;
    const float *vals = (const float *)a.val;

    floatx16 acc[S::NTILE];
#pragma unroll
    for (int t = 0; t < S::NTILE; ++t)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[t][e] = 0.0f;
    float bacc = 0.0f;
    if constexpr (BF16)
        gram_bf16<KP, WaveSync>(a.idx + b0, vals + b0, b1 - b0, a.other_bf16, a.shadow_stride, (int32_t)a.n_other,
                                rbar, (char *)u[wave], (uint32_t *)rv[wave], acc, bacc);
    else
        gram_f32<KP, WaveSync>(a.idx + b0, vals + b0, b1 - b0, (const float *)a.other, K, rbar, u[wave], rv[wave],
                               sidx[wave], acc, bacc);

    // fixed-order tree: at each level the upper half of the active wavefronts
    // hands its sums to the lower half
#pragma unroll
    for (int half = HW / 2; half >= 1; half /= 2) {
        if (wave >= half && wave < 2 * half) {
            float *dst = red[wave - half];
#pragma unroll
            for (int t = 0; t < S::NTILE; ++t)
#pragma unroll
                for (int e = 0; e < 16; e += 4)
                    *(float4 *)(dst + ((t * 16 + e) * 64 + lane * 4)) =
                        make_float4(acc[t][e], acc[t][e + 1], acc[t][e + 2], acc[t][e + 3]);
            bred[wave - half][lane] = bacc;
        }
        __syncthreads();
        if (wave < half) {
            const float *src = red[wave];
#pragma unroll
            for (int t = 0; t < S::NTILE; ++t)
#pragma unroll
                for (int e = 0; e < 16; e += 4) {
                    const float4 q = *(const float4 *)(src + ((t * 16 + e) * 64 + lane * 4));
                    acc[t][e] += q.x;
                    acc[t][e + 1] += q.y;
                    acc[t][e + 2] += q.z;
                    acc[t][e + 3] += q.w;
                }
            bacc += bred[wave][lane];
        }
        __syncthreads();
    }
    if (wave != 0) return;

    float *tri = u[0];
    store_precision_tri<KP>(tri, acc, alpha, hyp.Lambda_tri);
    const int ri = lane % KP;
    const float bb = fmaf(alpha, bacc, hyp.Lmu_f[ri < K ? ri : 0]) * (ri < K ? 1.0f : 0.0f);
    float z;
    if (draws.tape_rows) {
        z = (ri < K) ? (float)draws.tape_rows[(int64_t)row * K + ri] : 0.0f;
    } else {
        const uint32_t h = half_sweep_index(draws);
        if (lane < KP / 2) {
            float z0, z1;
            box_muller_f32(philox4x32_10(ctr4((uint32_t)lane, (uint32_t)row, h, 0u), draws.seed), z0, z1);
            colbuf[2 * lane] = z0;
            colbuf[2 * lane + 1] = z1;
        }
        WaveSync::sync();
        z = (ri < K) ? colbuf[ri] : 0.0f;
    }
    WaveSync::sync();
    bool fail;
    const float x = chol_solve<KP, WaveSync>(tri, colbuf, K, bb, z, fail);
    if (!fail) {
        float *X = (float *)a.X;
        if (lane < KP && ri < K) X[(int64_t)row * K + ri] = x;
        if (a.X_bf16 && lane < KP)
            a.X_bf16[(int64_t)row * a.shadow_stride + ri] = ri < K ? f32_to_bf16_rne(x) : (uint16_t)0;
    } else if (lane == 0) {
        const int pos = atomicAdd(&state->fb_count[side], 1);
        fb_list[pos] = row;
    }
}

}  // namespace

int heavy_min_ratings() { return 2048; }

hipError_t launch_rows_heavy(const SideArgs &a, int K, int KP, int bf16, double alpha, double rbar, HyperDev hyp,
                             DrawSrc draws, int32_t *fb_list, DevState *state, hipStream_t s)
{
    if (a.n_rows <= 0) return hipSuccess;
    const dim3 grid((unsigned)a.n_rows), block(64 * HW);
    const float fa = (float)alpha, fr = (float)rbar;
    if (KP == 64) {
        if (bf16) hipLaunchKernelGGL((rows_heavy_kernel<64, true>), grid, block, 0, s, a, K, fa, fr, hyp, draws, fb_list, state, draws.side);
        else hipLaunchKernelGGL((rows_heavy_kernel<64, false>), grid, block, 0, s, a, K, fa, fr, hyp, draws, fb_list, state, draws.side);
    } else if (KP == 32) {
        if (bf16) hipLaunchKernelGGL((rows_heavy_kernel<32, true>), grid, block, 0, s, a, K, fa, fr, hyp, draws, fb_list, state, draws.side);
        else hipLaunchKernelGGL((rows_heavy_kernel<32, false>), grid, block, 0, s, a, K, fa, fr, hyp, draws, fb_list, state, draws.side);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_rows_mixed(const SideArgs &a, int K, int KP, int bf16, double alpha, double rbar,
                             HyperDev hyp, DrawSrc draws, int32_t *fb_list, DevState *state,
                             hipStream_t s)
{
    if (a.n_rows <= 0) return hipSuccess;
    const dim3 grid((unsigned)a.n_rows), block(64);
    const float fa = (float)alpha, fr = (float)rbar;
    if (KP == 64) {
        if (bf16) hipLaunchKernelGGL((rows_mixed_kernel<64, true>), grid, block, 0, s, a, K, fa, fr, hyp, draws, fb_list, state, draws.side);
        else hipLaunchKernelGGL((rows_mixed_kernel<64, false>), grid, block, 0, s, a, K, fa, fr, hyp, draws, fb_list, state, draws.side);
    } else if (KP == 32) {
        if (bf16) hipLaunchKernelGGL((rows_mixed_kernel<32, true>), grid, block, 0, s, a, K, fa, fr, hyp, draws, fb_list, state, draws.side);
        else hipLaunchKernelGGL((rows_mixed_kernel<32, false>), grid, block, 0, s, a, K, fa, fr, hyp, draws, fb_list, state, draws.side);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace bpmf
