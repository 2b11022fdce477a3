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

// Rows with many ratings are cut into pieces that run as their own entries
// of the launch table (first, so they start before the rows): a piece
// writes its partial Gram tiles and right-hand side to `part`.  A second,
// short launch (`combine`) sums each heavy row's pieces in piece order (so
// the result does not depend on timing) and factors and samples the row.
// One wavefront per heavy row would leave a row with thousands of ratings
// running long after the rest of the launch (the load imbalance of heavy
// items, paper Section 3.2).
// Kernel variants (bpmf_launch_shape::kernel_variant; KP = 64 only): MT
// selects the matrix-core trailing updates of chol_factor, W the
// wavefronts per SIMD the register allocation is held to (W = 4: at most 128
// VGPRs; W = 3: 168).
template <int KP, bool BF16, bool MT = true, int W = 4>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(W, W))) void rows_mixed_kernel(SideArgs a, int K, float ialpha, float rsalpha, float rbar,
                                                        HyperDev hyp, DrawSrc draws,
                                                        int32_t *fb_list, DevState *state,
                                                        int side, PieceArgs pc)
{
    using S = RowShape<KP>;
    constexpr int PW = piece_floats(KP);
    __shared__ __attribute__((aligned(16))) float u[S::UNION];
    __shared__ __attribute__((aligned(16))) float rv[96];
    __shared__ __attribute__((aligned(16))) float colbuf[3 * KP];
    __shared__ int sidx[16];

    const int lane = threadIdx.x;
    const float *vals = (const float *)a.val;

    // The row is sampled from P / alpha = Lambda / alpha + G, whose factor is
    // chol(P) / sqrt(alpha): with b / alpha and z / sqrt(alpha) in place of b
    // and z the solves give the same x.  A row's Gram accumulators start from
    // Lambda / alpha (in their own layout); a piece's, and a combined heavy
    // row's, from zero.
    // BF16 at KP = 64: the ten lower 16 x 16 tiles (GramAcc)
    using Acc = GramAcc<KP, BF16 && KP == 64>;
    Acc acc;
    float bacc = 0.0f;
    auto clear_acc = [&]() {
#pragma unroll
        for (int i = 0; i < Acc::N; ++i) acc.set(i, 0.0f);
    };
    auto lambda_acc = [&]() {
#pragma unroll
        for (int i = 0; i < Acc::N; ++i) acc.set(i, hyp.Lambda_acc[i * 64 + lane]);
    };

    int row;
    if (pc.combine) {
        clear_acc();
        // {row, first piece, piece count, -}
        const int4 ct = pc.ctab[blockIdx.x];
        row = ct.x;
        for (int p = ct.y; p < ct.y + ct.z; ++p) {
            const float *src = pc.part + (int64_t)p * PW;
#pragma unroll
            for (int i = 0; i < Acc::N; ++i) acc.set(i, acc.get(i) + src[i * 64 + lane]);
            bacc += src[Acc::N * 64 + lane];
        }
    } else {
        // {row, rating count, first rating (low, high word)}; row < 0: piece -row - 1
        const int4 rt = a.rowtab[blockIdx.x];
        row = rt.x;
        const int64_t s0 = (int64_t)(((uint64_t)(uint32_t)rt.w << 32) | (uint32_t)rt.z), s1 = s0 + rt.y;
        if (row >= 0)
            lambda_acc();
        else
            clear_acc();
        if constexpr (BF16)
            gram_bf16<KP>(a.rec + 2 * a.recoff[blockIdx.x], s1 - s0, a.other_bf16, a.shadow_stride, (char *)u,
                          (uint32_t *)rv, acc, bacc);
        else
            gram_f32<KP>(a.idx + s0, vals + s0, s1 - s0, (const float *)a.other, K, rbar, u, rv,
                         sidx, acc.t, bacc);
        if (row < 0) {
            float *dst = pc.part + (int64_t)(-row - 1) * PW;
#pragma unroll
            for (int i = 0; i < Acc::N; ++i) dst[i * 64 + lane] = acc.get(i);
            dst[Acc::N * 64 + lane] = bacc;
            return;
        }
    }

    float *tri = u;
    if (pc.combine)
        store_precision_tri<KP, true>(tri, acc, hyp.Lambda_acc);
    else
        store_precision_tri<KP, false>(tri, acc, hyp.Lambda_acc);
    const int ri = lane % KP;
    // b / alpha; an unconditional load and a multiplicative mask: as a select,
    // the load would be moved behind a branch with its own wait
    const float bb = fmaf(hyp.Lmu_f[ri < K ? ri : 0], ialpha, bacc) * (ri < K ? 1.0f : 0.0f);

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
    const float x = chol_solve<KP, BlockSync, MT>(tri, colbuf, K, bb, z * rsalpha, fail);
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

// One workgroup per launch-table entry: its ratings as packed records (see
// SideArgs::rec), padded to a multiple of `chunk` ratings.  r' = r - rbar and
// its BF16 parts are formed exactly as a row kernel would form them from the
// FP32 rating, so the records change no result.
__global__ __launch_bounds__(256) void build_records_kernel(const int4 *rowtab, const int64_t *recoff,
                                                            const int32_t *idx, const float *vals, float rbar,
                                                            int32_t sentinel, int chunk, uint4 *rec)
{
    const int4 rt = rowtab[blockIdx.x];
    const int64_t s0 = (int64_t)(((uint64_t)(uint32_t)rt.w << 32) | (uint32_t)rt.z), cnt = rt.y;
    const int64_t groups = (cnt + chunk - 1) / chunk * (chunk / 4);
    uint4 *out = rec + 2 * recoff[blockIdx.x];
    for (int64_t g = threadIdx.x; g < groups; g += blockDim.x) {
        uint32_t c[4], hi[4], lo[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t n = 4 * g + q;
            const bool ok = n < cnt;
            c[q] = ok ? (uint32_t)idx[s0 + n] : (uint32_t)sentinel;
            const float v = ok ? vals[s0 + n] - rbar : 0.0f;
            hi[q] = f32_to_bf16_rne(v);
            lo[q] = f32_to_bf16_rne(v - bf16_to_f32((uint16_t)hi[q]));
        }
        out[2 * g] = make_uint4(c[0], c[1], c[2], c[3]);
        out[2 * g + 1] = make_uint4(hi[0] | (hi[1] << 16), hi[2] | (hi[3] << 16), lo[0] | (lo[1] << 16),
                                    lo[2] | (lo[3] << 16));
    }
}

}  // namespace

hipError_t launch_build_records(const SideArgs &a, int64_t n_entries, int chunk, float rbar, uint4 *rec,
                                hipStream_t s)
{
    if (n_entries <= 0) return hipSuccess;
    hipLaunchKernelGGL(build_records_kernel, dim3((unsigned)n_entries), dim3(256), 0, s, a.rowtab, a.recoff, a.idx,
                       (const float *)a.val, rbar, (int32_t)a.n_other, chunk, rec);
    return hipGetLastError();
}

int heavy_min_ratings() { return 2048; }

hipError_t launch_rows_mixed(const SideArgs &a, int K, int KP, int bf16, double alpha, double rbar,
                             HyperDev hyp, DrawSrc draws, int32_t *fb_list, DevState *state,
                             PieceArgs pc, int64_t n_entries, int variant, hipStream_t s)
{
    if (n_entries <= 0) return hipSuccess;
    const dim3 grid((unsigned)n_entries), block(64);
    const float fia = (float)(1.0 / alpha), frsa = (float)(1.0 / std::sqrt(alpha)), fr = (float)rbar;
#define BPMF_ROWS_MIXED(...) hipLaunchKernelGGL((rows_mixed_kernel<__VA_ARGS__>), grid, block, 0, s, a, K, fia, frsa, fr, \
                                                hyp, draws, fb_list, state, draws.side, pc)
    if (KP == 64) {
        // 1: matrix-core trailing updates, 4 wavefronts per SIMD (built-in);
        // 2: vector-unit updates within each 32-column half; 3: as 1 with 3
        // wavefronts per SIMD
        if (bf16) {
            if (variant == 2) BPMF_ROWS_MIXED(64, true, false, 4);
            else if (variant == 3) BPMF_ROWS_MIXED(64, true, true, 3);
            else BPMF_ROWS_MIXED(64, true, true, 4);
        } else {
            if (variant == 2) BPMF_ROWS_MIXED(64, false, false, 4);
            else if (variant == 3) BPMF_ROWS_MIXED(64, false, true, 3);
            else BPMF_ROWS_MIXED(64, false, true, 4);
        }
    } else if (KP == 32) {
        if (bf16) BPMF_ROWS_MIXED(32, true);
        else BPMF_ROWS_MIXED(32, false);
    } else {
        return hipErrorInvalidValue;
    }
#undef BPMF_ROWS_MIXED
    return hipGetLastError();
}

}  // namespace bpmf
