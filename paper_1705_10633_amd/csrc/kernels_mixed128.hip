// kernels_mixed128.hip -- mixed-precision row update for 64 < K <= 128 (BF16
// gathers), one 256-thread workgroup per row.
//
// The same conditional as the other row kernels (paper: Section 2 and
// Algorithm 1; Cholesky instead of an inverse, Section 3.1):
//   P = Lambda + alpha G,  G = sum_{j in Omega_i} v_j v_j^T,
//   b = Lambda mu + alpha sum_j (r_ij - rbar) v_j,  x_i = L^{-T}(L^{-1} b + z_i),
// with K padded to 128 (identity block) and P factored in 64-blocks:
//   L11 = chol(P11),  L21 = P21 L11^{-T},  L22 = chol(P22 - L21 L21^T),
//   y1 = L11^{-1} b1,  y2 = L22^{-1}(b2 - L21 y1),
//   x2 = L22^{-T}(y2 + z2),  x1 = L11^{-T}(y1 + z1 - L21^T x2).
//
// gfx950 mapping:
//  * gather: each thread fetches 16-byte pieces of 4 rated rows (BF16 copy,
//    row stride 128); chunks of 64 ratings are staged feature-major in LDS;
//  * Gram: the ten lower 32 x 32 tiles on v_mfma_f32_32x32x16_bf16, three,
//    three, two and two tiles on the four wavefronts; the right-hand side on
//    v_dot2c_f32_bf16 (threads 0..127, one feature each);
//  * wavefront 0 factors P11 with the 64-wide row-per-lane Cholesky and does
//    the forward solve of block 1, while wavefront 1 solves for L21 (a row
//    per lane) one 8-column panel behind it; wavefronts 1..3 form one tile
//    each of L21 L21^T on FP32 matrix cores; wavefront 2 factors the updated
//    P22 and solves block 2; wavefront 0 finishes block 1.
//  * a row whose pivot is not finite or not above 64 K 2^-24 max_k P_kk is
//    not written; it is appended to the FP64 recompute list.
#include "common.hpp"
#include "rng.hpp"
#include "rowsolve.hpp"

namespace bpmf {

namespace {

constexpr int K2 = 128;                       // padded size
constexpr int H2 = 64;                        // block size
constexpr int T2 = 256;                       // threads per row
constexpr int FB2 = K2 / 8;                   // 8-feature blocks
constexpr int RG2 = T2 / FB2;                 // 4-rating groups per chunk
constexpr int CH2 = 4 * RG2;                  // ratings per chunk (64)
constexpr int SB2 = CH2 * 2 + 16;             // bytes per staged feature row
constexpr int PTRI2 = K2 * (K2 + 1) / 2;      // packed lower triangle of P
constexpr int STAGE2 = K2 * SB2 / 4;          // staging (floats)
constexpr int U2 = (PTRI2 + K2) > STAGE2 ? (PTRI2 + K2) : STAGE2;
// L22 is stored in place of P22: row q of the block starts at
// rowoff(H2 + q) + H2 = P22OFF + q (q + 1) / 2 + H2 q
constexpr int P22OFF = H2 * (H2 + 1) / 2 + H2;

__device__ __forceinline__ int rowoff(int r) { return r * (r + 1) / 2; }

// Lower 32 x 32 tiles (a, b) of the 128 x 128 Gram, by wavefront:
// wave 0: (0,0) (1,0) (1,1); wave 1: (2,0) (2,1) (2,2); wave 2: (3,0) (3,1);
// wave 3: (3,2) (3,3).  `wave` is uniform, so these are scalar selects.
__device__ __forceinline__ void tile_of(int wave, int t, int &a, int &b)
{
    a = wave == 0 ? (t == 0 ? 0 : 1) : (wave == 1 ? 2 : 3);
    b = wave == 0 ? (t == 2 ? 1 : 0) : (wave == 3 ? 2 + t : t);
}

__global__ __launch_bounds__(T2) __attribute__((amdgpu_waves_per_eu(4, 4))) void rows_mixed128_kernel(
    SideArgs sa, int K, float alpha, float rbar, HyperDev hyp, DrawSrc draws, int32_t *fb_list,
    DevState *state, int side)
{
    __shared__ __attribute__((aligned(16))) float u[U2];     // staging, then P (packed), then L11 / L21 in place
    // panel buffer of the two 64-wide factorisations (never at the same time)
    __shared__ __attribute__((aligned(16))) float pb[H2 * 12];
    __shared__ __attribute__((aligned(16))) float bvec[K2], zvec[K2];
    __shared__ __attribute__((aligned(16))) float y1[H2], b2[H2], x2v[H2], inv11[H2], inv22[H2], yb2[H2],
        xb2[H2], xb0[H2];
    __shared__ __attribute__((aligned(16))) uint32_t rvp[CH2];
    __shared__ float red[4];
    __shared__ int fails[2];

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int4 rt = sa.rowtab[blockIdx.x];
    const int row = rt.x;
    const int64_t nnz = rt.y;
    const uint16_t *src = sa.other_bf16;

    // ---------------- Gram (matrix cores) and right-hand side ----------------
    // Records (SideArgs::rec, padded to 64-rating chunks): per 4 ratings the
    // column indices and the two-part BF16 offsets r - rbar.
    const int ntile = wave < 2 ? 3 : 2;
    floatx16 acc[3];
#pragma unroll
    for (int t = 0; t < 3; ++t)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[t][e] = 0.0f;
    float bacc = 0.0f;
    char *stage = (char *)u;
    const int fb = tid / RG2, rg = tid % RG2;
    static_assert(CH2 == bf16_chunk(K2), "records are padded to the kernel's chunk");
    auto load_rows = [&](const uint4 &c, uint4 *d) {
        d[0] = *(const uint4 *)(src + (int64_t)(int)c.x * K2 + fb * 8);
        d[1] = *(const uint4 *)(src + (int64_t)(int)c.y * K2 + fb * 8);
        d[2] = *(const uint4 *)(src + (int64_t)(int)c.z * K2 + fb * 8);
        d[3] = *(const uint4 *)(src + (int64_t)(int)c.w * K2 + fb * 8);
    };
    auto stage_chunk = [&](const uint4 *d, const uint4 &rp) {
        if (fb == 0) {
            *(uint2 *)(rvp + rg * 2) = make_uint2(rp.x, rp.y);
            *(uint2 *)(rvp + CH2 / 2 + rg * 2) = make_uint2(rp.z, rp.w);
        }
        const uint32_t w0[4] = {d[0].x, d[0].y, d[0].z, d[0].w};
        const uint32_t w1[4] = {d[1].x, d[1].y, d[1].z, d[1].w};
        const uint32_t w2[4] = {d[2].x, d[2].y, d[2].z, d[2].w};
        const uint32_t w3[4] = {d[3].x, d[3].y, d[3].z, d[3].w};
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const int f = fb * 8 + 2 * w;
            uint2 lo, hi;
            lo.x = (w0[w] & 0xffffu) | (w1[w] << 16);
            lo.y = (w2[w] & 0xffffu) | (w3[w] << 16);
            hi.x = (w0[w] >> 16) | (w1[w] & 0xffff0000u);
            hi.y = (w2[w] >> 16) | (w3[w] & 0xffff0000u);
            *(uint2 *)(stage + f * SB2 + rg * 8) = lo;
            *(uint2 *)(stage + (f + 1) * SB2 + rg * 8) = hi;
        }
    };
    auto multiply_chunk = [&]() {
#pragma unroll
        for (int ks = 0; ks < CH2 / 16; ++ks) {
            const int off = (ks * 16 + (lane >> 5) * 8) * 2;
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                if (t < ntile) {
                    int ta, tb;
                    tile_of(wave, t, ta, tb);
                    const bf16x8_t Fa = *(const bf16x8_t *)(stage + (32 * ta + (lane & 31)) * SB2 + off);
                    const bf16x8_t Fb = *(const bf16x8_t *)(stage + (32 * tb + (lane & 31)) * SB2 + off);
                    acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Fa, Fb, acc[t], 0, 0, 0);
                }
            }
        }
        if (tid < K2) {
            const uint4 *sp = (const uint4 *)(stage + tid * SB2);
            const uint4 *hp = (const uint4 *)rvp, *lp = (const uint4 *)(rvp + CH2 / 2);
#pragma unroll
            for (int p4 = 0; p4 < CH2 / 8; ++p4) {
                const uint4 sv = sp[p4], hv = hp[p4], lv = lp[p4];
                const uint32_t sa4[4] = {sv.x, sv.y, sv.z, sv.w};
                const uint32_t ha[4] = {hv.x, hv.y, hv.z, hv.w};
                const uint32_t la[4] = {lv.x, lv.y, lv.z, lv.w};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    bf16x2_t x, yh, yl;
                    __builtin_memcpy(&x, &sa4[q], 4);
                    __builtin_memcpy(&yh, &ha[q], 4);
                    __builtin_memcpy(&yl, &la[q], 4);
                    bacc = __builtin_amdgcn_fdot2_f32_bf16(x, yh, bacc, false);
                    bacc = __builtin_amdgcn_fdot2_f32_bf16(x, yl, bacc, false);
                }
            }
        }
    };
    {
        const int64_t nch = (nnz + CH2 - 1) / CH2;
        const uint4 *r0 = sa.rec + 2 * (sa.recoff[blockIdx.x] + rg);
        uint4 d[4], rpc, nc, nr;
        if (nch > 0) {
            nc = r0[0];
            rpc = r0[1];
            load_rows(nc, d);
            if (nch > 1) {
                nc = r0[2 * RG2];
                nr = r0[2 * RG2 + 1];
            }
        }
        for (int64_t c = 0; c < nch; ++c) {
            stage_chunk(d, rpc);
            if (c + 1 < nch) {
                load_rows(nc, d);
                rpc = nr;
                if (c + 2 < nch) {
                    nc = r0[2 * RG2 * (c + 2)];
                    nr = r0[2 * RG2 * (c + 2) + 1];
                }
            }
            __syncthreads();
            multiply_chunk();
            __syncthreads();
        }
    }

    // ---------------- P = Lambda + alpha G, b, z ----------------
    float *P = u;
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        if (t < ntile) {
            int ta, tb;
            tile_of(wave, t, ta, tb);
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = 32 * ta + 8 * j + 4 * (lane >> 5) + i;
                    const int c = 32 * tb + (lane & 31);
                    const int e = rowoff(r) + c;  // < PTRI2 + K2 for every lane
                    const float val = fmaf(alpha, acc[t][4 * j + i], hyp.Lambda_tri[e]);
                    // above the diagonal: a slot in the padding after the
                    // triangle, so the store (and the load) stay unconditional
                    P[c <= r ? e : PTRI2 + lane] = val;
                }
        }
    }
    if (tid < K2) {
        bvec[tid] = fmaf(alpha, bacc, hyp.Lmu_f[tid < K ? tid : 0]) * (tid < K ? 1.0f : 0.0f);
    }
    if (draws.tape_rows) {
        if (tid < K2) zvec[tid] = tid < K ? (float)draws.tape_rows[(int64_t)row * K + (tid < K ? tid : 0)] : 0.0f;
    } else if (tid < K2 / 2) {
        const uint32_t h = half_sweep_index(draws);
        float z0, z1;
        box_muller_f32(philox4x32_10(ctr4((uint32_t)tid, (uint32_t)row, h, 0u), draws.seed), z0, z1);
        zvec[2 * tid] = 2 * tid < K ? z0 : 0.0f;
        zvec[2 * tid + 1] = 2 * tid + 1 < K ? z1 : 0.0f;
    }
    __syncthreads();
    // tau = 64 K 2^-24 max_{k<K} P_kk
    if (wave < 2) {
        const int k = tid;
        float dg = k < K ? P[rowoff(k) + k] : 0.0f;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) dg = fmaxf(dg, __shfl_xor(dg, o));
        if (lane == 0) red[wave] = dg;
    }
    __syncthreads();
    const float tau = 64.0f * (float)K * 0x1.0p-24f * fmaxf(red[0], red[1]);

    // ---------------- block 1: L11 (wavefront 0) and L21 (wavefront 1), panel by panel ----------------
    // Wavefront 0 factors P11 with the 64-wide row-per-lane Cholesky in eight
    // steps of 8 columns; after step p it publishes the panel's columns of
    // L11 into the packed triangle (over P11, lower part only: entries right
    // of a row's diagonal would land in the next rows' slots).  Wavefront 1
    // keeps row r of P21 in registers and, one step behind, solves the same 8
    // columns of L21 = P21 L11^{-T} right-looking: x_k = a_k / L11_kk, then
    // a_j -= x_k L11_jk for the later columns.  Every thread passes the same
    // barriers; only the work between them differs by wavefront.
    float A[H2];
    if (wave == 0) {
#pragma unroll
        for (int c = 0; c < H2; ++c) A[c] = P[rowoff(lane) + c];
    } else if (wave == 1) {
#pragma unroll
        for (int c = 0; c < H2; ++c) A[c] = P[rowoff(H2 + lane) + c];
    }
    auto publish = [&](int c0) {
#pragma unroll
        for (int c = c0; c < c0 + 8; ++c)
            if (c <= lane) P[rowoff(lane) + c] = A[c];
    };
    auto trsm_panel = [&](int c0) {
#pragma unroll
        for (int k = c0; k < c0 + 8; ++k) {
            const float x = A[k] * inv11[k];
            A[k] = x;
#pragma unroll
            for (int j = k + 1; j < c0 + 8; ++j) A[j] = fmaf(-x, P[rowoff(j) + k], A[j]);
        }
#pragma unroll
        for (int j = c0 + 8; j < H2; ++j) {
            const float *lj = P + rowoff(j) + c0;
            float t = A[j];
#pragma unroll
            for (int k = 0; k < 8; ++k) t = fmaf(-A[c0 + k], lj[k], t);
            A[j] = t;
        }
    };
#define BLOCK1_STEP(Q)                                                   \
    if (wave == 0) {                                                     \
        chol64_step<Q, WaveSync>(A, inv11, pb);                          \
        publish(8 * (Q));                                                \
    }                                                                    \
    __syncthreads();                                                     \
    if (wave == 1) trsm_panel(8 * (Q));
    BLOCK1_STEP(0)
    BLOCK1_STEP(1)
    BLOCK1_STEP(2)
    BLOCK1_STEP(3)
    BLOCK1_STEP(4)
    BLOCK1_STEP(5)
    BLOCK1_STEP(6)
    BLOCK1_STEP(7)
#undef BLOCK1_STEP
    if (wave == 0) {
        const float iv = inv11[lane];
        const bool f0 = chol_pivots_fail(iv, lane, K < H2 ? K : H2, tau);
        if (lane == 0) fails[0] = f0 ? 1 : 0;
        forward_sub<H2, WaveSync>(A, iv, bvec[lane], y1);
    }
    __syncthreads();

    // ---------------- b2 - L21 y1 and L21 into LDS (wavefront 1) ----------------
    if (wave == 1) {
        float t = bvec[H2 + lane];
#pragma unroll
        for (int k = 0; k < H2; ++k) t = fmaf(-A[k], y1[k], t);
        b2[lane] = t;
        // L21 over P21 (the operands of L21 L21^T, then the block-1 back substitution)
#pragma unroll
        for (int c = 0; c < H2; ++c) P[rowoff(H2 + lane) + c] = A[c];
    }
    __syncthreads();

    // ---------------- P22 -= L21 L21^T: one 32 x 32 tile per wavefront 1..3 ----------------
    // Tile (a, b) of C = L21 L21^T (a, b in {0, 1}: rows 0-31 / 32-63 of L21)
    // in 32 rank-2 steps of v_mfma_f32_32x32x2_f32; operand lane l holds
    // L21[32 a + l % 32][2 kk + l / 32], read from LDS.  Result element
    // v = 4j + i of lane l is C[32 a + 8j + 4(l / 32) + i][32 b + l % 32].
    if (wave >= 1) {
        const int ta = wave == 1 ? 0 : 1, tb = wave == 3 ? 1 : 0;
        const float *ra = P + rowoff(H2 + 32 * ta + (lane & 31)) + (lane >> 5);
        const float *rb = P + rowoff(H2 + 32 * tb + (lane & 31)) + (lane >> 5);
        floatx16 c = {};
#pragma unroll
        for (int kk = 0; kk < H2 / 2; ++kk) {
            const float xa = ra[2 * kk], xb = rb[2 * kk];
            c = __builtin_amdgcn_mfma_f32_32x32x2f32(xa, xb, c, 0, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int m = 32 * ta + 8 * j + 4 * (lane >> 5) + i, n = 32 * tb + (lane & 31);
                if (n <= m) P[rowoff(H2 + m) + H2 + n] -= c[4 * j + i];
            }
    }
    __syncthreads();

    // ---------------- block 2: L22, y2, x2 (wavefront 2) ----------------
    if (wave == 2) {
#pragma unroll
        for (int c = 0; c < H2; ++c) A[c] = P[rowoff(H2 + lane) + H2 + c];
        WaveSync::sync();
        chol_factor<H2, WaveSync>(A, inv22, pb);
        const float iv = inv22[lane];
        const bool f2 = chol_pivots_fail(iv, lane, K - H2, tau);
        if (lane == 0) fails[1] = f2 ? 1 : 0;
        const float y = forward_sub<H2, WaveSync>(A, iv, b2[lane], yb2);
        // masked: past its diagonal a row would run into the next row's L21
        store_rows_lower<H2, H2>(A, P + P22OFF);
        WaveSync::sync();
        x2v[lane] = backward_sub<H2, WaveSync, H2>(P + P22OFF, iv, y + zvec[H2 + lane], xb2);
    }
    __syncthreads();

    // ---------------- block 1: x1 = L11^{-T}(y1 + z1 - L21^T x2) (wavefront 0) ----------------
    const bool fail = (fails[0] | fails[1]) != 0;
    if (wave == 0) {
        float w = y1[lane] + zvec[lane];
#pragma unroll
        for (int r = 0; r < H2; ++r) w = fmaf(-P[rowoff(H2 + r) + lane], x2v[r], w);
        const float x1 = backward_sub<H2, WaveSync>(P, inv11[lane], w, xb0);
        if (!fail) {
            float *X = (float *)sa.X;
            if (lane < K) X[(int64_t)row * K + lane] = x1;
            if (sa.X_bf16) sa.X_bf16[(int64_t)row * K2 + lane] = lane < K ? f32_to_bf16_rne(x1) : (uint16_t)0;
        }
    } else if (wave == 2 && !fail) {
        const float x2 = x2v[lane];
        float *X = (float *)sa.X;
        if (H2 + lane < K) X[(int64_t)row * K + H2 + lane] = x2;
        if (sa.X_bf16) sa.X_bf16[(int64_t)row * K2 + H2 + lane] = H2 + lane < K ? f32_to_bf16_rne(x2) : (uint16_t)0;
    }
    if (fail && tid == 0) {
        const int pos = atomicAdd(&state->fb_count[side], 1);
        fb_list[pos] = row;
    }
}

}  // namespace

hipError_t launch_rows_mixed128(const SideArgs &a, int K, double alpha, double rbar, HyperDev hyp,
                                DrawSrc draws, int32_t *fb_list, DevState *state, hipStream_t s)
{
    if (a.n_rows <= 0) return hipSuccess;
    if (K <= 64 || K > 128 || !a.other_bf16) return hipErrorInvalidValue;
    hipLaunchKernelGGL(rows_mixed128_kernel, dim3((unsigned)a.n_rows), dim3(T2), 0, s, a, K, (float)alpha,
                       (float)rbar, hyp, draws, fb_list, state, draws.side);
    return hipGetLastError();
}

}  // namespace bpmf
