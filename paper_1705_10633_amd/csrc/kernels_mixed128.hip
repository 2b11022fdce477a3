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
//    v_mfma_f32_16x16x32_bf16, 32 features per wavefront;
//  * wavefront 0 factors P11 with the 64-wide row-per-lane Cholesky and
//    carries the forward solve of block 1 along, panel by panel; wavefront 1
//    solves for L21 (a row per lane) one 8-column panel behind it, and
//    wavefronts 2 and 3 accumulate L21 L21^T on FP32 matrix cores one more
//    panel behind; wavefront 2 then factors the updated P22 with the forward
//    solve of block 2 carried along, and solves back; wavefront 0 finishes
//    block 1.
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
    // hi pairs, lo pairs, zero words of the chunk's r' (the right-hand side's A operand)
    __shared__ __attribute__((aligned(16))) uint32_t rvp[3 * CH2 / 2];
    __shared__ float red[4];
    __shared__ int fails[2];

    const int tid = threadIdx.x, lane = tid & 63;
    // wavefront index in a scalar register: the branches on it are uniform,
    // so the barriers inside them are executed by whole wavefronts
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
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
    // right-hand side: wavefront w collects features 32 w .. 32 w + 31 as two
    // 16-feature groups on v_mfma_f32_16x16x32_bf16 (A: row 0 the hi parts of
    // 32 ratings, row 1 their lo parts, rows 2..15 zero; B: the staged features)
    floatx4 bq[2];
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
        for (int e = 0; e < 4; ++e) bq[g][e] = 0.0f;
    if (tid < CH2 / 2) rvp[CH2 + tid] = 0u;
    const uint4 *aop = (const uint4 *)(rvp + (lane % 16 < 2 ? lane % 16 : 2) * (CH2 / 2)) + lane / 16;
    char *stage = (char *)u;
    const int fb = tid / RG2, rg = tid % RG2;
    static_assert(CH2 == bf16_chunk(K2), "records are padded to the kernel's chunk");
    // 32-bit byte offsets from the uniform base (the host keeps each side
    // below 2^24 rows): one multiply-add per load
    const char *base = (const char *)src;
    const uint32_t fbb = 16u * (uint32_t)fb;
    auto load_rows = [&](const uint4 &c, uint4 *d) {
        d[0] = *(const uint4 *)(base + (__umul24(c.x, 2u * K2) + fbb));
        d[1] = *(const uint4 *)(base + (__umul24(c.y, 2u * K2) + fbb));
        d[2] = *(const uint4 *)(base + (__umul24(c.z, 2u * K2) + fbb));
        d[3] = *(const uint4 *)(base + (__umul24(c.w, 2u * K2) + fbb));
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
            lo.x = __builtin_amdgcn_perm(w1[w], w0[w], 0x05040100u);
            lo.y = __builtin_amdgcn_perm(w3[w], w2[w], 0x05040100u);
            hi.x = __builtin_amdgcn_perm(w1[w], w0[w], 0x07060302u);
            hi.y = __builtin_amdgcn_perm(w3[w], w2[w], 0x07060302u);
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
#pragma unroll
        for (int ks = 0; ks < CH2 / 32; ++ks) {
            const bf16x8_t Ar = *(const bf16x8_t *)(aop + 4 * ks);
#pragma unroll
            for (int g = 0; g < 2; ++g) {
                const int f = 32 * wave + 16 * g + lane % 16;
                const bf16x8_t Bf = *(const bf16x8_t *)(stage + f * SB2 + (ks * 32 + (lane / 16) * 8) * 2);
                bq[g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ar, Bf, bq[g], 0, 0, 0);
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
            // the tile's 16 entries of Lambda are requested together, before
            // any of them is used: interleaved with the stores, each load
            // was issued only after the previous one had returned
            float lam[16];
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = 32 * ta + 8 * j + 4 * (lane >> 5) + i;
                    const int c = 32 * tb + (lane & 31);
                    lam[4 * j + i] = hyp.Lambda_tri[rowoff(r) + c];  // < PTRI2 + K2 for every lane
                }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = 32 * ta + 8 * j + 4 * (lane >> 5) + i;
                    const int c = 32 * tb + (lane & 31);
                    const int e = rowoff(r) + c;
                    const float val = fmaf(alpha, acc[t][4 * j + i], lam[4 * j + i]);
                    // above the diagonal: a slot in the padding after the
                    // triangle, so the store (and the load) stay unconditional
                    P[c <= r ? e : PTRI2 + lane] = val;
                }
        }
    }
    {
        // lane c < 16 of bq[g] holds the hi (element 0) and lo (element 1)
        // sums of feature 32 wave + 16 g + c
        const float v0 = __shfl(bq[0][0] + bq[0][1], lane % 16), v1 = __shfl(bq[1][0] + bq[1][1], lane % 16);
        if (lane < 32) {
            const int f = 32 * wave + lane;
            bvec[f] = fmaf(alpha, lane < 16 ? v0 : v1, hyp.Lmu_f[f < K ? f : 0]) * (f < K ? 1.0f : 0.0f);
        }
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

    // ---------------- block 1 and P22 - L21 L21^T, panel by panel ----------------
    // Eight steps of 8 columns; at each step, on its own wavefront:
    //  * wavefront 0 factors the panel of P11 with the 64-wide row-per-lane
    //    Cholesky, publishes its columns of L11 into the packed triangle (over
    //    P11, lower part only) and carries the forward solve y1 = L11^{-1} b1
    //    over the panel (y_k = t_k / L_kk, then t -= L[:, k] y_k);
    //  * wavefront 1, one step behind, solves the same columns of
    //    L21 = P21 L11^{-T} right-looking from the published panel, carries
    //    b2 - L21 y1 over them and publishes them over P21;
    //  * wavefronts 2 and 3, one more step behind, accumulate the panel's
    //    rank-8 part of L21 L21^T on FP32 matrix cores (wavefront 2 the
    //    diagonal tiles, wavefront 3 the off-diagonal one).
    // The branch on the wavefront is uniform and every path passes the same
    // ten barriers.
    auto publish = [&](const float (&A)[H2], int c0) {
#pragma unroll
        for (int c = c0; c < c0 + 8; ++c)
            if (c <= lane) P[rowoff(lane) + c] = A[c];
    };
    // forward solve over columns c0..c0+7 of the factored rows in A
    auto fwd_panel = [&](const float (&A)[H2], float &t, const float *inv, float *ybuf, int c0) {
#pragma unroll
        for (int k = c0; k < c0 + 8; ++k) {
            const float yk = readlane_f(t, k) * inv[k];
            ybuf[k] = yk;
            t = fmaf(-A[k], yk, t);
        }
    };
    if (wave == 0) {
        float A[H2];
#pragma unroll
        for (int c = 0; c < H2; ++c) A[c] = P[rowoff(lane) + c];
        float t = bvec[lane];
#define W0_STEP(Q)                                   \
    chol64_step<Q, WaveSync>(A, inv11, pb);              \
    publish(A, 8 * (Q));                             \
    fwd_panel(A, t, inv11, y1, 8 * (Q));             \
    __syncthreads();
        W0_STEP(0) W0_STEP(1) W0_STEP(2) W0_STEP(3) W0_STEP(4) W0_STEP(5) W0_STEP(6) W0_STEP(7)
#undef W0_STEP
        const bool f0 = chol_pivots_fail(inv11[lane], lane, K < H2 ? K : H2, tau);
        if (lane == 0) fails[0] = f0 ? 1 : 0;
        __syncthreads();
        __syncthreads();
    } else if (wave == 1) {
        float A[H2];
#pragma unroll
        for (int c = 0; c < H2; ++c) A[c] = P[rowoff(H2 + lane) + c];
        float t = bvec[H2 + lane];
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
                float u = A[j];
#pragma unroll
                for (int k = 0; k < 8; ++k) u = fmaf(-A[c0 + k], lj[k], u);
                A[j] = u;
            }
#pragma unroll
            for (int k = c0; k < c0 + 8; ++k) {
                t = fmaf(-A[k], y1[k], t);
                P[rowoff(H2 + lane) + k] = A[k];
            }
        };
#define W1_STEP(Q)   \
    __syncthreads(); \
    trsm_panel(8 * (Q));
        W1_STEP(0) W1_STEP(1) W1_STEP(2) W1_STEP(3) W1_STEP(4) W1_STEP(5) W1_STEP(6) W1_STEP(7)
#undef W1_STEP
        b2[lane] = t;
        __syncthreads();
        __syncthreads();
    } else {
        // wavefront 2: tiles (0, 0) and (1, 1) of C = L21 L21^T; wavefront 3:
        // tile (1, 0).  Operand lane l holds L21[32 a + l % 32][k + l / 32]
        // (read from the published panels); result element 4j + i of lane l
        // is C[32 a + 8j + 4(l / 32) + i][32 b + l % 32].
        const bool w2 = wave == 2;
        const float *r0 = P + rowoff(H2 + (lane & 31)) + (lane >> 5);
        const float *r1 = P + rowoff(H2 + 32 + (lane & 31)) + (lane >> 5);
        floatx16 c0 = {}, c1 = {};
        auto syrk_panel = [&](int k0) {
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const float x0 = r0[k0 + 2 * kk], x1 = r1[k0 + 2 * kk];
                if (w2) {
                    c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(x0, x0, c0, 0, 0, 0);
                    c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(x1, x1, c1, 0, 0, 0);
                } else {
                    c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(x1, x0, c0, 0, 0, 0);
                }
            }
        };
#define W23_STEP(Q)                          \
    __syncthreads();                         \
    if ((Q) >= 1) syrk_panel(8 * ((Q) - 1));
        W23_STEP(0) W23_STEP(1) W23_STEP(2) W23_STEP(3) W23_STEP(4) W23_STEP(5) W23_STEP(6) W23_STEP(7)
#undef W23_STEP
        __syncthreads();
        syrk_panel(56);
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int m = 8 * j + 4 * (lane >> 5) + i, n = lane & 31;
                if (w2) {
                    if (n <= m) {
                        P[rowoff(H2 + m) + H2 + n] -= c0[4 * j + i];
                        P[rowoff(H2 + 32 + m) + H2 + 32 + n] -= c1[4 * j + i];
                    }
                } else {
                    P[rowoff(H2 + 32 + m) + H2 + n] -= c0[4 * j + i];
                }
            }
        __syncthreads();
    }

    // ---------------- block 2: L22, y2, x2 (wavefront 2) ----------------
    if (wave == 2) {
        float A[H2];
#pragma unroll
        for (int c = 0; c < H2; ++c) A[c] = P[rowoff(H2 + lane) + H2 + c];
        float t = b2[lane];
        WaveSync::sync();
#define W2_STEP(Q)                     \
    chol64_step<Q, WaveSync>(A, inv22, pb); \
    fwd_panel(A, t, inv22, yb2, 8 * (Q));
        W2_STEP(0) W2_STEP(1) W2_STEP(2) W2_STEP(3) W2_STEP(4) W2_STEP(5) W2_STEP(6) W2_STEP(7)
#undef W2_STEP
        const float iv = inv22[lane];
        const bool f2 = chol_pivots_fail(iv, lane, K - H2, tau);
        if (lane == 0) fails[1] = f2 ? 1 : 0;
        // masked: past its diagonal a row would run into the next row's L21
        store_rows_lower<H2, H2>(A, P + P22OFF);
        WaveSync::sync();
        const float y = yb2[lane];
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
