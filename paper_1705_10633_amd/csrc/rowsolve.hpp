// rowsolve.hpp -- wavefront-level building blocks of the mixed-precision row
// update (one 64-lane wavefront per row, KP = 32 or 64 padded latent size):
//   gram_bf16 / gram_f32 : G = sum_j v_j v_j^T (lower 32x32 tiles) on the
//                          matrix cores and sum_j (r_j - rbar) v_j;
//   store_precision      : P = Lambda + alpha G into a packed lower triangle
//                          (padding rows/columns get the identity);
//   chol_solve           : x = L^{-T}(L^{-1} b + z) with L L^T = P, FP32,
//                          one matrix row per lane.
// The paper's row conditional (Section 2, Algorithm 1) and the choice of a
// Cholesky factorisation over an inverse (Section 3.1).
#pragma once
#include <type_traits>

#include "common.hpp"

namespace bpmf {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

template <int KP>
struct RowShape {
    static constexpr int TRI = KP * (KP + 1) / 2 + KP;   // packed lower triangle + pad
    static constexpr int FB = KP / 8;                    // 8-feature blocks per row
    static constexpr int RG = 64 / FB;                   // 4-row groups per chunk
    static constexpr int CH = 4 * RG;                    // BF16 chunk rows
    static constexpr int SB = CH * 2 + 16;               // bytes per staged feature row
    static constexpr int STAGE_BF16 = KP * SB / 4;       // floats
    static constexpr int CHF = 16;                       // FP32 chunk rows
    static constexpr int KSF = KP + 4;                   // FP32 stage row stride (floats)
    static constexpr int STAGE_F32 = CHF * KSF;
    static constexpr int U0 = TRI > STAGE_BF16 ? TRI : STAGE_BF16;
    static constexpr int UNION = U0 > STAGE_F32 ? U0 : STAGE_F32;
    static constexpr int NTILE = KP == 64 ? 3 : 1;
};

// Gram accumulators of a row, element i of N per lane (the layout the
// Normal-Wishart step writes Lambda / alpha in: HyperDev::Lambda_acc).
//  * G16 = false: lower 32 x 32 tiles, element 16 t + e of lane l is entry
//    (32 a + 8 (e / 4) + 4 (l / 32) + e % 4, 32 b + l % 32) of tile t
//    ((0,0), (1,0), (1,1));
//  * G16 = true (KP = 64, BF16 Gram on v_mfma_f32_16x16x32_bf16): the ten
//    lower 16 x 16 tiles, t = a (a + 1) / 2 + b, element 4 t + v of lane l is
//    entry (16 a + 4 (l / 16) + v, 16 b + l % 16).
template <int KP, bool G16>
struct GramAcc;
template <int KP>
struct GramAcc<KP, false> {
    static constexpr bool g16 = false;
    static constexpr int N = RowShape<KP>::NTILE * 16;
    floatx16 t[RowShape<KP>::NTILE];
    __device__ __forceinline__ float get(int i) const { return t[i >> 4][i & 15]; }
    __device__ __forceinline__ void set(int i, float v) { t[i >> 4][i & 15] = v; }
};
template <int KP>
struct GramAcc<KP, true> {
    static_assert(KP == 64, "16 x 16 Gram tiles for KP = 64");
    static constexpr bool g16 = true;
    static constexpr int N = 40;
    floatx4 t[10];
    __device__ __forceinline__ float get(int i) const { return t[i >> 2][i & 3]; }
    __device__ __forceinline__ void set(int i, float v) { t[i >> 2][i & 3] = v; }
};

__device__ __forceinline__ float readlane_f(float v, int lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// Synchronisation inside a factorisation or solve: BlockSync when the
// workgroup is the one wavefront doing the work; WaveSync when other
// wavefronts of the workgroup are busy elsewhere (LDS operations of one
// wavefront are processed in order, so only the compiler must keep the
// program order).
struct BlockSync {
    static __device__ __forceinline__ void sync() { __syncthreads(); }
};
struct WaveSync {
    static __device__ __forceinline__ void sync() { __asm__ volatile("" ::: "memory"); }
};

// BF16 gathers of a row's rated rows of `src` (BF16, row stride `stride`,
// 16-byte aligned rows) from the row's packed records `rec` (see
// SideArgs::rec: per 4 ratings the column indices and the two-part BF16
// offsets r - rbar; padded to whole chunks with the all-zero row and r' = 0,
// so no load needs a bound or a lane mask).  Each lane fetches
// one 16-byte piece of 4 rated rows per chunk.  The chunk is staged
// feature-major so each lane's matrix-core operand (8 consecutive ratings of
// one feature) is one 16-byte LDS read.
//
// The right-hand side sum_j r'_j v_j, with r' = hi + lo carried to about
// 2^-17 relative, runs on the matrix cores too: v_mfma_f32_16x16x32_bf16 with
// A = the 16 x 32 matrix whose row 0 holds the hi parts of 32 ratings, row 1
// their lo parts and the other rows zeros, and B = the 32 ratings' staged
// features 16t..16t+15, so C[0][f] and C[1][f] collect the hi and lo sums of
// feature 16t + f.  `rvp` holds the chunk's CH / 2 packed hi pairs, its CH / 2
// lo pairs and CH / 2 zero words (3 CH / 2 words).
template <int KP, class Sync = BlockSync, class Acc>
__device__ __forceinline__ void gram_bf16(const uint4 *rec, int64_t nnz, const uint16_t *src, int stride,
                                          char *stage, uint32_t *rvp, Acc &acc, float &bacc)
{
    using S = RowShape<KP>;
    static_assert(S::CH == bf16_chunk(KP), "records are padded to the kernel's chunk");
    static_assert(S::CH % 32 == 0, "the right-hand side takes 32 ratings per step");
    constexpr int NG = KP / 16;   // 16-feature groups of the right-hand side
    const int lane = threadIdx.x & 63;
    // the Gram accumulates onto acc as the caller set it up; the right-hand
    // side's accumulators start from the first chunk's products (a zero C
    // operand, so no register is cleared)
    floatx4 bq[NG];
    // rows 2..15 of the right-hand side's A operand read the zero words
    if (lane < S::CH / 2) rvp[S::CH + lane] = 0u;
    const uint4 *aop = (const uint4 *)(rvp + (lane % 16 < 2 ? lane % 16 : 2) * (S::CH / 2)) + lane / 16;
    // lanes 0..RG-1 stage feature block 0, lanes RG..2RG-1 block 1, ...: the
    // 8-byte staging writes of a quarter-wave then spread over more banks
    // than with consecutive lanes on consecutive feature blocks
    const int fb = lane / S::RG, rg = lane % S::RG;
    const int64_t nch = (nnz + S::CH - 1) / S::CH;
    // Loaded values stay raw until they are used (a chunk later), so no
    // arithmetic right after a load forces a wait for the loads in flight.
    // 32-bit byte offsets from the uniform base (the host keeps each side
    // below 2^24 rows, so they fit): one multiply-add per load
    const char *base = (const char *)src;
    const uint32_t rowb = 2u * (uint32_t)stride, fbb = 16u * (uint32_t)fb;
    auto load_rows = [&](const uint4 &c, uint4 *d) {
        d[0] = *(const uint4 *)(base + (__umul24(c.x, rowb) + fbb));
        d[1] = *(const uint4 *)(base + (__umul24(c.y, rowb) + fbb));
        d[2] = *(const uint4 *)(base + (__umul24(c.z, rowb) + fbb));
        d[3] = *(const uint4 *)(base + (__umul24(c.w, rowb) + fbb));
    };
    // r' pairs and the feature-major copy of one chunk into LDS
    auto stage_chunk = [&](const uint4 *d, const uint4 &rp) {
        if (fb == 0) {
            *(uint2 *)(rvp + rg * 2) = make_uint2(rp.x, rp.y);
            *(uint2 *)(rvp + S::CH / 2 + rg * 2) = make_uint2(rp.z, rp.w);
        }
        const uint32_t w0[4] = {d[0].x, d[0].y, d[0].z, d[0].w};
        const uint32_t w1[4] = {d[1].x, d[1].y, d[1].z, d[1].w};
        const uint32_t w2[4] = {d[2].x, d[2].y, d[2].z, d[2].w};
        const uint32_t w3[4] = {d[3].x, d[3].y, d[3].z, d[3].w};
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const int f = fb * 8 + 2 * w;
            // v_perm_b32 byte selects: low halves of (w0, w1), high halves
            uint2 lo, hi;
            lo.x = __builtin_amdgcn_perm(w1[w], w0[w], 0x05040100u);
            lo.y = __builtin_amdgcn_perm(w3[w], w2[w], 0x05040100u);
            hi.x = __builtin_amdgcn_perm(w1[w], w0[w], 0x07060302u);
            hi.y = __builtin_amdgcn_perm(w3[w], w2[w], 0x07060302u);
            *(uint2 *)(stage + f * S::SB + rg * 8) = lo;
            *(uint2 *)(stage + (f + 1) * S::SB + rg * 8) = hi;
        }
    };
    // Gram tiles and right-hand side of the staged chunk (the first chunk
    // starts the right-hand side's accumulators from zero)
    const floatx4 zero4 = {};
    auto multiply_chunk = [&](auto first_chunk) {
        constexpr bool FIRST = decltype(first_chunk)::value;
        if constexpr (Acc::g16) {
            // ten lower 16 x 16 tiles: lane l's operand for feature block b
            // (features 16 b + l % 16, 8 ratings from 8 (l / 16)) serves as
            // both A and B
#pragma unroll
            for (int ks = 0; ks < S::CH / 32; ++ks) {
                bf16x8_t F[4];
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    F[b] = *(const bf16x8_t *)(stage + (16 * b + lane % 16) * S::SB + (ks * 32 + (lane / 16) * 8) * 2);
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b <= a; ++b)
                        acc.t[a * (a + 1) / 2 + b] =
                            __builtin_amdgcn_mfma_f32_16x16x32_bf16(F[a], F[b], acc.t[a * (a + 1) / 2 + b], 0, 0, 0);
            }
        } else {
#pragma unroll
            for (int ks = 0; ks < S::CH / 16; ++ks) {
                const int off = (ks * 16 + (lane >> 5) * 8) * 2;
                const bf16x8_t F0 = *(const bf16x8_t *)(stage + (lane & 31) * S::SB + off);
                acc.t[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(F0, F0, acc.t[0], 0, 0, 0);
                if constexpr (KP == 64) {
                    const bf16x8_t F1 = *(const bf16x8_t *)(stage + (32 + (lane & 31)) * S::SB + off);
                    acc.t[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(F1, F0, acc.t[1], 0, 0, 0);
                    acc.t[2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(F1, F1, acc.t[2], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int ks = 0; ks < S::CH / 32; ++ks) {
            // A: lane l holds row l % 16, ratings 32 ks + 8 (l / 16) .. + 7
            const bf16x8_t Ar = *(const bf16x8_t *)(aop + 4 * ks);
#pragma unroll
            for (int t = 0; t < NG; ++t) {
                // B: lane l holds feature 16 t + l % 16 of the same ratings
                const bf16x8_t Bf =
                    *(const bf16x8_t *)(stage + (16 * t + lane % 16) * S::SB + (ks * 32 + (lane / 16) * 8) * 2);
                bq[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ar, Bf, (FIRST && ks == 0) ? zero4 : bq[t], 0, 0, 0);
            }
        }
    };
    // Software pipeline with one register set: as soon as a chunk is staged,
    // the rows of the next chunk (whose records are already loaded) and the
    // records of the one after are requested, and they arrive while the
    // staged chunk is multiplied.
    const uint4 *r0 = rec + 2 * rg;
    uint4 d[4], rpc, nc, nr;
    if (nch > 0) {
        nc = r0[0];
        rpc = r0[1];
        load_rows(nc, d);
        if (nch > 1) {
            nc = r0[2 * S::RG];
            nr = r0[2 * S::RG + 1];
        }
    }
    for (int64_t c = 0; c < nch; ++c) {
        stage_chunk(d, rpc);
        if (c + 1 < nch) {
            load_rows(nc, d);
            rpc = nr;
            if (c + 2 < nch) {
                nc = r0[2 * S::RG * (c + 2)];
                nr = r0[2 * S::RG * (c + 2) + 1];
            }
        }
        Sync::sync();
        if (c == 0)
            multiply_chunk(std::true_type{});
        else
            multiply_chunk(std::false_type{});
        Sync::sync();
    }
    if (nch == 0) {
#pragma unroll
        for (int t = 0; t < NG; ++t) bq[t] = zero4;
    }
    // lane c < 16 of bq[t] holds the hi (element 0) and lo (element 1) sums of
    // feature 16 t + c; lane l takes feature l % KP
    float bsum = 0.0f;
#pragma unroll
    for (int t = 0; t < NG; ++t) {
        const float v = __shfl(bq[t][0] + bq[t][1], lane % 16);
        bsum = (lane % KP) / 16 == t ? v : bsum;
    }
    bacc += bsum;
}

// FP32 gathers of rows `idx` of `src` (row stride K), Gram on FP32 matrix cores.
// IP and FP are the index and value pointer types: plain pointers, or
// pointers into the global address space where the caller cannot otherwise
// tell the compiler so (its loads would be flat loads, ordered against the
// LDS accesses).
template <int KP, class Sync = BlockSync, typename IP = const int32_t *, typename FP = const float *>
__device__ __forceinline__ void gram_f32(IP idx, FP vals, int64_t nnz,
                                         FP src, int K, float rbar, float *stage,
                                         float *rv, int *sidx, floatx16 *acc, float &bacc)
{
    using S = RowShape<KP>;
    const int lane = threadIdx.x & 63;
    for (int64_t c0 = 0; c0 < nnz; c0 += S::CHF) {
        const int cnt = (int)min((int64_t)S::CHF, nnz - c0);
        if (lane < S::CHF) {
            const int lc = lane < cnt ? lane : cnt - 1;  // clamped: unmasked loads
            sidx[lane] = blend_idx(lane < cnt, idx[c0 + lc], 0);
            rv[lane] = (vals[c0 + lc] - rbar) * (lane < cnt ? 1.0f : 0.0f);
        }
        Sync::sync();
#pragma unroll
        for (int t = 0; t < S::CHF * KP / 64; ++t) {
            const int e = lane + 64 * t;
            const int n = e / KP, f = e % KP;
            stage[n * S::KSF + f] = src[(int64_t)sidx[n] * K + (f < K ? f : K - 1)] * ((n < cnt && f < K) ? 1.0f : 0.0f);
        }
        Sync::sync();
#pragma unroll
        for (int ks = 0; ks < S::CHF / 2; ++ks) {
            const float *sr = stage + (2 * ks + (lane >> 5)) * S::KSF;
            const float A0 = sr[lane & 31];
            acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(A0, A0, acc[0], 0, 0, 0);
            if constexpr (KP == 64) {
                const float A1 = sr[32 + (lane & 31)];
                acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(A1, A0, acc[1], 0, 0, 0);
                acc[2] = __builtin_amdgcn_mfma_f32_32x32x2f32(A1, A1, acc[2], 0, 0, 0);
            }
        }
        {
            constexpr int SPLIT = 64 / KP;
            constexpr int PER = S::CHF / SPLIT;
            const int f = lane % KP, part = lane / KP;
#pragma unroll
            for (int n = 0; n < PER; ++n)
                bacc = fmaf(stage[(part * PER + n) * S::KSF + f], rv[part * PER + n], bacc);
        }
        Sync::sync();
    }
    if constexpr (KP == 32) bacc += __shfl_xor(bacc, 32);
}

// P = Lambda + alpha G into the packed lower triangle `tri` (row r starts at
// r(r+1)/2).  lam(r, c) returns Lambda_rc for r, c < K; it is evaluated for
// every entry (with clamped indices) so the loads are issued together.
template <int KP, typename LamFn>
__device__ __forceinline__ void store_precision(float *tri, const floatx16 *acc, int K, float alpha,
                                                LamFn lam)
{
    using S = RowShape<KP>;
    const int lane = threadIdx.x & 63;
    // entries above the diagonal go to the lane's own slot in the padding
    // after the triangle, so no store (and no load feeding it) sits behind a
    // branch of its own
    const int dump = KP * (KP + 1) / 2 + lane % KP;
#pragma unroll
    for (int t = 0; t < S::NTILE; ++t) {
        const int ta = (t == 0) ? 0 : 1, tb = (t == 2) ? 1 : 0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            // half a tile's entries of Lambda are requested before any is used
            float lv[8];
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = 32 * ta + 8 * (2 * h + j) + 4 * (lane >> 5) + i;
                    const int c = 32 * tb + (lane & 31);
                    const bool in = r < K && c < K;
                    lv[4 * j + i] = lam(in ? r : 0, in ? c : 0);
                }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = 32 * ta + 8 * (2 * h + j) + 4 * (lane >> 5) + i;
                    const int c = 32 * tb + (lane & 31);
                    const bool in = r < K && c < K;
                    const float v = in ? fmaf(alpha, acc[t][4 * (2 * h + j) + i], lv[4 * j + i]) : ((r == c) ? 1.0f : 0.0f);
                    tri[c <= r ? r * (r + 1) / 2 + c : dump] = v;
                }
        }
    }
}

// The same from Lambda stored as the padded packed triangle `lamtri` (the
// padding entries of the Gram are zero): no index checks, and every load and
// store uses the same offset.
// P / alpha = Lambda / alpha + G into the packed triangle `tri` from the
// Gram accumulators: ADD = false when they started from Lambda / alpha
// (`lamacc`, the same accumulator layout), ADD = true when they hold G alone
// and Lambda / alpha is added here (each load one coalesced 256-byte access
// at a fixed offset).
template <int KP, bool ADD, class Acc>
__device__ __forceinline__ void store_precision_tri(float *tri, const Acc &acc, const float *lamacc)
{
    const int lane = threadIdx.x & 63;
    // entries above the diagonal of a diagonal tile go to the lane's own slot
    // in the padding after the triangle: the store stays unconditional, so
    // the compiler cannot sink a load of Lambda behind a branch of its own
    const unsigned pad4 = 4u * (KP * (KP + 1) / 2 + (unsigned)(lane % KP));
    char *base = (char *)tri;
    if constexpr (Acc::g16) {
        // Entry (r, c) of 16 x 16 tile (a, b), r = R + 4 q with R = 16 a + v
        // and q = lane / 16, c = 16 b + lane % 16, sits at r (r + 1) / 2 + c =
        // R (R + 1) / 2 + 4 q R + 8 q^2 + 2 q + c: in bytes a per-lane part
        // R * 16 q + 4 (8 q^2 + 2 q + lane % 16) and a compile-time part
        // 4 R (R + 1) / 2 + 64 b that goes into the store's offset.
        const int q = lane >> 4, cl = lane & 15;
        const unsigned q16 = 16u * q, lc = 4u * (8u * q * q + 2u * q + cl);
        const int above = cl - 4 * q;  // c - r + v in a diagonal tile
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b <= a; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = 4 * (a * (a + 1) / 2 + b) + v;
                    const unsigned R = 16u * a + v;
                    const unsigned fixed = 4u * (R * (R + 1) / 2) + 64u * b;
                    float x = acc.get(i);
                    if constexpr (ADD) x += lamacc[i * 64 + lane];
                    unsigned off = R * q16 + lc;
                    if (a == b) off = above > v ? pad4 - fixed : off;
                    *(float *)(base + off + fixed) = x;
                }
    } else {
        using S = RowShape<KP>;
        const int hh = lane >> 5, cc = lane & 31;
        // Entry (r, c) of tile (ta, tb), r = R + 4 hh with R = 32 ta + 8 j + i,
        // c = 32 tb + cc, sits at r (r + 1) / 2 + c = R (R + 1) / 2 + 4 hh R +
        // (10 hh + c).  In bytes: a per-lane part R * 16 hh + 4 (10 hh + c) and
        // a compile-time part 4 R (R + 1) / 2 that goes into the store's offset.
        const unsigned u16 = 16u * hh, v4 = 4u * (10u * hh + cc);
        const int above = cc - 4 * hh;  // above the diagonal: cc - 4 hh > 8 j + i
#pragma unroll
        for (int t = 0; t < S::NTILE; ++t) {
            const int ta = (t == 0) ? 0 : 1, tb = (t == 2) ? 1 : 0;
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const unsigned R = 32u * ta + 8u * j + i;
                    const unsigned fixed = 4u * (R * (R + 1) / 2);
                    float x = acc.get(t * 16 + 4 * j + i);
                    if constexpr (ADD) x += lamacc[(t * 16 + 4 * j + i) * 64 + lane];
                    unsigned off = R * u16 + v4 + 128u * tb;
                    if (t != 1) off = above > 8 * j + i ? pad4 - fixed : off;
                    *(float *)(base + off + fixed) = x;
                }
        }
    }
}

// Matrix-core updates of the KP = 64 factorisation, where lane i holds row i
// of the matrix in A[0..63] (registers).  They run as rank-2 steps of
// v_mfma_f32_32x32x2_f32, whose operand lane l holds element (l % 32, l / 32)
// of a 32 x 2 block and whose result register 4j + i of lane l holds
// C[8j + 4(l / 32) + i][l % 32].  One v_permlane32_swap of two columns
// (registers) moves a 32-row block's two columns into the operand layout.
//
// Rows 32..63 (lanes 32..63), columns 32 + 8j + .. for j >= JMIN:
//   A[32 + c] -= sum_{k in K0..K0+NK-1} X[r][k] X[c][k],  X = rows 32..63.
// C = X X^T is symmetric, so lane 32 + r already holds C[r][8j + 4 + i]
// and receives C[r][8j + i] from lane r by a second swap.  Lanes 0..31
// update entries right of their diagonal, which are never read.
template <int K0, int NK, int JMIN>
__device__ __forceinline__ void syrk_lower_rows(float *A)
{
    floatx16 c = {};
#pragma unroll
    for (int kk = 0; kk < NK / 2; ++kk) {
        const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(A[K0 + 2 * kk]),
                                                         __float_as_uint(A[K0 + 2 * kk + 1]), false, false);
        const float x = __uint_as_float(sw[1]);
        c = __builtin_amdgcn_mfma_f32_32x32x2f32(x, x, c, 0, 0, 0);
    }
#pragma unroll
    for (int j = JMIN; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float own = c[4 * j + i];
            const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(own), __float_as_uint(own),
                                                             false, false);
            A[32 + 8 * j + 4 + i] -= own;
            A[32 + 8 * j + i] -= __uint_as_float(sw[0]);
        }
}

// All 64 rows, columns 16..31 from the first 16 columns:
//   A[r][c] -= sum_{k < 16} L[r][k] L[c][k]   (c = 16..31).
// D0 = L[0..31] L[0..31]^T and D1 = L[0..31] L[32..63]^T, both with the
// column index c in the result's row position, so lane r (r < 32) holds
// D0[8j + i][r] and lane 32 + r holds D1[8j + 4 + i][r]; one swap per result
// register hands each lane the other half of its row.
__device__ __forceinline__ void gemm_cols16_31(float *A)
{
    floatx16 d0 = {}, d1 = {};
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
        const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(A[2 * kk]), __float_as_uint(A[2 * kk + 1]),
                                                         false, false);
        const float xa = __uint_as_float(sw[0]), xb = __uint_as_float(sw[1]);
        d0 = __builtin_amdgcn_mfma_f32_32x32x2f32(xa, xa, d0, 0, 0, 0);
        d1 = __builtin_amdgcn_mfma_f32_32x32x2f32(xa, xb, d1, 0, 0, 0);
    }
#pragma unroll
    for (int j = 2; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(d0[4 * j + i]),
                                                             __float_as_uint(d1[4 * j + i]), false, false);
            A[8 * j + i] -= __uint_as_float(sw[0]);
            A[8 * j + 4 + i] -= __uint_as_float(sw[1]);
        }
}

// Columns c0..c0+7 of the matrix whose row ri = lane % KP is in A: column k
// is scaled by 1/sqrt(P_kk) (lane k thereby holds L_kk, invbuf[k] = 1/L_kk)
// and the later panel columns are updated with values read across lanes with
// readlane.  Afterwards lane ri holds L[ri][c0..c0+7] (for ri >= c0).
template <int KP>
__device__ __forceinline__ void chol_inpanel(float (&A)[KP], float *invbuf, int c0)
{
#pragma unroll
    for (int k = c0; k < c0 + 8; ++k) {
        const float inv = __builtin_amdgcn_rsqf(readlane_f(A[k], k));
        A[k] *= inv;
        invbuf[k] = inv;
#pragma unroll
        for (int j = k + 1; j < c0 + 8; ++j) A[j] = fmaf(-A[k], readlane_f(A[k], j), A[j]);
    }
}

// The rank-8 update of columns c0 + 8 .. jend - 1 by the factored panel
// c0..c0+7: every lane publishes its 8 panel entries through LDS (`pbuf`)
// and updates its own row.
template <int KP, class Sync>
__device__ __forceinline__ void chol_next(float (&A)[KP], float *pbuf, int c0, int jend)
{
    // pbuf rows are 12 floats apart, so 16 consecutive lanes cover all 64
    // LDS banks with their 16-byte writes
    constexpr int PS = 12;
    const int lane = threadIdx.x & 63;
    if (c0 + 8 < jend) {
        if (lane < KP) {
            *(float4 *)(pbuf + lane * PS) = make_float4(A[c0], A[c0 + 1], A[c0 + 2], A[c0 + 3]);
            *(float4 *)(pbuf + lane * PS + 4) = make_float4(A[c0 + 4], A[c0 + 5], A[c0 + 6], A[c0 + 7]);
        }
        Sync::sync();
#pragma unroll
        for (int j = c0 + 8; j < jend; ++j) {
            const float4 p0 = *(const float4 *)(pbuf + j * PS);
            const float4 p1 = *(const float4 *)(pbuf + j * PS + 4);
            float t = A[j];
            t = fmaf(-A[c0 + 0], p0.x, t);
            t = fmaf(-A[c0 + 1], p0.y, t);
            t = fmaf(-A[c0 + 2], p0.z, t);
            t = fmaf(-A[c0 + 3], p0.w, t);
            t = fmaf(-A[c0 + 4], p1.x, t);
            t = fmaf(-A[c0 + 5], p1.y, t);
            t = fmaf(-A[c0 + 6], p1.z, t);
            t = fmaf(-A[c0 + 7], p1.w, t);
            A[j] = t;
        }
        Sync::sync();
    }
}

template <int KP, class Sync>
__device__ __forceinline__ void chol_panel(float (&A)[KP], float *invbuf, float *pbuf, int c0, int jend)
{
    chol_inpanel<KP>(A, invbuf, c0);
    chol_next<KP, Sync>(A, pbuf, c0, jend);
}

// Step P (0..7) of the KP = 64 factorisation below: what precedes panel P's
// columns (the updates by the earlier panels that are still pending) and the
// panel itself.  After step P, lane ri holds its final L[ri][8P..8P+7].
template <int P, class Sync>
__device__ __forceinline__ void chol64_step(float (&A)[64], float *invbuf, float *pbuf)
{
    if constexpr (P == 1 || P == 3 || P == 5 || P == 7) chol_next<64, Sync>(A, pbuf, 8 * (P - 1), 8 * (P + 1));
    if constexpr (P == 2) gemm_cols16_31(A);
    if constexpr (P == 4) syrk_lower_rows<0, 32, 0>(A);
    if constexpr (P == 6) syrk_lower_rows<32, 16, 2>(A);
    chol_inpanel<64>(A, invbuf, 8 * P);
}

// Factor the KP x KP matrix whose row ri = lane % KP is in A (registers):
// afterwards A holds row ri of L (lower, L L^T = P) and invbuf[k] = 1/L_kk.
// `pbuf` is KP x 12 floats of LDS scratch.
//
// The factorisation runs in panels of 8 columns (chol_panel).  Entries right
// of the diagonal are updated too but never read, so the loops need no lane
// masks.  An unusable pivot gives a NaN, infinite or zero 1/sqrt, caught by
// chol_pivots_fail.
//
// KP = 64: the panels' updates reach only the next panel of their 16-column
// block on the vector units; everything further right is a matrix-core
// product: columns 16..31 of all rows from columns 0..15 (gemm_cols16_31),
// the trailing 32 x 32 block A22 -= L21 L21^T from columns 0..31, and
// columns 48..63 of rows 32..63 from columns 32..47 (syrk_lower_rows).
// That leaves 480 multiply-add instructions per lane on the vector units (224
// inside the panels, 256 for the next panel), against 992 when only A22 was
// a matrix-core product.  (The next-panel updates on the matrix cores too
// measured neutral in the sampler and 15 % slower in the fold-in kernel,
// where many more wavefronts share the matrix cores.)
//
// MT = false (a launch-shape variant): KP = 64 with the panels' updates on the
// vector units up to the end of their 32-column half, and only A22 -= L21
// L21^T (columns 0..31 into 32..63 of rows 32..63) as a matrix-core product.
template <int KP, class Sync = BlockSync, bool MT = true>
__device__ __forceinline__ void chol_factor(float (&A)[KP], float *invbuf, float *pbuf)
{
    if constexpr (KP == 64 && !MT) {
#pragma unroll
        for (int c0 = 0; c0 < KP; c0 += 8) {
            chol_panel<KP, Sync>(A, invbuf, pbuf, c0, c0 < 32 ? 32 : 64);
            if (c0 == 24) syrk_lower_rows<0, 32, 0>(A);
        }
    } else if constexpr (KP == 64) {
        chol64_step<0, Sync>(A, invbuf, pbuf);
        chol64_step<1, Sync>(A, invbuf, pbuf);
        chol64_step<2, Sync>(A, invbuf, pbuf);
        chol64_step<3, Sync>(A, invbuf, pbuf);
        chol64_step<4, Sync>(A, invbuf, pbuf);
        chol64_step<5, Sync>(A, invbuf, pbuf);
        chol64_step<6, Sync>(A, invbuf, pbuf);
        chol64_step<7, Sync>(A, invbuf, pbuf);
    } else {
#pragma unroll
        for (int c0 = 0; c0 < KP; c0 += 8) chol_panel<KP, Sync>(A, invbuf, pbuf, c0, KP);
    }
}

// A pivot d_k (k < kmax) fails when it is not finite or d_k <= tau, i.e. when
// 1/sqrt(d_k) is not a positive finite number with tau / d_k < 1; the
// identity pivots of the padding (k >= kmax) are not checked.  Uniform.
__device__ __forceinline__ bool chol_pivots_fail(float inv_own, int ri, int kmax, float tau)
{
    const bool bk = (ri < kmax) && !((inv_own > 0.0f) && (inv_own * inv_own * tau < 1.0f));
    return __ballot(bk) != 0;
}

// y = L^{-1} b with row ri of L in A and b_ri in bb; returns y_ri.  y_k is
// taken from lane k before later steps overwrite it; ybuf holds KP floats.
template <int KP, class Sync = BlockSync>
__device__ __forceinline__ float forward_sub(const float (&A)[KP], float invd, float bb, float *ybuf)
{
    const int ri = (threadIdx.x & 63) % KP;
#pragma unroll
    for (int k = 0; k < KP; ++k) {
        const float yk = readlane_f(bb * invd, k);
        ybuf[k] = yk;
        bb = fmaf(-A[k], yk, bb);
    }
    Sync::sync();
    return ybuf[ri];
}

// Rows of L into the packed triangle `tri` (row r at r(r+1)/2).  Every lane
// stores its whole row, last column first, one store instruction per column.
// A lane's entries right of its diagonal (garbage) land in later rows'
// slots: r(r+1)/2 + c' with r > ri and c' < c, which their owners write at
// a later step.  The compiler fence keeps the columns in separate
// instructions: merged into one ds_write2, two lanes could write one slot
// in the same instruction.
template <int KP>
__device__ __forceinline__ void store_rows(const float (&A)[KP], float *tri)
{
    const int lane = threadIdx.x & 63;
    const int ri = lane % KP;
    const int rbase = ri * (ri + 1) / 2;
    if (lane < KP) {
#pragma unroll
        for (int c = KP - 1; c >= 0; --c) {
            tri[rbase + c] = A[c];
            __asm__ volatile("" ::: "memory");
        }
    }
}

// Lower triangle of the rows of L only (lane-masked), into a packed layout
// whose row r starts at r(r+1)/2 + G r: G = 0 is the plain packed triangle,
// G > 0 a triangle embedded in a larger packed one (row r of the block at
// column offset G of row G + r), where the entries right of the diagonal
// would overwrite other data.
template <int KP, int G>
__device__ __forceinline__ void store_rows_lower(const float (&A)[KP], float *tri)
{
    const int lane = threadIdx.x & 63;
    const int ri = lane % KP;
    const int rbase = ri * (ri + 1) / 2 + G * ri;
    if (lane < KP) {
#pragma unroll
        for (int c = 0; c < KP; ++c)
            if (c <= ri) tri[rbase + c] = A[c];
    }
}

// x = L^{-T} w with L packed in `tri` (row r at r(r+1)/2 + G r) and w_ri in
// w; returns x_ri.  xbuf holds KP floats.
template <int KP, class Sync = BlockSync, int G = 0>
__device__ __forceinline__ float backward_sub(const float *tri, float invd, float w, float *xbuf)
{
    const int ri = (threadIdx.x & 63) % KP;
#pragma unroll
    for (int k = KP - 1; k >= 0; --k) {
        const float xk = readlane_f(w * invd, k);
        xbuf[k] = xk;
        w = fmaf(-tri[k * (k + 1) / 2 + G * k + ri], xk, w);
    }
    Sync::sync();
    return xbuf[ri];
}

// The two solves with every row of L divided by its own diagonal entry
// (L' = D^-1 L, unit diagonal, D = diag(L)):
//  * L y = b  is  L' y = D^-1 b;
//  * L^T x = w  is  L'^T u = w  with  u = D x  (L_ik x_i = L'_ik u_i), so
//    x = D^-1 u.
// Both are unit-diagonal solves: each step of their serial chains is one
// broadcast and one multiply-add.  A holds row ri of L' (registers); `tri` its
// packed rows.  ybuf and xbuf hold KP floats.
template <int KP, class Sync = BlockSync>
__device__ __forceinline__ float forward_sub_unit(const float (&A)[KP], float bb, float *ybuf)
{
    const int ri = (threadIdx.x & 63) % KP;
#pragma unroll
    for (int k = 0; k < KP; ++k) {
        const float yk = readlane_f(bb, k);
        ybuf[k] = yk;
        bb = fmaf(-A[k], yk, bb);
    }
    Sync::sync();
    return ybuf[ri];
}

template <int KP, class Sync = BlockSync>
__device__ __forceinline__ float backward_sub_unit(const float *tri, float w, float *xbuf)
{
    const int ri = (threadIdx.x & 63) % KP;
#pragma unroll
    for (int k = KP - 1; k >= 0; --k) {
        const float uk = readlane_f(w, k);
        xbuf[k] = uk;
        w = fmaf(-tri[k * (k + 1) / 2 + ri], uk, w);
    }
    Sync::sync();
    return xbuf[ri];
}

// Factor P (packed in `tri`) and return x = L^{-T}(L^{-1} b + z) on lane
// ri = lane % KP, where lane ri holds b_ri and z_ri.  `fail` is set (uniformly
// across the wave) when a pivot is not finite or not above
// 64 K 2^-24 max_{k<K} P_kk.  Overwrites `tri` with D^-1 L (rows of L divided
// by their diagonal entries); `aux` holds 3 KP floats.
// Lane ri keeps row ri of P in registers through chol_factor.
template <int KP, class Sync = BlockSync, bool MT = true>
__device__ __forceinline__ float chol_solve(float *tri, float *aux, int K, float bb, float z,
                                            bool &fail)
{
    const int lane = threadIdx.x & 63;
    const int ri = lane % KP;
    float *invbuf = aux, *ybuf = aux + KP, *xbuf = aux + 2 * KP;
    const int rbase = ri * (ri + 1) / 2;
    float A[KP];
#pragma unroll
    for (int c = 0; c < KP; ++c) A[c] = tri[rbase + c];
    float dg = (ri < K) ? tri[rbase + ri] : 0.0f;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) dg = fmaxf(dg, __shfl_xor(dg, o));
    const float tau = 64.0f * (float)K * 0x1.0p-24f * dg;
    Sync::sync();
    chol_factor<KP, Sync, MT>(A, invbuf, tri);  // P is in registers: tri serves as the panel buffer
    fail = chol_pivots_fail(invbuf[ri], ri, K, tau);
    const float invd = invbuf[ri];
    // rows of L' = D^-1 L for the unit-diagonal solves
#pragma unroll
    for (int c = 0; c < KP; ++c) A[c] *= invd;
    const float y = forward_sub_unit<KP, Sync>(A, bb * invd, ybuf);
    store_rows<KP>(A, tri);
    Sync::sync();
    const float x = backward_sub_unit<KP, Sync>(tri, y + z, xbuf) * invd;
    Sync::sync();
    return x;
}

}  // namespace bpmf
