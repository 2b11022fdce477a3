// kernels_rank1.hip -- mixed-precision row update by rank-one Cholesky updates,
// for rows with very few ratings (paper: Section 3.1 recommends a rank-one
// update when an item has few ratings; Section 3.2 routes such items to it).
//
// The conditional of a row is the same as in the full path (Section 2,
// Algorithm 1):
//   P = Lambda + alpha sum_{t} v_t v_t^T,  b = Lambda mu + alpha sum_t r'_t v_t,
//   x = L^{-T}(L^{-1} b + z),  L = chol(P).
// With L0 = chol(Lambda) (the Normal-Wishart step leaves it behind as its T
// factor), chol(P) follows from m = nnz rank-one updates L L^T + w w^T,
// w = sqrt(alpha) v_t.  Each update is a sweep of Givens rotations over the
// columns: for column k, with r = sqrt(L_kk^2 + w_k^2), c = L_kk / r and
// s = w_k / r, every row i >= k maps (L_ik, w_i) to
// (c L_ik + s w_i, c w_i - s L_ik); row k gets L_kk = r and w_k = 0.  That is
// O(m K^2) work instead of the K^3 / 3 of factoring P, and the diagonal only
// grows, so there is no cancellation in the pivots.
//
// Layout: the rows with at most RANK1_MAX ratings are the tail of the
// rating-count order.  Persistent workgroups of four wavefronts; a wavefront
// takes B <= 64 consecutive slots of that tail (B is chosen so that small
// tails still spread over many wavefronts), loads their order, row pointers,
// column indices and ratings with one load each (lane l for slot l), then
// handles the rows one after another with lane i holding row i of L in
// registers.  L0 stays in LDS for the whole launch; the other side's rows
// for the next row are requested before the current row's arithmetic.
// Same pivot rule and FP64 fallback list as the full mixed-precision kernel.
#include "common.hpp"
#include "rng.hpp"
#include "rowsolve.hpp"

namespace bpmf {

namespace {

constexpr int RANK1_MAX = 4;  // the kernel handles rows with up to this many ratings
constexpr int R1_WAVES = 4;

template <int KP, bool BF16>
__global__ __launch_bounds__(64 * R1_WAVES) void rows_rank1_kernel(SideArgs a, int K, float alpha, float salpha,
                                                                    float rbar, HyperDev hyp, DrawSrc draws,
                                                                    int32_t *fb_list, DevState *state, int side,
                                                                    int64_t slot0, int64_t slot1, int64_t nnz,
                                                                    int B)
{
    constexpr int LS = KP + 4;  // L0 row stride in LDS: 16-byte row reads stay conflict-free
    constexpr int TRI = KP * (KP + 1) / 2;
    __shared__ __attribute__((aligned(16))) float l0[KP * LS];
    __shared__ __attribute__((aligned(16))) float wbuf[R1_WAVES][TRI + 2 * KP];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ri = lane % KP;
    const bool live = ri < K;
    const int rbase = ri * (ri + 1) / 2;
    float *tri = wbuf[wave];
    float *ybuf = tri + TRI, *xbuf = ybuf + KP;

    for (int e = threadIdx.x; e < KP * KP; e += 64 * R1_WAVES) l0[(e / KP) * LS + (e % KP)] = hyp.Lchol[e];
    const float lamdiag = hyp.Lambda_tri[rbase + ri];
    const float lmu = hyp.Lmu_f[live ? ri : 0];
    __syncthreads();

    const float *vals = (const float *)a.val;
    const float *ofp = (const float *)a.other;
    const uint32_t h = draws.tape_rows ? 0u : half_sweep_index(draws);
    const float pad = live ? 1.0f : 0.0f;
    const int64_t nbatch = (slot1 - slot0 + B - 1) / B;

    for (int64_t bt = (int64_t)blockIdx.x * R1_WAVES + wave; bt < nbatch; bt += (int64_t)gridDim.x * R1_WAVES) {
        const int64_t base = slot0 + bt * B;
        const int nb = (int)((slot1 - base) < B ? (slot1 - base) : B);
        // lane l describes slot base + l (lanes past the end repeat the last slot)
        const int row_l = a.order[base + (lane < nb ? lane : nb - 1)];
        const int64_t p0 = a.ptr[row_l];
        const int nz_l = (int)(a.ptr[row_l + 1] - p0);
        int j_l[RANK1_MAX];
        float r_l[RANK1_MAX];
#pragma unroll
        for (int t = 0; t < RANK1_MAX; ++t) {
            const bool ok = t < nz_l;
            const int64_t e = ok ? p0 + t : 0;
            if (nnz > 0) {
                j_l[t] = a.idx[e];
                r_l[t] = (vals[e] - rbar) * (ok ? 1.0f : 0.0f);
            } else {
                j_l[t] = 0;
                r_l[t] = 0.0f;
            }
        }

        // gathered entries of the rated rows (lane ri: component ri)
        auto gather = [&](int r, float (&g)[RANK1_MAX]) {
#pragma unroll
            for (int t = 0; t < RANK1_MAX; ++t) {
                const int j = __builtin_amdgcn_readlane(j_l[t], r);
                if constexpr (BF16)
                    g[t] = bf16_to_f32(a.other_bf16[(int64_t)j * a.shadow_stride + ri]);
                else
                    g[t] = ofp[(int64_t)j * K + (live ? ri : 0)];
            }
        };
        float g[RANK1_MAX];
        if (nnz > 0) gather(0, g);

        for (int r = 0; r < nb; ++r) {
            const int row = __builtin_amdgcn_readlane(row_l, r);
            const int nz = __builtin_amdgcn_readlane(nz_l, r);
            float v[RANK1_MAX];
            float bacc = 0.0f, vsq = 0.0f;
#pragma unroll
            for (int t = 0; t < RANK1_MAX; ++t) {
                v[t] = t < nz ? g[t] * pad : 0.0f;
                bacc = fmaf(readlane_f(r_l[t], r), v[t], bacc);
                vsq = fmaf(v[t], v[t], vsq);
            }
            if (nnz > 0 && r + 1 < nb) gather(r + 1, g);

            float z;
            if (draws.tape_rows) {
                z = live ? (float)draws.tape_rows[(int64_t)row * K + ri] : 0.0f;
            } else {
                float z0, z1;
                box_muller_f32(philox4x32_10(ctr4((uint32_t)(ri >> 1), (uint32_t)row, h, 0u), draws.seed), z0, z1);
                z = live ? ((ri & 1) ? z1 : z0) : 0.0f;
            }

            float A[KP];
#pragma unroll
            for (int c = 0; c < KP; c += 4) {
                const float4 q = *(const float4 *)(l0 + ri * LS + c);
                A[c] = q.x;
                A[c + 1] = q.y;
                A[c + 2] = q.z;
                A[c + 3] = q.w;
            }
#pragma unroll
            for (int t = 0; t < RANK1_MAX; ++t) {
                if (t < nz) {
                    float w = salpha * v[t];
#pragma unroll
                    for (int k = 0; k < KP; ++k) {
                        const float lkk = readlane_f(A[k], k), wk = readlane_f(w, k);
                        const float rho = __builtin_amdgcn_rsqf(fmaf(wk, wk, lkk * lkk));
                        const float cs = lkk * rho, sn = wk * rho;
                        const float ak = A[k];
                        A[k] = fmaf(cs, ak, sn * w);
                        w = fmaf(cs, w, -(sn * ak));
                    }
                }
            }

            store_rows<KP>(A, tri);
            WaveSync::sync();
            const float invd = 1.0f / tri[rbase + ri];
            float pk = live ? fmaf(alpha, vsq, lamdiag) : 0.0f;
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) pk = fmaxf(pk, __shfl_xor(pk, o));
            const float tau = 64.0f * (float)K * 0x1.0p-24f * pk;
            const bool fail = chol_pivots_fail(invd, ri, K, tau);

            const float bb = live ? fmaf(alpha, bacc, lmu) : 0.0f;
            const float y = forward_sub<KP, WaveSync>(A, invd, bb, ybuf);
            const float x = backward_sub<KP, WaveSync>(tri, invd, y + z, xbuf);
            if (!fail) {
                float *X = (float *)a.X;
                if (lane < KP && live) X[(int64_t)row * K + ri] = x;
                if (a.X_bf16 && lane < KP)
                    a.X_bf16[(int64_t)row * a.shadow_stride + ri] = live ? f32_to_bf16_rne(x) : (uint16_t)0;
            } else if (lane == 0) {
                const int pos = atomicAdd(&state->fb_count[side], 1);
                fb_list[pos] = row;
            }
        }
    }
}

// Rows with at most one rating and K <= 32: one lane per row.
//
// With L0 = chol(Lambda), p = sqrt(alpha) L0^{-1} v and c = L0^{-1} b, the
// factor of P = L0 (I + p p^T) L0^T is L0 Lt with Lt = chol(I + p p^T).  The
// LDL^T form of I + p p^T is known in closed form (the rank-one modification
// formulas of Gill, Golub, Murray and Saunders, Math. Comp. 28 (1974)): with
// t_j = 1 + sum_{m<=j} p_m^2 (t_{-1} = 1), D = diag(t_j / t_{j-1}) and the
// unit lower factor U_ij = p_i p_j / t_j (i > j).  Solving with it takes
// running sums only:
//   (U^{-1} c)_i = c_i - p_i S_i / t_{i-1},   S_i = sum_{j<i} p_j c_j,
//   (U^{-T} h)_j = h_j - p_j Q_j,             Q_j = sum_{i>j} p_i h_i / t_{i-1}.
// So x = L0^{-T} U^{-T} D^{-1/2} (D^{-1/2} U^{-1} c + z): two triangular solves
// with the fixed L0, whose entries are the same for every lane (read from LDS
// at one address per wavefront, a broadcast), and O(K) further work per row.  The pivots of chol(P) are
// L0_kk^2 t_k / t_{k-1}; the rule and the FP64 fallback are the other kernels'.
// All 32 components are computed: the padding has L0 = I, v = 0, c0 = 0 and
// z = 0, so it stays zero.  `lc` holds L0 (32 x 32 row-major), then 32 floats
// each of 1 / L0_ii, L0^T mu (= L0^{-1} Lambda mu), Lambda_ii (0 in the
// padding) and 1 / 0 flags of the live components.
__device__ __forceinline__ float4 lds4(const float *p) { return *(const float4 *)p; }

template <bool BF16, bool VEC>
__global__ __launch_bounds__(256) void rows_tiny_kernel(SideArgs a, int K, float alpha, float salpha, float rbar,
                                                        const float *lc, DrawSrc draws,
                                                        int32_t *fb_list, DevState *state, int side,
                                                        int64_t slot0, int64_t slot1, int64_t nnz)
{
    constexpr int KP = 32;
    // L0 row-major, L0 transposed, then 1 / L0_ii, c0, Lambda_ii, live flags;
    // zb: each thread's normals, component-major (zb[i * 256 + thread])
    __shared__ __attribute__((aligned(16))) float sm[2 * KP * KP + 4 * KP];
    __shared__ float zb[KP * 256];
    float *Lm = sm, *Lt = sm + KP * KP;
    for (int e = threadIdx.x; e < KP * KP; e += blockDim.x) {
        const float x = lc[e];
        Lm[e] = x;
        Lt[(e % KP) * KP + e / KP] = x;
    }
    for (int e = threadIdx.x; e < 4 * KP; e += blockDim.x) sm[2 * KP * KP + e] = lc[KP * KP + e];
    __syncthreads();
    const float *invd = sm + 2 * KP * KP;
    const float *c0 = invd + KP;
    const float *lamd = c0 + KP;
    const float *live = lamd + KP;
    const int64_t slot = slot0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= slot1) return;
    const int row = a.order[slot];
    const int64_t p0 = a.ptr[row];
    const float has = a.ptr[row + 1] > p0 ? 1.0f : 0.0f;
    float *zt = zb + threadIdx.x;

    // the row's normals (a rolled loop, so that the generator's temporaries
    // are not all live at once)
    if (draws.tape_rows) {
        const double *tz = draws.tape_rows + (int64_t)row * K;
#pragma unroll
        for (int i0 = 0; i0 < KP; i0 += 4) {
            const float4 lv = lds4(live + i0);
            zt[(i0 + 0) * 256] = (float)tz[i0 + 0 < K ? i0 + 0 : K - 1] * lv.x;
            zt[(i0 + 1) * 256] = (float)tz[i0 + 1 < K ? i0 + 1 : K - 1] * lv.y;
            zt[(i0 + 2) * 256] = (float)tz[i0 + 2 < K ? i0 + 2 : K - 1] * lv.z;
            zt[(i0 + 3) * 256] = (float)tz[i0 + 3 < K ? i0 + 3 : K - 1] * lv.w;
        }
    } else {
        const uint32_t h = half_sweep_index(draws);
#pragma unroll 1
        for (int q = 0; q < KP / 2; ++q) {
            float z0, z1;
            box_muller_f32(philox4x32_10(ctr4((uint32_t)q, (uint32_t)row, h, 0u), draws.seed), z0, z1);
            zt[(2 * q) * 256] = z0 * live[2 * q];
            zt[(2 * q + 1) * 256] = z1 * live[2 * q + 1];
        }
    }

    float v[KP];
    float rr = 0.0f;
#pragma unroll
    for (int i = 0; i < KP; ++i) v[i] = 0.0f;
    if (nnz > 0) {
        const int64_t e = has != 0.0f ? p0 : 0;
        const int j = a.idx[e];
        rr = (((const float *)a.val)[e] - rbar) * has;
        if constexpr (BF16) {
            const uint4 *src = (const uint4 *)(a.other_bf16 + (int64_t)j * a.shadow_stride);
#pragma unroll
            for (int q = 0; q < KP / 8; ++q) {
                const uint4 w = src[q];
                const uint32_t u[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    v[8 * q + 2 * m] = __uint_as_float(u[m] << 16) * has;
                    v[8 * q + 2 * m + 1] = __uint_as_float(u[m] & 0xffff0000u) * has;
                }
            }
        } else if constexpr (VEC) {
            // K % 4 == 0: K / 4 aligned 16-byte pieces, the rest of the pieces repeat the last one
            const float4 *src = (const float4 *)((const float *)a.other + (int64_t)j * K);
            const int nq = K / 4;
#pragma unroll
            for (int q = 0; q < KP / 4; ++q) {
                const float4 w = src[q < nq ? q : nq - 1];
                const float m = q < nq ? has : 0.0f;
                v[4 * q] = w.x * m;
                v[4 * q + 1] = w.y * m;
                v[4 * q + 2] = w.z * m;
                v[4 * q + 3] = w.w * m;
            }
        } else {
            const float *src = (const float *)a.other + (int64_t)j * K;
#pragma unroll
            for (int i = 0; i < KP; ++i) v[i] = src[i < K ? i : K - 1] * (i < K ? has : 0.0f);
        }
    }

    // w = sqrt(alpha) v; pivot threshold 64 K 2^-24 max_k P_kk, P_kk = Lambda_kk + w_k^2
    float pmax = 0.0f;
#pragma unroll
    for (int i0 = 0; i0 < KP; i0 += 4) {
        const float4 ld = lds4(lamd + i0);
        const float l4[4] = {ld.x, ld.y, ld.z, ld.w};
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            v[i0 + m] *= salpha;
            pmax = fmaxf(pmax, fmaf(v[i0 + m], v[i0 + m], l4[m]));
        }
    }
    const float tau = 64.0f * (float)K * 0x1.0p-24f * pmax;

    // p = L0^{-1} w, in place
#pragma unroll
    for (int i = 0; i < KP; ++i) {
        float acc = v[i];
#pragma unroll
        for (int k0 = 0; k0 < i; k0 += 4) {
            const float4 l = lds4(Lm + i * KP + k0);
            acc = fmaf(-l.x, v[k0], acc);
            if (k0 + 1 < i) acc = fmaf(-l.y, v[k0 + 1], acc);
            if (k0 + 2 < i) acc = fmaf(-l.z, v[k0 + 2], acc);
            if (k0 + 3 < i) acc = fmaf(-l.w, v[k0 + 3], acc);
        }
        v[i] = acc * invd[i];
    }
    // c = L0^{-1} b = c0 + sqrt(alpha) r' p; y = D^{-1/2} U^{-1} c; pivots
    float c[KP], rs[KP];  // rs_i = 1 / sqrt(t_i)
    float worst = 0.0f;  // max over live pivots of tau / pivot; NaN-safe via the sign test below
    bool nonpos = false;
    {
        const float ar = salpha * rr;
        float tp = 1.0f, rsp = 1.0f, S = 0.0f;  // t_{i-1}, 1/sqrt(t_{i-1}), S_i
#pragma unroll
        for (int i = 0; i < KP; ++i) {
            const float p = v[i];
            const float ci = fmaf(ar, p, c0[i]);
            const float tn = fmaf(p, p, tp);
            const float r = __builtin_amdgcn_rsqf(tn);
            const float di = (tp * rsp) * r;  // sqrt(t_{i-1} / t_i)
            const float it = rsp * rsp;       // 1 / t_{i-1}
            c[i] = (ci - p * (S * it)) * di;
            S = fmaf(p, ci, S);
            rs[i] = r;
            const float inv = invd[i] * di;   // 1 / sqrt(pivot i)
            nonpos |= !(inv > 0.0f);
            worst = fmaxf(worst, (inv * inv) * (tau * live[i]));
            tp = tn;
            rsp = r;
        }
    }
    const bool fail = nonpos || !(worst < 1.0f);
    // u = U^{-T} D^{-1/2} (y + z), then x = L0^{-T} u, both in place
    {
        float Q = 0.0f;
#pragma unroll
        for (int j = KP - 1; j >= 0; --j) {
            const float rp = j > 0 ? rs[j - 1] : 1.0f;                 // 1 / sqrt(t_{j-1})
            const float hj = (c[j] + zt[j * 256]) * (rs[j] * __builtin_amdgcn_rcpf(rp));  // D^{-1/2} (y + z)
            c[j] = hj - v[j] * Q;
            Q = fmaf(v[j] * hj, rp * rp, Q);
        }
    }
#pragma unroll
    for (int i = KP - 1; i >= 0; --i) {
        float acc = c[i];
#pragma unroll
        for (int k0 = (i + 1) & ~3; k0 < KP; k0 += 4) {
            const float4 l = lds4(Lt + i * KP + k0);  // L0_{k,i}, k = k0..k0+3
            if (k0 > i) acc = fmaf(-l.x, c[k0], acc);
            if (k0 + 1 > i) acc = fmaf(-l.y, c[k0 + 1], acc);
            if (k0 + 2 > i) acc = fmaf(-l.z, c[k0 + 2], acc);
            acc = fmaf(-l.w, c[k0 + 3], acc);
        }
        c[i] = acc * invd[i];
    }

    if (fail) {
        const int pos = atomicAdd(&state->fb_count[side], 1);
        fb_list[pos] = row;
        return;
    }
    float *X = (float *)a.X + (int64_t)row * K;
    if constexpr (VEC) {
#pragma unroll
        for (int q = 0; q < KP / 4; ++q)
            if (4 * q < K) ((float4 *)X)[q] = make_float4(c[4 * q], c[4 * q + 1], c[4 * q + 2], c[4 * q + 3]);
    } else {
#pragma unroll
        for (int i = 0; i < KP; ++i)
            if (i < K) X[i] = c[i];
    }
    if (a.X_bf16) {
        // the padding of c is zero, and so is its BF16 image
        uint4 *dst = (uint4 *)(a.X_bf16 + (int64_t)row * a.shadow_stride);
#pragma unroll
        for (int q = 0; q < KP / 8; ++q) {
            uint32_t u[4];
#pragma unroll
            for (int m = 0; m < 4; ++m)
                u[m] = (uint32_t)f32_to_bf16_rne(c[8 * q + 2 * m]) |
                       ((uint32_t)f32_to_bf16_rne(c[8 * q + 2 * m + 1]) << 16);
            dst[q] = make_uint4(u[0], u[1], u[2], u[3]);
        }
    }
}

}  // namespace

int rank1_max_ratings() { return RANK1_MAX; }

hipError_t launch_rows_tiny(const SideArgs &a, int K, int bf16, double alpha, double rbar, HyperDev hyp,
                            DrawSrc draws, int32_t *fb_list, DevState *state, int64_t slot0, int64_t slot1,
                            int64_t nnz, hipStream_t s)
{
    if (slot1 <= slot0) return hipSuccess;
    if (!hyp.Lchol || K > 32) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((slot1 - slot0 + 255) / 256)), block(256);
    const float fa = (float)alpha, fsa = std::sqrt((float)alpha), fr = (float)rbar;
    if (bf16)
        hipLaunchKernelGGL((rows_tiny_kernel<true, false>), grid, block, 0, s, a, K, fa, fsa, fr, hyp.Lchol, draws, fb_list, state, draws.side, slot0, slot1, nnz);
    else if (K % 4 == 0)
        hipLaunchKernelGGL((rows_tiny_kernel<false, true>), grid, block, 0, s, a, K, fa, fsa, fr, hyp.Lchol, draws, fb_list, state, draws.side, slot0, slot1, nnz);
    else
        hipLaunchKernelGGL((rows_tiny_kernel<false, false>), grid, block, 0, s, a, K, fa, fsa, fr, hyp.Lchol, draws, fb_list, state, draws.side, slot0, slot1, nnz);
    return hipGetLastError();
}

hipError_t launch_rows_rank1(const SideArgs &a, int K, int KP, int bf16, double alpha, double rbar, HyperDev hyp,
                             DrawSrc draws, int32_t *fb_list, DevState *state, int64_t slot0, int64_t slot1,
                             int64_t nnz, hipStream_t s)
{
    if (slot1 <= slot0) return hipSuccess;
    if (!hyp.Lchol) return hipErrorInvalidValue;
    // rows per wavefront batch: whole 64-row batches once the tail fills
    // about 8 wavefronts per SIMD (256 CUs x 4 SIMDs), fewer rows before that
    const int64_t n = slot1 - slot0;
    const int B = (int)std::min<int64_t>(64, std::max<int64_t>(1, (n + 8191) / 8192));
    const int64_t nbatch = (n + B - 1) / B;
    const int64_t wg = (nbatch + R1_WAVES - 1) / R1_WAVES;
    const dim3 grid((unsigned)(wg < 2048 ? wg : 2048)), block(64 * R1_WAVES);
    const float fa = (float)alpha, fsa = std::sqrt((float)alpha), fr = (float)rbar;
    if (KP == 64) {
        if (bf16) hipLaunchKernelGGL((rows_rank1_kernel<64, true>), grid, block, 0, s, a, K, fa, fsa, fr, hyp, draws, fb_list, state, draws.side, slot0, slot1, nnz, B);
        else hipLaunchKernelGGL((rows_rank1_kernel<64, false>), grid, block, 0, s, a, K, fa, fsa, fr, hyp, draws, fb_list, state, draws.side, slot0, slot1, nnz, B);
    } else if (KP == 32) {
        if (bf16) hipLaunchKernelGGL((rows_rank1_kernel<32, true>), grid, block, 0, s, a, K, fa, fsa, fr, hyp, draws, fb_list, state, draws.side, slot0, slot1, nnz, B);
        else hipLaunchKernelGGL((rows_rank1_kernel<32, false>), grid, block, 0, s, a, K, fa, fsa, fr, hyp, draws, fb_list, state, draws.side, slot0, slot1, nnz, B);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace bpmf
