// kernels_f64.hip -- the plain FP64 row update (one workgroup per row), the
// side statistics for the hyper-parameter step, predictions and small helpers.
//
// Row update (paper: Section 2, Algorithm 1 inner loops; Section 3.1): for
// row i with rated items Omega_i,
//   P = Lambda + alpha sum_j v_j v_j^T,  b = Lambda mu + alpha sum_j (r_ij - rbar) v_j,
//   L L^T = P,  x_i = L^{-T}(L^{-1} b + z_i).
// This kernel keeps P in LDS (K <= 128: at most 128 KB of FP64), gathers the
// rated rows in chunks of 16 into LDS, accumulates the lower triangle of the
// Gram in 4x4 register tiles, factors P with a right-looking Cholesky across
// the workgroup, and solves with one thread per element.
#include <algorithm>

#include "common.hpp"
#include "rng.hpp"

namespace bpmf {

namespace {

constexpr int F64_CH = 16;  // gathered rows per LDS chunk

__device__ __forceinline__ void tri_decode(int t, int &r, int &c)
{
    int q = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while (q * (q + 1) / 2 > t) --q;
    while ((q + 1) * (q + 2) / 2 <= t) ++q;
    r = q;
    c = t - q * (q + 1) / 2;
}

template <typename T>
__device__ __forceinline__ double ld(const void *p, int64_t i)
{
    return (double)((const T *)p)[i];
}

template <typename VT, typename XT, int MT>
__global__ __launch_bounds__(256) void rows_f64_kernel(SideArgs a, int K, double alpha,
                                                       double rbar, HyperDev hyp, DrawSrc draws,
                                                       const int32_t *list,
                                                       const int32_t *list_count,
                                                       int64_t max_rows, DevState *state)
{
    extern __shared__ double sm[];
    __shared__ int s_flag;
    __shared__ int s_idx[F64_CH];
    const int tid = threadIdx.x;
    const int nb = (K + 3) >> 2;
    const int KS = nb * 4;
    const int T = nb * (nb + 1) / 2;
    double *P = sm;                   // K*K
    double *bv = P + K * K;           // K
    double *zv = bv + K;              // K
    double *stage = zv + K;           // F64_CH * KS
    double *rv = stage + F64_CH * KS; // F64_CH

    int tr[MT], tc[MT];
    bool tv[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        int t = tid + 256 * m;
        tv[m] = t < T;
        tri_decode(tv[m] ? t : 0, tr[m], tc[m]);
    }
    const XT *other = (const XT *)a.other;
    XT *X = (XT *)a.X;
    const uint32_t h = draws.tape_rows ? 0u : half_sweep_index(draws);

    const int64_t count = list ? (int64_t)(*list_count) : max_rows;
    for (int64_t item = blockIdx.x; item < count; item += gridDim.x) {
        const int row = list ? list[item] : (a.order ? a.order[item] : (int)item);
        const int64_t s0 = a.ptr[row], s1 = a.ptr[row + 1];

        double acc[MT][16];
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[m][e] = 0.0;
        double bacc = 0.0;

        for (int64_t c0 = s0; c0 < s1; c0 += F64_CH) {
            const int cnt = (int)min((int64_t)F64_CH, s1 - c0);
            if (tid < F64_CH) {
                // clamped indices: every load is valid, so they are not masked
                const int tc = tid < cnt ? tid : cnt - 1;
                s_idx[tid] = blend_idx(tid < cnt, a.idx[c0 + tc], 0);
                rv[tid] = (ld<VT>(a.val, c0 + tc) - rbar) * (tid < cnt ? 1.0 : 0.0);
            }
            __syncthreads();
            for (int e = tid; e < F64_CH * KS; e += 256) {
                int n = e / KS, f = e - n * KS;
                stage[e] = (double)other[(int64_t)s_idx[n] * K + (f < K ? f : K - 1)] * ((n < cnt && f < K) ? 1.0 : 0.0);
            }
            __syncthreads();
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                if (!tv[m]) continue;
                for (int n = 0; n < cnt; ++n) {
                    const double *sr = stage + n * KS;
                    double x0 = sr[4 * tr[m] + 0], x1 = sr[4 * tr[m] + 1];
                    double x2 = sr[4 * tr[m] + 2], x3 = sr[4 * tr[m] + 3];
                    double y0 = sr[4 * tc[m] + 0], y1 = sr[4 * tc[m] + 1];
                    double y2 = sr[4 * tc[m] + 2], y3 = sr[4 * tc[m] + 3];
                    double xs[4] = {x0, x1, x2, x3}, ys[4] = {y0, y1, y2, y3};
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int j = 0; j < 4; ++j) acc[m][i * 4 + j] = fma(xs[i], ys[j], acc[m][i * 4 + j]);
                }
            }
            if (tid < K)
                for (int n = 0; n < cnt; ++n) bacc = fma(rv[n], stage[n * KS + tid], bacc);
            __syncthreads();
        }

        // P = Lambda + alpha G (lower triangle), b = Lambda mu + alpha sum r' v
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            if (!tv[m]) continue;
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    int r = 4 * tr[m] + i, c = 4 * tc[m] + j;
                    if (r < K && c <= r) P[r * K + c] = hyp.Lambda[r * K + c] + alpha * acc[m][i * 4 + j];
                }
        }
        if (tid < K) bv[tid] = hyp.Lmu[tid] + alpha * bacc;
        if (draws.tape_rows) {
            for (int i = tid; i < K; i += 256) zv[i] = draws.tape_rows[(int64_t)row * K + i];
        } else {
            for (int p = tid; 2 * p < K; p += 256) {
                double z0, z1;
                box_muller_f64(philox4x32_10(ctr4((uint32_t)p, (uint32_t)row, h, 0u), draws.seed), z0, z1);
                zv[2 * p] = z0;
                if (2 * p + 1 < K) zv[2 * p + 1] = z1;
            }
        }
        if (tid == 0) s_flag = 0;
        __syncthreads();

        // right-looking Cholesky, lower triangle in place
        for (int k = 0; k < K; ++k) {
            if (tid == 0) {
                double d = P[k * K + k];
                if (!(d > 0.0) || !isfinite(d)) {
                    s_flag = 1;
                    d = 1.0;
                }
                P[k * K + k] = sqrt(d);
            }
            __syncthreads();
            const double dk = P[k * K + k];
            for (int i = k + 1 + tid; i < K; i += 256) P[i * K + k] /= dk;
            __syncthreads();
            const int mrem = K - k - 1;
            for (int ii = tid >> 4; ii < mrem; ii += 16) {
                const int i = k + 1 + ii;
                const double lik = P[i * K + k];
                for (int jj = tid & 15; jj <= ii; jj += 16) {
                    const int j = k + 1 + jj;
                    P[i * K + j] = fma(-lik, P[j * K + k], P[i * K + j]);
                }
            }
            __syncthreads();
        }
        // y = L^{-1} b
        for (int k = 0; k < K; ++k) {
            const double yk = bv[k] / P[k * K + k];
            __syncthreads();
            for (int i = k + 1 + tid; i < K; i += 256) bv[i] = fma(-P[i * K + k], yk, bv[i]);
            if (tid == 0) bv[k] = yk;
            __syncthreads();
        }
        // w = y + z ; x = L^{-T} w
        for (int i = tid; i < K; i += 256) bv[i] += zv[i];
        __syncthreads();
        for (int k = K - 1; k >= 0; --k) {
            const double xk = bv[k] / P[k * K + k];
            __syncthreads();
            for (int i = tid; i < k; i += 256) bv[i] = fma(-P[k * K + i], xk, bv[i]);
            if (tid == 0) bv[k] = xk;
            __syncthreads();
        }
        for (int i = tid; i < K; i += 256) {
            const double x = bv[i];
            if (!isfinite(x)) s_flag = 1;
            X[(int64_t)row * K + i] = (XT)x;
            if (a.X_bf16) a.X_bf16[(int64_t)row * a.shadow_stride + i] = f32_to_bf16_rne((float)x);
        }
        if (a.X_bf16)
            for (int i = K + tid; i < a.shadow_stride; i += 256)
                a.X_bf16[(int64_t)row * a.shadow_stride + i] = 0;
        __syncthreads();
        if (tid == 0 && s_flag) atomicAdd((unsigned long long *)&state->nonfinite_rows, 1ull);
        __syncthreads();
    }
}

// Side statistics on FP64 matrix cores (K <= 64): one wavefront per chunk of
// rows; every 4 rows feed v_mfma_f64_16x16x4_f64 for each lower 16x16 tile
// of sum x x^T (operand lane l = row l/16 of the group, feature l%16 of the
// block; accumulator lane l, element v = tile row 4v + l/16, column l%16).
typedef double f64x4 __attribute__((ext_vector_type(4)));
constexpr int STATS_THREADS = 512;

// The Normal-Wishart randoms of one half-sweep, in the tape layout (see the
// hyper-parameter kernel): K chi^2(nu* - k) by Marsaglia-Tsang, then the
// Bartlett and mean normals (normal q of a stream is member q % 2 of the
// Box-Muller pair q / 2).
__device__ void nw_draws_block(const DrawSrc &d, int K, double nstar, double *out)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    const int NB = K * (K - 1) / 2;
    const uint32_t h = half_sweep_index(d);
    for (int k = tid; k < K; k += nt) out[k] = 2.0 * gamma_mt(d.seed, h, (uint32_t)k, 0.5 * (nstar - (double)k));
    for (int p = tid; 2 * p < NB; p += nt) {
        double z0, z1;
        box_muller_f64(philox4x32_10(ctr4((uint32_t)p, 0u, h, 1u), d.seed), z0, z1);
        out[K + 2 * p] = z0;
        if (2 * p + 1 < NB) out[K + 2 * p + 1] = z1;
    }
    for (int p = tid; 2 * p < K; p += nt) {
        double z0, z1;
        box_muller_f64(philox4x32_10(ctr4((uint32_t)p, 0u, h, 2u), d.seed), z0, z1);
        out[K + NB + 2 * p] = z0;
        if (2 * p + 1 < K) out[K + NB + 2 * p + 1] = z1;
    }
}

template <typename XT, int NB>
__global__ __launch_bounds__(STATS_THREADS) void stats_mfma_kernel(StatsSides ss, int K)
{
    const int nstat = ss.n_chunks[0] + ss.n_chunks[1];
    if ((int)blockIdx.x >= nstat) {
        const int sd = (int)blockIdx.x - nstat;
        nw_draws_block(ss.draws[sd], K, ss.nu0 + (double)ss.n[sd], ss.draw_out[sd]);
        return;
    }
    // blocks [0, n_chunks[0]) take side 0, the rest side 1
    const int side = (int)blockIdx.x >= ss.n_chunks[0] ? 1 : 0;
    const XT *X = (const XT *)ss.X[side];
    const int64_t n = ss.n[side];
    double *partials = ss.partials[side];
    const int n_chunks = ss.n_chunks[side];
    const int chunk = (int)blockIdx.x - (side ? ss.n_chunks[0] : 0);
    constexpr int NT = NB * (NB + 1) / 2;
    constexpr int NWV = STATS_THREADS / 64;       // wavefronts per block (two per SIMD)
    constexpr int PER_WAVE = (4 * NT + NB) * 64;  // doubles one wave contributes to the reduction
    __shared__ double red[NWV / 2][PER_WAVE];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t r0 = n * chunk / n_chunks, r1 = n * (chunk + 1) / n_chunks;
    const int i16 = lane & 15, g = lane >> 4;
    f64x4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
    double sx[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) sx[b] = 0.0;
    // wave w takes row groups r0 + 4 (w + NWV i), GB groups at a time: all
    // their loads are issued before any of them is multiplied
    constexpr int GB = 8;
    for (int64_t q0 = r0 + 4 * wave; q0 < r1; q0 += 4 * NWV * GB) {
        double x[GB][NB];
#pragma unroll
        for (int u = 0; u < GB; ++u) {
            const int64_t r = q0 + 4 * NWV * u + g;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int f = 16 * b + i16;
                // clamped indices (r1 > r0 here): the loads carry no lane masks
                // and are issued together
                x[u][b] = (double)X[(r < r1 ? r : r1 - 1) * K + (f < K ? f : K - 1)] * ((r < r1 && f < K) ? 1.0 : 0.0);
            }
        }
#pragma unroll
        for (int u = 0; u < GB; ++u) {
            int t = 0;
#pragma unroll
            for (int a = 0; a < NB; ++a)
#pragma unroll
                for (int b = 0; b <= a; ++b, ++t)
                    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[u][a], x[u][b], acc[t], 0, 0, 0);
#pragma unroll
            for (int b = 0; b < NB; ++b) sx[b] += x[u][b];
        }
    }
    // fixed-order tree reduction of the waves: w += w + NWV/2, then halves
    auto put = [&](double *dst) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) dst[(t * 4 + v) * 64 + lane] = acc[t][v];
#pragma unroll
        for (int b = 0; b < NB; ++b) dst[(4 * NT + b) * 64 + lane] = sx[b];
    };
    auto add = [&](const double *src) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[t][v] += src[(t * 4 + v) * 64 + lane];
#pragma unroll
        for (int b = 0; b < NB; ++b) sx[b] += src[(4 * NT + b) * 64 + lane];
    };
#pragma unroll
    for (int h = NWV / 2; h >= 1; h >>= 1) {
        if (wave >= h && wave < 2 * h) put(red[wave - h]);
        __syncthreads();
        if (wave < h) add(red[wave]);
        __syncthreads();
    }
    if (wave != 0) return;
    const int E = K + K * (K + 1) / 2;
    double *out = partials + (int64_t)chunk * E;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        double v = sx[b];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        const int f = 16 * b + i16;
        if (g == 0 && f < K) out[f] = v;
    }
    int t = 0;
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b, ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int rr = 16 * a + 4 * v + g, cc = 16 * b + i16;
                if (rr < K && cc <= rr) out[K + rr * (rr + 1) / 2 + cc] = acc[t][v];
            }
}

// Side statistics on FP64 matrix cores for 64 < K <= 128: the 36 lower
// 16 x 16 tiles of sum x x^T are dealt to the eight wavefronts of a block
// (tile t to wavefront t % 8, at most five each), so every wavefront runs
// every row of the chunk through its own tiles and no reduction across
// wavefronts is needed.  Rows are staged 32 at a time in LDS (FP32 as
// stored), one coalesced load per thread and row block; wavefront 0 also
// sums x.  Padding features (K <= f < 128) are zero.
constexpr int SB_NB = 8;
constexpr int SB_NT = SB_NB * (SB_NB + 1) / 2;
constexpr int SB_ROWS = 32;

__device__ __forceinline__ void tile_ab(int t, int &a, int &b)
{
    a = 0;
    while ((a + 1) * (a + 2) / 2 <= t) ++a;
    b = t - a * (a + 1) / 2;
}

template <typename XT>
__global__ __launch_bounds__(STATS_THREADS) void stats_mfma_big_kernel(StatsSides ss, int K)
{
    const int nstat = ss.n_chunks[0] + ss.n_chunks[1];
    if ((int)blockIdx.x >= nstat) {
        const int sd = (int)blockIdx.x - nstat;
        nw_draws_block(ss.draws[sd], K, ss.nu0 + (double)ss.n[sd], ss.draw_out[sd]);
        return;
    }
    __shared__ double stage[SB_ROWS][SB_NB * 16 + 1];
    const int side = (int)blockIdx.x >= ss.n_chunks[0] ? 1 : 0;
    const XT *X = (const XT *)ss.X[side];
    const int64_t n = ss.n[side];
    double *partials = ss.partials[side];
    const int n_chunks = ss.n_chunks[side];
    const int chunk = (int)blockIdx.x - (side ? ss.n_chunks[0] : 0);
    constexpr int NWV = STATS_THREADS / 64;
    constexpr int TPW = (SB_NT + NWV - 1) / NWV;  // tiles per wavefront (5)
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int i16 = lane & 15, g = lane >> 4;
    const int64_t r0 = n * chunk / n_chunks, r1 = n * (chunk + 1) / n_chunks;
    f64x4 acc[TPW];
    int ta[TPW], tb[TPW];
#pragma unroll
    for (int j = 0; j < TPW; ++j) {
        acc[j] = f64x4{0.0, 0.0, 0.0, 0.0};
        const int t = wave + NWV * j;
        tile_ab(t < SB_NT ? t : 0, ta[j], tb[j]);
    }
    double sx[SB_NB];
#pragma unroll
    for (int b = 0; b < SB_NB; ++b) sx[b] = 0.0;
    for (int64_t c0 = r0; c0 < r1; c0 += SB_ROWS) {
        const int cnt = (int)min((int64_t)SB_ROWS, r1 - c0);
        for (int e = tid; e < SB_ROWS * SB_NB * 16; e += STATS_THREADS) {
            const int q = e / (SB_NB * 16), f = e - q * (SB_NB * 16);
            // clamped indices, zero beyond the chunk and the padding features
            stage[q][f] = (double)X[(c0 + (q < cnt ? q : cnt - 1)) * K + (f < K ? f : K - 1)] *
                          ((q < cnt && f < K) ? 1.0 : 0.0);
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < SB_ROWS / 4; ++u) {
            const double *xr = stage[4 * u + g];
#pragma unroll
            for (int j = 0; j < TPW; ++j)
                if (wave + NWV * j < SB_NT)
                    acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(xr[16 * ta[j] + i16], xr[16 * tb[j] + i16], acc[j],
                                                                  0, 0, 0);
            if (wave == 0)
#pragma unroll
                for (int b = 0; b < SB_NB; ++b) sx[b] += xr[16 * b + i16];
        }
        __syncthreads();
    }
    double *out = partials + (int64_t)chunk * (K + K * (K + 1) / 2);
    if (wave == 0) {
#pragma unroll
        for (int b = 0; b < SB_NB; ++b) {
            double v = sx[b];
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            const int f = 16 * b + i16;
            if (g == 0 && f < K) out[f] = v;
        }
    }
#pragma unroll
    for (int j = 0; j < TPW; ++j) {
        if (wave + NWV * j >= SB_NT) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int rr = 16 * ta[j] + 4 * v + g, cc = 16 * tb[j] + i16;
            if (rr < K && cc <= rr) out[K + rr * (rr + 1) / 2 + cc] = acc[j][v];
        }
    }
}

// 16 lanes per group of 4 consecutive (row-sorted) pairs: all eight factor
// row reads of a lane are issued together, FP64 accumulation, shuffle
// reduction inside the 16-lane group.
template <typename XT>
__global__ __launch_bounds__(256) void predict_kernel(const XT *U, const XT *V, int K, double rbar,
                                                      int64_t n, const int32_t *rows,
                                                      const int32_t *cols, double *out,
                                                      double *accum, const DevState *state,
                                                      int burnin)
{
    constexpr int PP = 4;
    const int64_t t0 = (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4) * PP;
    const int l = threadIdx.x & 15;
    double p[PP];
    const XT *u[PP], *v[PP];
#pragma unroll
    for (int q = 0; q < PP; ++q) {
        p[q] = 0.0;
        const int64_t t = t0 + q < n ? t0 + q : n - 1;
        u[q] = U + (int64_t)rows[t] * K;
        v[q] = V + (int64_t)cols[t] * K;
    }
    for (int f = l; f < K; f += 16) {
        XT a[PP], b[PP];
#pragma unroll
        for (int q = 0; q < PP; ++q) {
            a[q] = u[q][f];
            b[q] = v[q][f];
        }
#pragma unroll
        for (int q = 0; q < PP; ++q) p[q] = fma((double)a[q], (double)b[q], p[q]);
    }
#pragma unroll
    for (int q = 0; q < PP; ++q)
#pragma unroll
        for (int o = 8; o >= 1; o >>= 1) p[q] += __shfl_xor(p[q], o, 16);
    if (l < PP && t0 + l < n) {
        double r = p[0];
#pragma unroll
        for (int q = 1; q < PP; ++q) r = (l == q) ? p[q] : r;
        r += rbar;
        const int64_t t = t0 + l;
        if (out) out[t] = r;
        if (accum && state->sweep >= burnin) accum[t] += r;
    }
}

__global__ void advance_kernel(DevState *s, int burnin)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (s->sweep >= burnin) s->pred_count += 1;
        s->fallback_rows += s->fb_count[0] + s->fb_count[1];
        s->fb_count[0] = 0;  // the next sweep's recompute lists start empty
        s->fb_count[1] = 0;
        s->sweep += 1;
    }
}

// Deterministic sum of the rating values: block b adds a fixed strided subset
// in a fixed order, then a fixed-shape tree inside the block.
template <typename VT>
__global__ void sum_values_kernel(const VT *v, int64_t n, double *partials)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) s += (double)v[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

__global__ void mean_from_sum_kernel(const double *accum, const int64_t *perm, int64_t n,
                                     const DevState *state, double *out)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int64_t c = state->pred_count;
    out[perm[t]] = c > 0 ? accum[t] / (double)c : 0.0;
}


__global__ void to_bf16_kernel(const float *X, int64_t n, int K, int stride, uint16_t *out)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * stride) return;
    int64_t r = t / stride;
    int c = (int)(t - r * stride);
    out[t] = c < K ? f32_to_bf16_rne(X[r * K + c]) : (uint16_t)0;
}

__global__ void f64_to_f32_kernel(const double *in, float *out, int64_t n)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) out[t] = (float)in[t];
}

__global__ void fill_zero_kernel(uint32_t *p, int64_t n_words)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n_words) p[t] = 0u;
}

template <typename XT>
__global__ void copy_f32_kernel(const XT *in, float *out, int64_t n)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) out[t] = (float)in[t];
}

inline unsigned grid_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

size_t rows_f64_lds_bytes(int K)
{
    const int KS = ((K + 3) >> 2) * 4;
    return sizeof(double) * ((size_t)K * K + 2 * K + (size_t)F64_CH * KS + F64_CH);
}

hipError_t launch_rows_f64(const SideArgs &a, int K, double alpha, double rbar, HyperDev hyp,
                           DrawSrc draws, const int32_t *list, const int32_t *list_count,
                           int64_t max_rows, int x_is_f32, DevState *state, hipStream_t s)
{
    if (max_rows <= 0) return hipSuccess;
    const size_t lds = rows_f64_lds_bytes(K);
    const int nb = (K + 3) >> 2;
    (void)0;
    const bool big = nb * (nb + 1) / 2 > 256;
    unsigned grid = list ? (unsigned)std::min<int64_t>(max_rows, 2048) : (unsigned)max_rows;
#define BPMF_LAUNCH_F64(VT, XT, MT)                                                              \
    do {                                                                                          \
        auto kfn = rows_f64_kernel<VT, XT, MT>;                                                   \
        hipLaunchKernelGGL(kfn, dim3(grid), dim3(256), lds, s, a, K, alpha, rbar, hyp, draws,     \
                           list, list_count, max_rows, state);                                    \
    } while (0)
    if (a.val_is_f64) {
        if (x_is_f32) {
            if (big) BPMF_LAUNCH_F64(double, float, 3); else BPMF_LAUNCH_F64(double, float, 1);
        } else {
            if (big) BPMF_LAUNCH_F64(double, double, 3); else BPMF_LAUNCH_F64(double, double, 1);
        }
    } else {
        if (x_is_f32) {
            if (big) BPMF_LAUNCH_F64(float, float, 3); else BPMF_LAUNCH_F64(float, float, 1);
        } else {
            if (big) BPMF_LAUNCH_F64(float, double, 3); else BPMF_LAUNCH_F64(float, double, 1);
        }
    }
#undef BPMF_LAUNCH_F64
    return hipGetLastError();
}

hipError_t prepare_rows_f64(int K)
{
    const int lds = (int)rows_f64_lds_bytes(K);
    const void *fns[] = {(const void *)rows_f64_kernel<double, double, 1>, (const void *)rows_f64_kernel<double, double, 3>,
                         (const void *)rows_f64_kernel<double, float, 1>, (const void *)rows_f64_kernel<double, float, 3>,
                         (const void *)rows_f64_kernel<float, double, 1>, (const void *)rows_f64_kernel<float, double, 3>,
                         (const void *)rows_f64_kernel<float, float, 1>, (const void *)rows_f64_kernel<float, float, 3>};
    for (const void *f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_sum_values(const void *vals, int is_f64, int64_t n, double *partials, int nblk, hipStream_t s)
{
    if (is_f64) hipLaunchKernelGGL(sum_values_kernel<double>, dim3(nblk), dim3(256), 0, s, (const double *)vals, n, partials);
    else hipLaunchKernelGGL(sum_values_kernel<float>, dim3(nblk), dim3(256), 0, s, (const float *)vals, n, partials);
    return hipGetLastError();
}

hipError_t launch_mean_from_sum(const double *accum, const int64_t *perm, int64_t n, const DevState *state,
                                double *out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(mean_from_sum_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, accum, perm, n, state, out);
    return hipGetLastError();
}

// Row chunks of the side statistics (one 512-thread block per chunk): the two
// sides share one round of the blocks the device holds at once (`slots`, less
// the two blocks that draw the Normal-Wishart randoms) in
// proportion to their rows, at least 64 rows a chunk, so no compute unit runs
// a block after the others are done.
int stats_chunks(int64_t n, int64_t n_other, int K, int slots)
{
    const int64_t budget = std::max(2, slots - 2);
    const int64_t c = budget * n / std::max<int64_t>(1, n + n_other);
    return (int)std::max<int64_t>(1, std::min<int64_t>(c, (n + 63) / 64));
}

// Blocks of the statistics kernel for K the current device holds at once
// (compute units x blocks per unit); 256 when the queries fail.
int stats_slots(int K, int x_is_f64)
{
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        return 256;
    const int NB = (K + 15) / 16;
    const void *fn = nullptr;
#define BPMF_STATS_FN(XT, N) fn = (const void *)stats_mfma_kernel<XT, N>
    if (K > 64)
        fn = x_is_f64 ? (const void *)stats_mfma_big_kernel<double> : (const void *)stats_mfma_big_kernel<float>;
    else if (x_is_f64) {
        if (NB == 1) BPMF_STATS_FN(double, 1);
        else if (NB == 2) BPMF_STATS_FN(double, 2);
        else if (NB == 3) BPMF_STATS_FN(double, 3);
        else BPMF_STATS_FN(double, 4);
    } else {
        if (NB == 1) BPMF_STATS_FN(float, 1);
        else if (NB == 2) BPMF_STATS_FN(float, 2);
        else if (NB == 3) BPMF_STATS_FN(float, 3);
        else BPMF_STATS_FN(float, 4);
    }
#undef BPMF_STATS_FN
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, STATS_THREADS, 0) != hipSuccess || per <= 0) per = 1;
    return cus * per;
}

hipError_t launch_stats(const StatsSides &ss, int x_is_f64, int K, hipStream_t s)
{
    if (K <= 64) {
        const int NB = (K + 15) / 16;
        const unsigned grid = (unsigned)(ss.n_chunks[0] + ss.n_chunks[1] + (ss.with_draws ? 2 : 0));
        if (grid == 0) return hipSuccess;
#define BPMF_STATS_MFMA(XT, NBV) \
    hipLaunchKernelGGL((stats_mfma_kernel<XT, NBV>), dim3(grid), dim3(STATS_THREADS), 0, s, ss, K)
        if (x_is_f64) {
            if (NB == 1) BPMF_STATS_MFMA(double, 1);
            else if (NB == 2) BPMF_STATS_MFMA(double, 2);
            else if (NB == 3) BPMF_STATS_MFMA(double, 3);
            else BPMF_STATS_MFMA(double, 4);
        } else {
            if (NB == 1) BPMF_STATS_MFMA(float, 1);
            else if (NB == 2) BPMF_STATS_MFMA(float, 2);
            else if (NB == 3) BPMF_STATS_MFMA(float, 3);
            else BPMF_STATS_MFMA(float, 4);
        }
#undef BPMF_STATS_MFMA
        return hipGetLastError();
    }
    if (K <= SB_NB * 16) {
        const unsigned grid = (unsigned)(ss.n_chunks[0] + ss.n_chunks[1] + (ss.with_draws ? 2 : 0));
        if (grid == 0) return hipSuccess;
        if (x_is_f64)
            hipLaunchKernelGGL((stats_mfma_big_kernel<double>), dim3(grid), dim3(STATS_THREADS), 0, s, ss, K);
        else
            hipLaunchKernelGGL((stats_mfma_big_kernel<float>), dim3(grid), dim3(STATS_THREADS), 0, s, ss, K);
        return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

// FP32 factors with K a multiple of 4 and at most 64 NV: lane l of a 16-lane
// group loads features 4l..4l+3 (and 64 + 4l.. when NV = 2) of each of its
// group's 4 pairs as 16-byte loads, so a group reads its 4 U rows and 4 V rows
// in one round trip.
template <int NV>
__global__ __launch_bounds__(256) void predict_vec4_kernel(const float *U, const float *V, int K, double rbar,
                                                           int64_t n, const int32_t *rows, const int32_t *cols,
                                                           double *out, double *accum, const DevState *state,
                                                           int burnin)
{
    constexpr int PP = 4;
    const int64_t t0 = (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4) * PP;
    const int l = threadIdx.x & 15;
    bool lane_on[NV];
    int fo[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        lane_on[v] = 64 * v + 4 * l < K;
        fo[v] = lane_on[v] ? 64 * v + 4 * l : 0;  // clamped: the loads stay unmasked
    }
    float4 a[PP][NV], b[PP][NV];
#pragma unroll
    for (int q = 0; q < PP; ++q) {
        const int64_t t = t0 + q < n ? t0 + q : n - 1;
        const float *ur = U + (int64_t)rows[t] * K, *vr = V + (int64_t)cols[t] * K;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            a[q][v] = *(const float4 *)(ur + fo[v]);
            b[q][v] = *(const float4 *)(vr + fo[v]);
        }
    }
    double p[PP];
#pragma unroll
    for (int q = 0; q < PP; ++q) {
        double s = 0.0;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double sv = 0.0;
            sv = fma((double)a[q][v].x, (double)b[q][v].x, sv);
            sv = fma((double)a[q][v].y, (double)b[q][v].y, sv);
            sv = fma((double)a[q][v].z, (double)b[q][v].z, sv);
            sv = fma((double)a[q][v].w, (double)b[q][v].w, sv);
            s += lane_on[v] ? sv : 0.0;
        }
        p[q] = s;
    }
#pragma unroll
    for (int q = 0; q < PP; ++q)
#pragma unroll
        for (int o = 8; o >= 1; o >>= 1) p[q] += __shfl_xor(p[q], o, 16);
    if (l < PP && t0 + l < n) {
        double r = p[0];
#pragma unroll
        for (int q = 1; q < PP; ++q) r = (l == q) ? p[q] : r;
        r += rbar;
        const int64_t t = t0 + l;
        if (out) out[t] = r;
        if (accum && state->sweep >= burnin) accum[t] += r;
    }
}

hipError_t launch_predict(const void *U, const void *V, int x_is_f64, int K, double rbar, int64_t n,
                          const int32_t *rows, const int32_t *cols, double *out, double *accum,
                          const DevState *state, int burnin, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (x_is_f64)
        hipLaunchKernelGGL(predict_kernel<double>, dim3(grid_for((n + 3) / 4 * 16, 256)), dim3(256), 0, s,
                           (const double *)U, (const double *)V, K, rbar, n, rows, cols, out, accum, state, burnin);
    else if (K % 4 == 0 && K <= 128 && ((uintptr_t)U % 16 == 0) && ((uintptr_t)V % 16 == 0)) {
        if (K <= 64)
            hipLaunchKernelGGL(predict_vec4_kernel<1>, dim3(grid_for((n + 3) / 4 * 16, 256)), dim3(256), 0, s,
                               (const float *)U, (const float *)V, K, rbar, n, rows, cols, out, accum, state, burnin);
        else
            hipLaunchKernelGGL(predict_vec4_kernel<2>, dim3(grid_for((n + 3) / 4 * 16, 256)), dim3(256), 0, s,
                               (const float *)U, (const float *)V, K, rbar, n, rows, cols, out, accum, state, burnin);
    }
    else
        hipLaunchKernelGGL(predict_kernel<float>, dim3(grid_for((n + 3) / 4 * 16, 256)), dim3(256), 0, s,
                           (const float *)U, (const float *)V, K, rbar, n, rows, cols, out, accum, state, burnin);
    return hipGetLastError();
}

hipError_t launch_advance_burnin(DevState *state, int burnin, hipStream_t s)
{
    hipLaunchKernelGGL(advance_kernel, dim3(1), dim3(64), 0, s, state, burnin);
    return hipGetLastError();
}


hipError_t launch_to_bf16(const float *X, int64_t n, int K, int stride, uint16_t *out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_for(n * stride, 256)), dim3(256), 0, s, X, n, K, stride, out);
    return hipGetLastError();
}

hipError_t launch_f64_to_f32(const double *in, float *out, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(f64_to_f32_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, in, out, n);
    return hipGetLastError();
}

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s)
{
    int64_t words = (int64_t)(bytes / 4);
    if (words <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for(words, 256)), dim3(256), 0, s, (uint32_t *)p, words);
    return hipGetLastError();
}

hipError_t launch_copy_f32_from(const void *X, int x_is_f64, int64_t n, float *out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (x_is_f64)
        hipLaunchKernelGGL(copy_f32_kernel<double>, dim3(grid_for(n, 256)), dim3(256), 0, s, (const double *)X, out, n);
    else
        hipLaunchKernelGGL(copy_f32_kernel<float>, dim3(grid_for(n, 256)), dim3(256), 0, s, (const float *)X, out, n);
    return hipGetLastError();
}

}  // namespace bpmf
