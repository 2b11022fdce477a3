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
// One workgroup per side, both sides in one launch, every work matrix in LDS.
#include "common.hpp"
#include "rng.hpp"

namespace bpmf {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

// sums[e] = sum over chunks of partials[c][e]: 8 threads per entry over fixed
// chunk ranges, combined by a fixed xor tree.
__global__ __launch_bounds__(256) void stats_reduce_kernel(StatsSides ss, double *sums0, double *sums1,
                                                           int E, int blocks_per_side)
{
    const int side = (int)blockIdx.x >= blocks_per_side ? 1 : 0;
    const double *partials = ss.partials[side];
    const int n_chunks = ss.n_chunks[side];
    double *sums = side ? sums1 : sums0;
    const int e = ((int)blockIdx.x - side * blocks_per_side) * 32 + (threadIdx.x >> 3);
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

// ---------------------------------------------------------------------------
__device__ __forceinline__ double readlane_d(double v, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// 64 < K <= 128: both sides in one launch, one 512-thread workgroup per side,
// every matrix in LDS as a packed lower triangle (row k at k (k + 1) / 2):
//  * PL holds P (lower part), then row by row R^T: the factorisation from the
//    last pivot computes column k of R, R_ik = P_ki / R_kk (i < k), into row
//    k of PL in place.  It runs in panels of 8 columns: wavefront 0 factors a
//    panel with rows l and l + 64 on lane l (pivots and in-panel values
//    broadcast by readlane), copies the panel's columns into `pan`, and then
//    all wavefronts remove the panel's rank-8 part from the leading block;
//  * TL holds A (Bartlett factor, written straight from the draws) and then
//    T, the solution of R^T T = A (R_mi with m < i is PL(i, m)), in blocks of
//    8 rows: wavefront 0 solves a block with columns l and l + 64 on lane l,
//    then all wavefronts remove the block from the rows below;
//  * Lambda = T T^T (and the packed FP32 copy the 128-wide row kernel reads)
//    goes to global memory; the mean solve T^T d = z / sqrt(beta*) runs on
//    one wavefront; Lambda mu = T (T^T mu).
// Every element of P sees the same sequence of multiply-adds as in an
// unblocked right-looking factorisation.  Two packed 128 x 128 triangles, the
// panel buffer and the vectors take 146 KB of LDS.
// ---------------------------------------------------------------------------
constexpr int NWP_THREADS = 512;
constexpr int NWP_MAXK = 128;
constexpr int NWP_W = 8;  // panel width

__host__ __device__ constexpr size_t nw_packed_lds_doubles(int K)
{
    return (size_t)K * (K + 1) + 7 * (size_t)K + (size_t)NWP_W * NWP_MAXK;
}

__device__ __forceinline__ int ptri(int r, int c) { return r * (r + 1) / 2 + c; }

__global__ __launch_bounds__(NWP_THREADS) void nw_packed_kernel(NwSide side0, NwSide side1, int K,
                                                                const double *mu0, double beta0, double nu0,
                                                                const double *W0inv, DevState *state)
{
    extern __shared__ double lds[];
    __shared__ int s_flag;
    const NwSide sd = blockIdx.x == 0 ? side0 : side1;
    const double *sums = sd.sums;
    const int tid = threadIdx.x, lane = tid & 63;
    // wavefront index in a scalar register: the branches on it are uniform
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int KT = K * (K + 1) / 2;
    double *PL = lds;             // P, then R^T (packed lower)
    double *TL = PL + KT;         // A, then T (packed lower)
    double *xbar = TL + KT;       // K
    double *rd = xbar + K;        // K: 1 / diagonal of R
    double *chi2 = rd + K;        // K
    double *zm = chi2 + K;        // K
    double *dvec = zm + K;        // K
    double *dout = dvec + K;      // K
    double *tv = dout + K;        // K: T^T mu
    double *pan = tv + K;         // NWP_W x 128: pan[q * 128 + i] = R_{i, c0 + q} of the current panel
    const double dn = (double)sd.n;
    const double bstar = beta0 + dn;

    if (tid == 0) s_flag = 0;
    // draws (always a tape: the statistics launch draws them when the sampler
    // draws on the device): chi^2 and mean normals into vectors, Bartlett
    // normals straight into TL
    const double *tape = sd.draws.tape_nw;
    for (int k = tid; k < K; k += NWP_THREADS) chi2[k] = tape[k];
    for (int q = tid; q < K; q += NWP_THREADS) zm[q] = tape[K + K * (K - 1) / 2 + q];
    for (int a = tid; a < K; a += NWP_THREADS) xbar[a] = sd.n > 0 ? sums[a] / dn : 0.0;
    __syncthreads();
    // A: the Bartlett normal q = i (i - 1) / 2 + c at (i, c), c < i, and
    // sqrt(chi^2) on the diagonal; P = W0^{-1} + S + coef (xbar - mu0)(xbar - mu0)^T,
    // lower part; one row per 16 threads
    {
        const double coef = beta0 * dn / bstar;
        for (int i = tid >> 4; i < K; i += NWP_THREADS / 16) {
            for (int c = tid & 15; c <= i; c += 16) {
                const int e = ptri(i, c), q = i * (i - 1) / 2 + c;
                const double v = tape[c == i ? 0 : K + q];
                TL[e] = c == i ? sqrt(chi2[c]) : v;
                const double S = sums[K + e] - dn * xbar[i] * xbar[c];
                PL[e] = W0inv[i * K + c] + S + coef * (xbar[i] - mu0[i]) * (xbar[c] - mu0[c]);
            }
        }
    }
    __syncthreads();

    // P = R R^T from the last pivot up, 8-column panels [c0, c1)
    for (int c1 = K; c1 > 0; c1 -= NWP_W) {
        const int c0 = c1 > NWP_W ? c1 - NWP_W : 0, w = c1 - c0;
        if (wave == 0) {
            // a[s][q] = PL(c0 + q, i) for row i = lane + 64 s; entries with
            // i > c0 + q do not exist and are never stored
            double a[2][NWP_W];
#pragma unroll
            for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
                for (int q = 0; q < NWP_W; ++q) {
                    const int i = lane + 64 * s2, k = c0 + q;
                    a[s2][q] = (q < w && i <= k) ? PL[ptri(k, i)] : 0.0;
                }
#pragma unroll
            for (int q = NWP_W - 1; q >= 0; --q) {
                if (q >= w) continue;
                const int k = c0 + q;
                double akk = readlane_d((k >> 6) ? a[1][q] : a[0][q], k & 63);
                if (!(akk > 0.0) || !isfinite(akk)) {
                    if (lane == 0) s_flag = 1;
                    akk = 1.0;
                }
                // 1/sqrt(akk): hardware estimate refined by three Newton steps
                double inv = __builtin_amdgcn_rsq(akk);
                inv = inv * fma(-0.5 * akk * inv, inv, 1.5);
                inv = inv * fma(-0.5 * akk * inv, inv, 1.5);
                inv = inv * fma(-0.5 * akk * inv, inv, 1.5);
                const double rkk = akk * inv;
                if (lane == 0) rd[k] = inv;
#pragma unroll
                for (int s2 = 0; s2 < 2; ++s2) {
                    const int i = lane + 64 * s2;
                    a[s2][q] = i < k ? a[s2][q] * inv : (i == k ? rkk : a[s2][q]);
                }
                // the panel's earlier columns: PL(k2, i) -= R_ik R_{k2,k}, c0 <= k2 < k
#pragma unroll
                for (int q2 = 0; q2 < NWP_W; ++q2) {
                    if (q2 >= q) continue;
                    const int k2 = c0 + q2;
                    const double rk2 = readlane_d((k2 >> 6) ? a[1][q] : a[0][q], k2 & 63);
#pragma unroll
                    for (int s2 = 0; s2 < 2; ++s2) a[s2][q2] = fma(-a[s2][q], rk2, a[s2][q2]);
                }
            }
#pragma unroll
            for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
                for (int q = 0; q < NWP_W; ++q) {
                    const int i = lane + 64 * s2, k = c0 + q;
                    if (q < w && i <= k) PL[ptri(k, i)] = a[s2][q];
                    if (q < w && i < c0) pan[q * NWP_MAXK + i] = a[s2][q];
                }
        }
        __syncthreads();
        if (c0 == 0) break;
        // leading block: PL(i, j) -= R_ik R_jk over the panel, last column
        // first, for j <= i < c0; one row per 16 threads
        for (int i = tid >> 4; i < c0; i += NWP_THREADS / 16) {
            double ri[NWP_W];
#pragma unroll
            for (int q = 0; q < NWP_W; ++q) ri[q] = q < w ? pan[q * NWP_MAXK + i] : 0.0;
            double *row = PL + ptri(i, 0);
            // four entries of the row at a time: their loads are issued together
            for (int j0 = tid & 15; j0 <= i; j0 += 64) {
                double t[4], pv[4][NWP_W];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int j = j0 + 16 * u, jc = j <= i ? j : i;
                    t[u] = row[jc];
#pragma unroll
                    for (int q = 0; q < NWP_W; ++q) pv[u][q] = pan[q * NWP_MAXK + jc];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int q = NWP_W - 1; q >= 0; --q)
                        if (q < w) t[u] = fma(-ri[q], pv[u][q], t[u]);
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (j0 + 16 * u <= i) row[j0 + 16 * u] = t[u];
            }
        }
        __syncthreads();
    }
    __syncthreads();
    // R^T T = A in blocks of 8 rows [i0, i1): T_i = (A_i - sum_{m < i} R_mi T_m) / R_ii
    for (int i0 = 0; i0 < K; i0 += NWP_W) {
        const int i1 = i0 + NWP_W < K ? i0 + NWP_W : K, w = i1 - i0;
        if (wave == 0) {
            // t[s][q] = TL(i0 + q, c) for column c = lane + 64 s (c <= i0 + q)
            double t[2][NWP_W];
#pragma unroll
            for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
                for (int q = 0; q < NWP_W; ++q) {
                    const int c = lane + 64 * s2, i = i0 + q;
                    t[s2][q] = (q < w && c <= i) ? TL[ptri(i, c)] : 0.0;
                }
#pragma unroll
            for (int q = 0; q < NWP_W; ++q) {
                if (q >= w) continue;
                const double irm = rd[i0 + q];
#pragma unroll
                for (int s2 = 0; s2 < 2; ++s2) t[s2][q] *= irm;
#pragma unroll
                for (int q2 = 0; q2 < NWP_W; ++q2) {
                    if (q2 <= q || q2 >= w) continue;
                    const double r = PL[ptri(i0 + q2, i0 + q)];  // R_{i0+q, i0+q2}
#pragma unroll
                    for (int s2 = 0; s2 < 2; ++s2) t[s2][q2] = fma(-r, t[s2][q], t[s2][q2]);
                }
            }
#pragma unroll
            for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
                for (int q = 0; q < NWP_W; ++q) {
                    const int c = lane + 64 * s2, i = i0 + q;
                    if (q < w && c <= i) TL[ptri(i, c)] = t[s2][q];
                }
        }
        __syncthreads();
        if (i1 == K) break;
        // rows below: TL(i, c) -= R_{i0+q, i} T_{i0+q, c} over the block, for
        // i >= i1 and c < i1 (T_{i0+q, c} = 0 for c > i0 + q); one row per 16 threads
        for (int i = i1 + (tid >> 4); i < K; i += NWP_THREADS / 16) {
            double rr[NWP_W];
#pragma unroll
            for (int q = 0; q < NWP_W; ++q) rr[q] = q < w ? PL[ptri(i, i0 + q)] : 0.0;
            double *ti = TL + ptri(i, 0);
            // four entries of the row at a time: their loads are issued together
            for (int cb = tid & 15; cb < i1; cb += 64) {
                double u[4], tv2[4][NWP_W];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int c = cb + 16 * v, cc = c < i1 ? c : i1 - 1;
                    u[v] = ti[cc];
#pragma unroll
                    for (int q = 0; q < NWP_W; ++q) tv2[v][q] = TL[ptri(i0 + q, cc <= i0 + q ? cc : i0 + q)];
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int c = cb + 16 * v;
#pragma unroll
                    for (int q = 0; q < NWP_W; ++q)
                        if (q < w && c <= i0 + q) u[v] = fma(-rr[q], tv2[v][q], u[v]);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    if (cb + 16 * v < i1) ti[cb + 16 * v] = u[v];
            }
        }
        __syncthreads();
    }
    // Lambda = T T^T (T(a, m) = 0 for m > a), entries (a, c) with a >= c and
    // their mirror, one row a per 16 threads; also the padded packed FP32
    // triangle of the 128-wide row kernel (identity in the padding)
    for (int a = tid >> 4; a < NWP_MAXK; a += NWP_THREADS / 16) {
        const double *ta = TL + ptri(a < K ? a : 0, 0);
        float *tri = sd.hyp.Lambda_tri + ptri(a, 0);
        for (int c = tid & 15; c <= a; c += 16) {
            if (a < K) {
                const double *tc = TL + ptri(c, 0);
                double acc = 0.0;
                for (int m = 0; m <= c; ++m) acc = fma(ta[m], tc[m], acc);
                sd.hyp.Lambda[a * K + c] = acc;
                sd.hyp.Lambda[c * K + a] = acc;
                sd.hyp.Lambda_f[a * K + c] = (float)acc;
                sd.hyp.Lambda_f[c * K + a] = (float)acc;
                tri[c] = (float)acc;
            } else {
                tri[c] = a == c ? 1.0f : 0.0f;
            }
        }
    }
    // mean: T^T d = z / sqrt(beta*), column-oriented backward substitution on
    // wavefront 0 with entries l and l + 64 on lane l
    if (wave == 0) {
        const double isb = 1.0 / sqrt(bstar);
        double r0 = lane < K ? zm[lane] * isb : 0.0, r1 = lane + 64 < K ? zm[lane + 64] * isb : 0.0;
        for (int k = K - 1; k >= 0; --k) {
            const double dk = readlane_d(k >= 64 ? r1 : r0, k & 63) / TL[ptri(k, k)];
            if (lane == 0) dout[k] = dk;
            const double t0 = TL[ptri(k, lane < k ? lane : k)], t1 = TL[ptri(k, lane + 64 < k ? lane + 64 : k)];
            if (lane < k) r0 = fma(-t0, dk, r0);
            if (lane + 64 < k) r1 = fma(-t1, dk, r1);
        }
    }
    __syncthreads();
    for (int a = tid; a < K; a += NWP_THREADS) {
        const double mus = (beta0 * mu0[a] + dn * xbar[a]) / bstar;
        sd.hyp.mu[a] = mus + dout[a];
        dvec[a] = mus + dout[a];
    }
    __syncthreads();
    // Lambda mu = T (T^T mu)
    for (int m = tid; m < K; m += NWP_THREADS) {
        double v = 0.0;
        for (int a = m; a < K; ++a) v = fma(TL[ptri(a, m)], dvec[a], v);
        tv[m] = v;
    }
    __syncthreads();
    for (int a = tid; a < K; a += NWP_THREADS) {
        double v = 0.0;
        for (int m = 0; m <= a; ++m) v = fma(TL[ptri(a, m)], tv[m], v);
        sd.hyp.Lmu[a] = v;
        sd.hyp.Lmu_f[a] = (float)v;
    }
    if (tid == 0 && s_flag) atomicAdd((unsigned long long *)&state->nonfinite_rows, 1ull);
}

constexpr int NWK = 64;       // padded size (K <= 64)
constexpr int NPW = 8;        // panel width

// ---------------------------------------------------------------------------
// K <= 64, compact form: P, R and T live in LDS (padded to 64, identity in
// the padding).  One wavefront runs the three sequential parts with one matrix
// row (or column) per lane and an 8-wide panel in registers: the
// factorisation from the last pivot, the solve R^T T = A and the mean solve;
// all four wavefronts draw the random numbers, form P and compute
// Lambda = T T^T.  The loops over panels and rows are not unrolled, so the
// code stays small enough for the instruction cache.
// ---------------------------------------------------------------------------
constexpr int NCS = NWK + 1;  // LDS row stride (doubles) of P/R and T

constexpr int NSUMS = NWK + NWK * (NWK + 1) / 2;  // sum x and packed sum x x^T at K = 64

size_t nw_compact_lds_bytes()
{
    return sizeof(double) * ((size_t)2 * NWK * NCS + 11 * NWK + NSUMS);
}

// NP: the padded size the three sequential parts and Lambda run to (32 when
// K <= 32, else 64); the padding beyond is the identity, which they would
// leave unchanged.  A template parameter, so every loop bound is a constant.
template <int NP>
__global__ __launch_bounds__(256) void nw_compact_kernel(NwSide side0, NwSide side1, int K,
                                                         const double *mu0, double beta0, double nu0,
                                                         const double *W0inv, DevState *state)
{
    extern __shared__ double lds[];
    double *Pm = lds;                  // P, then R in its upper triangle (row-major)
    double *Tm = Pm + NWK * NCS;       // A, then T (lower, row-major)
    double *xbar = Tm + NWK * NCS;
    double *chi2 = xbar + NWK, *zm = chi2 + NWK, *vinv = zm + NWK, *dvec = vinv + NWK, *mul = dvec + NWK;
    double *lpart = mul + NWK;         // 4 x 64 partial sums of Lambda mu
    double *mu0s = lpart + 4 * NWK;    // the prior mean
    double *sl = mu0s + NWK;           // the side's sums, copied once
    __shared__ int s_flag;
    const NwSide &sd = blockIdx.x == 0 ? side0 : side1;
    const double *sums = sd.sums;
    const int64_t n = sd.n;
    const DrawSrc draws = sd.draws;
    const HyperDev hyp = sd.hyp;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int NB = K * (K - 1) / 2;
    const double dn = (double)n, bstar = beta0 + dn;

    // Every global read of the side is issued first, together: the sums, the
    // prior's W0^{-1} (16 entries per thread, kept in registers), mu0 and the
    // draws (chi^2 of the Bartlett diagonal, its strict lower part in row-major
    // order q = r (r - 1) / 2 + c, the mean normals; at K <= 64 they always
    // come as a tape, drawn by the statistics launch when the sampler draws on
    // the device).  A = Tm is written whole: the draws below the diagonal,
    // sqrt(chi^2) on it, the identity in the padding and zeros above.
    if (tid == 0) s_flag = 0;
    const double *tape = draws.tape_nw;
    double w0r[NWK * NWK / 256];
#pragma unroll
    for (int u = 0; u < NWK * NWK / 256; ++u) {
        const int e = tid + 256 * u, i = e >> 6, j = e & 63;
        const bool in = i < K && j < K;
        w0r[u] = W0inv[in ? i * K + j : 0] * (in ? 1.0 : 0.0);
    }
    constexpr int SU = (NSUMS + 255) / 256;
    const int E = K + K * (K + 1) / 2;
    double sv[SU];
#pragma unroll
    for (int u = 0; u < SU; ++u) sv[u] = sums[min(tid + 256 * u, E - 1)];
    // (all loads first, unconditionally, so none waits behind a branch)
    double tv[NWK * NWK / 256];
#pragma unroll
    for (int u = 0; u < NWK * NWK / 256; ++u) {
        const int e = tid + 256 * u, r = e >> 6, c = e & 63;
        tv[u] = tape[(r < K && c < r) ? K + r * (r - 1) / 2 + c : 0];
    }
    const int kk = tid < K ? tid : 0;
    const double chi = tape[kk], zq = tape[K + NB + kk], m0 = mu0[kk];
#pragma unroll
    for (int u = 0; u < SU; ++u)
        if (tid + 256 * u < E) sl[tid + 256 * u] = sv[u];
    if (tid < K) {
        mu0s[tid] = m0;
        zm[tid] = zq;
    }
#pragma unroll
    for (int u = 0; u < NWK * NWK / 256; ++u) {
        const int e = tid + 256 * u, r = e >> 6, c = e & 63;
        if (!(r < K && c == r)) Tm[r * NCS + c] = (r < K && c < r) ? tv[u] : (c == r ? 1.0 : 0.0);
    }
    if (tid < K) Tm[tid * NCS + tid] = sqrt(chi);
    __syncthreads();
    for (int a = tid; a < NWK; a += 256) xbar[a] = (a < K && n > 0) ? sl[a] / dn : 0.0;
    __syncthreads();
    // P = W0^{-1} + S + coef (xbar - mu0)(xbar - mu0)^T, identity padding
    {
        const double coef = beta0 * dn / bstar;
#pragma unroll
        for (int u = 0; u < NWK * NWK / 256; ++u) {
            const int e = tid + 256 * u, i = e >> 6, j = e & 63;
            double v = (i == j) ? 1.0 : 0.0;
            if (i < K && j < K) {
                const int hi = i > j ? i : j, lo = i > j ? j : i;
                const double S = sl[K + hi * (hi + 1) / 2 + lo] - dn * xbar[i] * xbar[j];
                v = w0r[u] + S + coef * (xbar[i] - mu0s[i]) * (xbar[j] - mu0s[j]);
            }
            Pm[i * NCS + j] = v;
        }
    }
    __syncthreads();

    // P = R R^T from the last pivot up, 8-column panels.  Wavefront 0 factors
    // a panel with lane i holding row i; then all four wavefronts update the
    // leading block (columns j < c0 split over the wavefronts).
    for (int c0 = NP - NPW; c0 >= 0; c0 -= NPW) {
        if (wave == 0) {
            double a[NPW];
#pragma unroll
            for (int m = 0; m < NPW; ++m) a[m] = Pm[lane * NCS + c0 + m];
#pragma unroll
            for (int kk = NPW - 1; kk >= 0; --kk) {
                const int k = c0 + kk;
                double pkk = readlane_d(a[kk], k);
                if (!(pkk > 0.0) || !(pkk < INFINITY)) {
                    if (lane == 0) s_flag = 1;
                    pkk = 1.0;
                }
                // 1/sqrt(pkk): hardware estimate refined by three Newton steps
                double y = __builtin_amdgcn_rsq(pkk);
                y = y * fma(-0.5 * pkk * y, y, 1.5);
                y = y * fma(-0.5 * pkk * y, y, 1.5);
                y = y * fma(-0.5 * pkk * y, y, 1.5);
                a[kk] *= y;  // lanes i < k: R_ik; lane k: R_kk
                if (lane == 0) vinv[k] = y;
#pragma unroll
                for (int jj = 0; jj < kk; ++jj) a[jj] = fma(-a[kk], readlane_d(a[kk], c0 + jj), a[jj]);
            }
#pragma unroll
            for (int m = 0; m < NPW; ++m) Pm[lane * NCS + c0 + m] = a[m];
        }
        if (c0 == 0) break;
        __syncthreads();
        {
            double a[NPW];
#pragma unroll
            for (int m = 0; m < NPW; ++m) a[m] = Pm[lane * NCS + c0 + m];
            // leading block: P_ij -= sum over the panel of R_im R_jm, j < c0
#pragma unroll 2
            for (int j = wave; j < c0; j += 4) {
                const double *rj = Pm + j * NCS + c0;
                double t = Pm[lane * NCS + j];
#pragma unroll
                for (int m = 0; m < NPW; ++m) t = fma(-a[m], rj[m], t);
                Pm[lane * NCS + j] = t;
            }
        }
        __syncthreads();
    }
    __syncthreads();
    // R^T T = A, forward over 8-row blocks with lane m holding column m:
    // wavefront 0 solves a block's diagonal part, then all four wavefronts
    // update the rows below (split over the wavefronts)
    for (int i0 = 0; i0 < NP; i0 += NPW) {
        if (wave == 0) {
            double t[NPW];
#pragma unroll
            for (int q = 0; q < NPW; ++q) t[q] = Tm[(i0 + q) * NCS + lane];
#pragma unroll
            for (int q = 0; q < NPW; ++q) {
                t[q] *= vinv[i0 + q];
#pragma unroll
                for (int q2 = q + 1; q2 < NPW; ++q2) t[q2] = fma(-Pm[(i0 + q) * NCS + i0 + q2], t[q], t[q2]);
            }
#pragma unroll
            for (int q = 0; q < NPW; ++q) Tm[(i0 + q) * NCS + lane] = t[q];
        }
        if (i0 + NPW == NP) break;
        __syncthreads();
        {
            double t[NPW];
#pragma unroll
            for (int q = 0; q < NPW; ++q) t[q] = Tm[(i0 + q) * NCS + lane];
#pragma unroll 2
            for (int i = i0 + NPW + wave; i < NP; i += 4) {
                double u = Tm[i * NCS + lane];
#pragma unroll
                for (int q = 0; q < NPW; ++q) u = fma(-Pm[(i0 + q) * NCS + i], t[q], u);
                Tm[i * NCS + lane] = u;
            }
        }
        __syncthreads();
    }
    __syncthreads();
    if (wave == 0) {
        // mean: T^T d = z / sqrt(beta*), backward; lane i holds right-hand side i
        const double it = 1.0 / Tm[lane * NCS + lane];
        double rhs = lane < K ? zm[lane] * (1.0 / sqrt(bstar)) : 0.0;
        for (int k = NP - 1; k >= 0; --k) {
            const double dk = readlane_d(rhs * it, k);
            if (lane == 0) dvec[k] = dk;
            rhs = fma(-Tm[k * NCS + lane], dk, rhs);
        }
        __asm__ volatile("" ::: "memory");  // dvec written by lane 0
        double mu = 0.0;
        if (lane < K) {
            mu = (beta0 * mu0[lane] + dn * xbar[lane]) / bstar + dvec[lane];
            hyp.mu[lane] = mu;
        }
        mul[lane] = mu;
    }
    __syncthreads();

    // Lambda = T T^T on FP64 matrix cores: the ten lower 16 x 16 tiles (ta, tc)
    // of the padded 64 x 64 product, tile (ta, tc) over k < 16 (tc + 1) (T is
    // lower triangular), dealt to the wavefronts so each runs 20 rank-4 steps
    // of v_mfma_f64_16x16x4_f64: wave 0 (3,3) (0,0); wave 1 (2,2) (1,1);
    // wave 2 (3,2) (2,1); wave 3 (3,1) (1,0) (2,0) (3,0).  Operand lane l
    // holds T[16 t + l % 16][4 kk + l / 16]; result element v of lane l is
    // tile entry (4 v + l / 16, l % 16).  The padded T has the identity in the
    // padding, so the product is Lambda with the identity padding.  Lambda
    // also goes into Pm (free after the solve) for Lambda mu.
    {
        const int KPm = K <= 32 ? 32 : 64;  // padded size of the mixed row kernel
        const int i16 = lane & 15, g = lane >> 4;
        auto tile = [&](int ta, int tc) {
            if (16 * ta >= NP) return;
            f64x4 c = {0.0, 0.0, 0.0, 0.0};
            const double *ra = Tm + (16 * ta + i16) * NCS + g, *rc = Tm + (16 * tc + i16) * NCS + g;
            for (int kk = 0; kk < 4 * (tc + 1); ++kk)
                c = __builtin_amdgcn_mfma_f64_16x16x4f64(ra[4 * kk], rc[4 * kk], c, 0, 0, 0);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = 16 * ta + 4 * v + g, cc = 16 * tc + i16;
                const double x = c[v];
                Pm[r * NCS + cc] = x;
                Pm[cc * NCS + r] = x;
                if (r < K && cc < K) {
                    hyp.Lambda[r * K + cc] = x;
                    hyp.Lambda[cc * K + r] = x;
                    hyp.Lambda_f[r * K + cc] = (float)x;
                    hyp.Lambda_f[cc * K + r] = (float)x;
                }
                const int hi = r > cc ? r : cc, lo = r > cc ? cc : r;
                if (hi < KPm) {
                    hyp.Lambda_tri[hi * (hi + 1) / 2 + lo] = (float)x;
                    if (hyp.Lambda_acc) {
                        // Lambda / alpha (the identity in the padding)
                        const float xa = (r < K && cc < K) ? (float)(x / hyp.alpha) : (float)x;
                        const int q0 = lambda_acc_index(r, cc, hyp.acc16), q1 = lambda_acc_index(cc, r, hyp.acc16);
                        if (q0 >= 0) hyp.Lambda_acc[q0] = xa;
                        if (q1 >= 0) hyp.Lambda_acc[q1] = xa;
                    }
                }
            }
        };
        if (wave == 0) {
            tile(3, 3);
            tile(0, 0);
        } else if (wave == 1) {
            tile(2, 2);
            tile(1, 1);
        } else if (wave == 2) {
            tile(3, 2);
            tile(2, 1);
        } else {
            tile(3, 1);
            tile(1, 0);
            tile(2, 0);
            tile(3, 0);
        }
        // T is chol(Lambda): lower with a positive diagonal, Lambda = T T^T
        if (hyp.Lchol) {
            for (int e = tid; e < KPm * KPm; e += 256) {
                const int r = e / KPm, c = e % KPm;
                hyp.Lchol[e] = (r < K && c < K) ? (c <= r ? (float)Tm[r * NCS + c] : 0.0f) : (r == c ? 1.0f : 0.0f);
            }
        }
    }
    __syncthreads();
    // Lambda mu: thread (a, quarter w) sums columns 16 w .. 16 w + 15 of row a
    {
        const int a = lane, cb = 16 * wave;
        double lmu = 0.0;
        if (cb < NP) {
#pragma unroll
            for (int cc = 0; cc < 16; ++cc) lmu = fma(Pm[a * NCS + cb + cc], mul[cb + cc], lmu);
        }
        lpart[wave * NWK + a] = lmu;
    }
    if (hyp.Lchol && wave == 1) {
        // for the rank-one row paths: 1 / T_ll, T^T mu, Lambda_ll and live-component flags
        const int KPm = K <= 32 ? 32 : 64;
        if (lane < KPm) {
            const bool in = lane < K;
            double tmu = 0.0, ll = 0.0;
            for (int k = lane; k < K; ++k) tmu = fma(Tm[k * NCS + lane], mul[k], tmu);
            for (int m = 0; m <= lane && m < K; ++m) ll = fma(Tm[lane * NCS + m], Tm[lane * NCS + m], ll);
            float *ext = hyp.Lchol + KPm * KPm;
            ext[lane] = in ? (float)(1.0 / Tm[lane * NCS + lane]) : 1.0f;
            ext[KPm + lane] = in ? (float)tmu : 0.0f;
            ext[2 * KPm + lane] = in ? (float)ll : 0.0f;
            ext[3 * KPm + lane] = in ? 1.0f : 0.0f;
        }
    }
    __syncthreads();
    if (wave == 0 && lane < K) {
        // the four 16-column partial sums of row lane, in column order
        const double lmu = ((lpart[lane] + lpart[NWK + lane]) + lpart[2 * NWK + lane]) + lpart[3 * NWK + lane];
        hyp.Lmu[lane] = lmu;
        hyp.Lmu_f[lane] = (float)lmu;
    }
    if (tid == 0 && s_flag) atomicAdd((unsigned long long *)&state->nonfinite_rows, 1ull);
}

// Lambda_tri from Lambda_f, and Lambda_acc from the FP64 Lambda (after a
// state restore).
__global__ __launch_bounds__(256) void lambda_tri_kernel(HyperDev hyp, int K, int KP)
{
    for (int t = threadIdx.x; t < KP * KP; t += blockDim.x) {
        const int r = t / KP, c = t - r * KP;
        const float v = (r < K && c < K) ? hyp.Lambda_f[r * K + c] : (r == c ? 1.0f : 0.0f);
        if (c <= r) hyp.Lambda_tri[r * (r + 1) / 2 + c] = v;
        if (hyp.Lambda_acc && KP <= 64) {
            // Lambda / alpha from the FP64 Lambda, as the Normal-Wishart step writes it
            const int q = lambda_acc_index(r, c, hyp.acc16);
            if (q >= 0) hyp.Lambda_acc[q] = (r < K && c < K) ? (float)(hyp.Lambda[r * K + c] / hyp.alpha) : v;
        }
    }
}

}  // namespace

hipError_t prepare_nw()
{
    hipError_t e = hipFuncSetAttribute((const void *)nw_compact_kernel<32>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)nw_compact_lds_bytes());
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)nw_compact_kernel<NWK>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)nw_compact_lds_bytes());
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void *)nw_packed_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(sizeof(double) * nw_packed_lds_doubles(NWP_MAXK)));
}

hipError_t launch_lambda_tri(HyperDev hyp, int K, int KP, hipStream_t s)
{
    if (K > 128) return hipSuccess;
    hipLaunchKernelGGL(lambda_tri_kernel, dim3(1), dim3(256), 0, s, hyp, K, KP);
    return hipGetLastError();
}



hipError_t launch_stats_reduce(const StatsSides &ss, double *const sums[2], int K, hipStream_t s)
{
    const int E = K + K * (K + 1) / 2;
    const int bps = (E + 31) / 32;
    hipLaunchKernelGGL(stats_reduce_kernel, dim3((unsigned)(2 * bps)), dim3(256), 0, s, ss, sums[0], sums[1],
                       E, bps);
    return hipGetLastError();
}

hipError_t launch_nw(const NwSide sides[2], int K, const double *mu0, double beta0, double nu0,
                     const double *W0inv, DevState *state, hipStream_t s)
{
    // the statistics launch always provides the draws as a tape here
    if (!sides[0].draws.tape_nw || !sides[1].draws.tape_nw) return hipErrorInvalidValue;
    if (K <= NWK) {
        if (K <= 32)
            hipLaunchKernelGGL(nw_compact_kernel<32>, dim3(2), dim3(256), nw_compact_lds_bytes(), s, sides[0],
                               sides[1], K, mu0, beta0, nu0, W0inv, state);
        else
            hipLaunchKernelGGL(nw_compact_kernel<NWK>, dim3(2), dim3(256), nw_compact_lds_bytes(), s, sides[0],
                               sides[1], K, mu0, beta0, nu0, W0inv, state);
        return hipGetLastError();
    }
    if (K <= NWP_MAXK) {
        hipLaunchKernelGGL(nw_packed_kernel, dim3(2), dim3(NWP_THREADS), sizeof(double) * nw_packed_lds_doubles(K), s,
                           sides[0], sides[1], K, mu0, beta0, nu0, W0inv, state);
        return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

}  // namespace bpmf
