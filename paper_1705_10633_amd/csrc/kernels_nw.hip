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
// 64 < K <= 128: both sides in one launch, one 512-thread workgroup per side,
// every matrix in LDS as a packed lower triangle (row k at k (k + 1) / 2):
//  * PL holds P (lower part), then row by row R^T: the factorisation from the
//    last pivot computes column k of R, R_ik = P_ki / R_kk (i < k), into row
//    k of PL in place and then removes R_k R_k^T from the leading block;
//  * TL holds A (Bartlett factor, written straight from the draws) and then
//    T, the solution of R^T T = A (R_mi with m < i is PL(i, m));
//  * Lambda = T T^T goes to global memory, Lambda mu = T (T^T mu) and the mean
//    solve T^T d = z / sqrt(beta*) read TL.
// Two packed 128 x 128 triangles and the vectors take 139 KB of LDS.
// ---------------------------------------------------------------------------
constexpr int NWP_THREADS = 512;
constexpr int NWP_MAXK = 128;

__host__ __device__ constexpr size_t nw_packed_lds_doubles(int K)
{
    return (size_t)K * (K + 1) + 7 * (size_t)K;
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
    const int tid = threadIdx.x;
    const int KT = K * (K + 1) / 2;
    double *PL = lds;             // P, then R^T (packed lower)
    double *TL = PL + KT;         // A, then T (packed lower)
    double *xbar = TL + KT;       // K
    double *rd = xbar + K;        // K: diagonal of R
    double *chi2 = rd + K;        // K
    double *zm = chi2 + K;        // K
    double *dvec = zm + K;        // K
    double *dout = dvec + K;      // K
    double *tv = dout + K;        // K: T^T mu
    const double dn = (double)sd.n;
    const double bstar = beta0 + dn, nstar = nu0 + dn;

    if (tid == 0) s_flag = 0;
    // draws: chi^2 and mean normals into vectors, Bartlett normals straight into TL
    if (sd.draws.tape_nw) {
        for (int k = tid; k < K; k += NWP_THREADS) chi2[k] = sd.draws.tape_nw[k];
        for (int q = tid; q < K; q += NWP_THREADS) zm[q] = sd.draws.tape_nw[K + K * (K - 1) / 2 + q];
    } else {
        const uint32_t h = half_sweep_index(sd.draws);
        for (int k = tid; k < K; k += NWP_THREADS)
            chi2[k] = 2.0 * gamma_mt(sd.draws.seed, h, (uint32_t)k, 0.5 * (nstar - (double)k));
        for (int q = tid; q < K; q += NWP_THREADS) zm[q] = stream_normal_f64(sd.draws.seed, h, 2u, (uint32_t)q);
    }
    for (int a = tid; a < K; a += NWP_THREADS) xbar[a] = sd.n > 0 ? sums[a] / dn : 0.0;
    __syncthreads();
    // A below the diagonal: Bartlett normal q = i (i - 1) / 2 + c for (i, c), c < i
    for (int e = tid; e < KT; e += NWP_THREADS) {
        int i = (int)((sqrt(8.0 * (double)e + 1.0) - 1.0) * 0.5);
        while (ptri(i, 0) > e) --i;
        while (ptri(i + 1, 0) <= e) ++i;
        const int c = e - ptri(i, 0);
        double v;
        if (c == i) {
            v = sqrt(chi2[c]);
        } else {
            const int q = i * (i - 1) / 2 + c;
            v = sd.draws.tape_nw ? sd.draws.tape_nw[K + q] : stream_normal_f64(sd.draws.seed, half_sweep_index(sd.draws), 1u, (uint32_t)q);
        }
        TL[e] = v;
        // P = W0^{-1} + S + coef (xbar - mu0)(xbar - mu0)^T, lower part
        const double coef = beta0 * dn / bstar;
        const double S = sums[K + e] - dn * xbar[i] * xbar[c];
        PL[e] = W0inv[i * K + c] + S + coef * (xbar[i] - mu0[i]) * (xbar[c] - mu0[c]);
    }
    // P = R R^T from the last pivot up
    for (int k = K - 1; k >= 0; --k) {
        __syncthreads();
        double akk = PL[ptri(k, k)];
        if (!(akk > 0.0) || !isfinite(akk)) {
            if (tid == 0) s_flag = 1;
            akk = 1.0;
        }
        const double rkk = sqrt(akk), inv = 1.0 / rkk;
        __syncthreads();
        if (tid == 0) {
            rd[k] = rkk;
            PL[ptri(k, k)] = rkk;
        }
        for (int i = tid; i < k; i += NWP_THREADS) PL[ptri(k, i)] *= inv;
        __syncthreads();
        // leading block: PL(ii, jj) -= R_ii,k R_jj,k for jj <= ii < k; 32
        // rows at a time, 16 threads along a row
        const double *rk = PL + ptri(k, 0);
        for (int ii = tid >> 4; ii < k; ii += NWP_THREADS / 16) {
            const double r = rk[ii];
            double *row = PL + ptri(ii, 0);
            for (int jj = tid & 15; jj <= ii; jj += 16) row[jj] = fma(-r, rk[jj], row[jj]);
        }
    }
    __syncthreads();
    // R^T T = A, right-looking: step m fixes row m of T and removes it from
    // the rows below (TL(i, c) -= R_mi T_mc for i > m, c <= m)
    for (int m = 0; m < K; ++m) {
        const double irm = 1.0 / rd[m];
        const double *tm = TL + ptri(m, 0);
        for (int i = m + 1 + (tid >> 4); i < K; i += NWP_THREADS / 16) {
            const double rmi = PL[ptri(i, m)] * irm;
            double *ti = TL + ptri(i, 0);
            for (int c = tid & 15; c <= m; c += 16) ti[c] = fma(-rmi, tm[c], ti[c]);
        }
        __syncthreads();
        for (int c = tid; c <= m; c += NWP_THREADS) TL[ptri(m, c)] *= irm;
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
    // mean: T^T d = z / sqrt(beta*), column-oriented backward substitution
    const double isb = 1.0 / sqrt(bstar);
    for (int a = tid; a < K; a += NWP_THREADS) dvec[a] = zm[a] * isb;
    for (int k = K - 1; k >= 0; --k) {
        __syncthreads();
        const double dk = dvec[k] / TL[ptri(k, k)];
        __syncthreads();
        if (tid == 0) dout[k] = dk;
        for (int i = tid; i < k; i += NWP_THREADS) dvec[i] = fma(-TL[ptri(k, i)], dk, dvec[i]);
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

__device__ __forceinline__ double readlane_d(double v, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

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
    for (int c0 = NWK - NPW; c0 >= 0; c0 -= NPW) {
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
    for (int i0 = 0; i0 < NWK; i0 += NPW) {
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
        if (i0 + NPW == NWK) break;
        __syncthreads();
        {
            double t[NPW];
#pragma unroll
            for (int q = 0; q < NPW; ++q) t[q] = Tm[(i0 + q) * NCS + lane];
#pragma unroll 2
            for (int i = i0 + NPW + wave; i < NWK; i += 4) {
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
        for (int k = NWK - 1; k >= 0; --k) {
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
                        const int q0 = lambda_acc_index(r, cc), q1 = lambda_acc_index(cc, r);
                        if (q0 >= 0) hyp.Lambda_acc[q0] = (float)x;
                        if (q1 >= 0) hyp.Lambda_acc[q1] = (float)x;
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
#pragma unroll
        for (int cc = 0; cc < 16; ++cc) lmu = fma(Pm[a * NCS + cb + cc], mul[cb + cc], lmu);
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

// Lambda_tri (and Lambda_acc) from Lambda_f (after a state restore, and
// after the Normal-Wishart step for K > 64).
__global__ __launch_bounds__(256) void lambda_tri_kernel(HyperDev hyp, int K, int KP)
{
    for (int t = threadIdx.x; t < KP * KP; t += blockDim.x) {
        const int r = t / KP, c = t - r * KP;
        const float v = (r < K && c < K) ? hyp.Lambda_f[r * K + c] : (r == c ? 1.0f : 0.0f);
        if (c <= r) hyp.Lambda_tri[r * (r + 1) / 2 + c] = v;
        if (hyp.Lambda_acc && KP <= 64) {
            const int q = lambda_acc_index(r, c);
            if (q >= 0) hyp.Lambda_acc[q] = v;
        }
    }
}

}  // namespace

hipError_t prepare_nw()
{
    hipError_t e = hipFuncSetAttribute((const void *)nw_compact_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
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
    if (K <= NWK) {
        // the statistics launch always provides the draws as a tape here
        if (!sides[0].draws.tape_nw || !sides[1].draws.tape_nw) return hipErrorInvalidValue;
        hipLaunchKernelGGL(nw_compact_kernel, dim3(2), dim3(256), nw_compact_lds_bytes(), s, sides[0], sides[1],
                           K, mu0, beta0, nu0, W0inv, state);
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
