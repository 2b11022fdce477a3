/*
 * bpmf_oracle.c -- plain FP64 CPU oracle for the BPMF Gibbs sampler.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU baseline leg of
 * the benchmark do.  It shares no code, header or constant table with the HIP
 * path.
 *
 * What it computes (paper: Section 2 "BPMF", Algorithm 1, and Section 3.1
 * "Single Core Optimizations"):
 *   - Algorithm 1 alternates, per sampling iteration, a hyper-parameter draw
 *     for one side from that side's factor matrix, then an update of every row
 *     of that side given the other side, plus noise; then the same for the
 *     other side; then a prediction of every test point.
 *   - The paper names the model (Gaussian rows with shared mean/precision per
 *     side, Normal-Wishart hyperpriors, Gaussian ratings) but prints no
 *     formula, so the conditionals here are the standard conjugate ones:
 *       row i:  P = Lambda + alpha * sum_{j in Omega_i} v_j v_j^T
 *               b = Lambda mu + alpha * sum_{j in Omega_i} (r_ij - rbar) v_j
 *               x_i ~ N(P^{-1} b, P^{-1})
 *       side:   (mu, Lambda) ~ NormalWishart(mu*, beta*, W*, nu*) given X
 *   - Section 3.1: the precision matrix is used only once, so the row draw
 *     factors it (Cholesky, lower, positive diagonal) instead of inverting:
 *       L L^T = P,  x_i = L^{-T} (L^{-1} b + z_i),  z_i ~ N(0, I).
 *
 * Every random number is an input (the "draw tape"); a counter-based
 * generator (Philox4x32-10, Salmon et al., SC'11) plus Box-Muller normals and
 * Marsaglia-Tsang gamma draws can fill such a tape from a seed.
 *
 * Conventions that are not fixed by the paper (each is a reading):
 *   - users' half first, then movies'; hypers of a side come from the current
 *     matrix of that side;
 *   - S is the centred scatter sum (two-pass), Wishart density
 *     |L|^{(nu-K-1)/2} exp(-tr(W^{-1} L)/2);
 *   - Bartlett factor uses L_W = chol(W*) with W* = P^{-1} formed explicitly
 *     and symmetrised; A_kk = sqrt(chi2(nu* - k)), k = 0..K-1;
 *   - tape per half-sweep over n rows: [K chi2][K(K-1)/2 Bartlett normals,
 *     row-major strict lower][K mean normals][n*K row normals, row-major].
 *
 * Plain loops, row-major matrices, no BLAS.  Rows of a half-sweep are
 * independent, so the half-sweep can split them over threads in fixed chunks
 * without changing any result.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_NOT_SPD 1
#define OR_INVALID 2
#define OR_NOMEM 3

/* ------------------------------------------------------------------------ */
/* Dense helpers (row-major, n x n)                                          */
/* ------------------------------------------------------------------------ */

/* Cholesky-Banachiewicz: A = L L^T, L lower with positive diagonal. Only the
 * lower triangle of A is read; the upper triangle of L is set to zero. */
int oracle_cholesky(int n, const double *A, double *L)
{
    for (int i = 0; i < n * n; ++i) L[i] = 0.0;
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j <= i; ++j) {
            double s = A[i * n + j];
            for (int k = 0; k < j; ++k) s -= L[i * n + k] * L[j * n + k];
            if (i == j) {
                if (!(s > 0.0) || !isfinite(s)) return OR_NOT_SPD;
                L[i * n + i] = sqrt(s);
            } else {
                L[i * n + j] = s / L[j * n + j];
            }
        }
    }
    return OR_OK;
}

/* y = L^{-1} b */
static void forward_solve(int n, const double *L, const double *b, double *y)
{
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= L[i * n + k] * y[k];
        y[i] = s / L[i * n + i];
    }
}

/* x = L^{-T} y */
static void backward_solve(int n, const double *L, const double *y, double *x)
{
    for (int i = n - 1; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * x[k];
        x[i] = s / L[i * n + i];
    }
}

/* Ainv = A^{-1} for SPD A, by solving A x = e_c column by column. */
int oracle_spd_inverse(int n, const double *A, double *Ainv)
{
    double *L = malloc(sizeof(double) * n * n);
    double *e = malloc(sizeof(double) * n);
    double *y = malloc(sizeof(double) * n);
    double *x = malloc(sizeof(double) * n);
    int rc = (L && e && y && x) ? oracle_cholesky(n, A, L) : OR_NOMEM;
    if (rc == OR_OK) {
        for (int c = 0; c < n; ++c) {
            for (int i = 0; i < n; ++i) e[i] = (i == c) ? 1.0 : 0.0;
            forward_solve(n, L, e, y);
            backward_solve(n, L, y, x);
            for (int i = 0; i < n; ++i) Ainv[i * n + c] = x[i];
        }
    }
    free(L); free(e); free(y); free(x);
    return rc;
}

static void symmetrize(int n, double *A)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) {
            double m = 0.5 * (A[i * n + j] + A[j * n + i]);
            A[i * n + j] = m;
            A[j * n + i] = m;
        }
}

/* ------------------------------------------------------------------------ */
/* Row conditional (Section 2 / Section 3.1)                                 */
/* ------------------------------------------------------------------------ */

/* One row: gather the rated items' factor rows, build P and b, factor P,
 * solve for the mean and draw.  `other` is the other side's factor matrix
 * (n_other x K).  `Lmu` = Lambda * mu.  Writes the draw to `out` and, if
 * `mean_out` is not NULL, the conditional mean P^{-1} b. */
int oracle_row_update(int K, int64_t nnz, const int32_t *idx, const double *val,
                      const double *other, double alpha, double rbar,
                      const double *Lambda, const double *Lmu, const double *z,
                      double *out, double *mean_out)
{
    double *P = malloc(sizeof(double) * K * K);
    double *L = malloc(sizeof(double) * K * K);
    double *b = malloc(sizeof(double) * K);
    double *y = malloc(sizeof(double) * K);
    int rc = OR_OK;
    if (!P || !L || !b || !y) { rc = OR_NOMEM; goto done; }
    for (int a = 0; a < K * K; ++a) P[a] = Lambda[a];
    for (int a = 0; a < K; ++a) b[a] = Lmu[a];
    for (int64_t t = 0; t < nnz; ++t) {
        const double *v = other + (int64_t)idx[t] * K;
        double r = val[t] - rbar;
        for (int a = 0; a < K; ++a) {
            b[a] += alpha * r * v[a];
            for (int c = 0; c < K; ++c) P[a * K + c] += alpha * v[a] * v[c];
        }
    }
    rc = oracle_cholesky(K, P, L);
    if (rc != OR_OK) goto done;
    forward_solve(K, L, b, y);
    if (mean_out) backward_solve(K, L, y, mean_out);
    for (int a = 0; a < K; ++a) y[a] += z[a];
    backward_solve(K, L, y, out);
done:
    free(P); free(L); free(b); free(y);
    return rc;
}

typedef struct {
    int64_t lo, hi;
    int K;
    const int64_t *ptr;
    const int32_t *idx;
    const double *val;
    const double *other;
    double alpha, rbar;
    const double *Lambda, *Lmu, *Z;
    double *X;
    int rc;
} half_job;

static void *half_worker(void *arg)
{
    half_job *j = (half_job *)arg;
    j->rc = OR_OK;
    for (int64_t i = j->lo; i < j->hi; ++i) {
        int64_t s = j->ptr[i], e = j->ptr[i + 1];
        int rc = oracle_row_update(j->K, e - s, j->idx + s, j->val + s, j->other, j->alpha,
                                   j->rbar, j->Lambda, j->Lmu, j->Z + i * j->K,
                                   j->X + i * j->K, NULL);
        if (rc != OR_OK && j->rc == OR_OK) j->rc = rc;
    }
    return NULL;
}

/* Update every row of one side (Algorithm 1, inner loops). Rows are split
 * over `nthreads` threads in fixed contiguous chunks; results do not depend
 * on the thread count. */
int oracle_half_sweep(int64_t n_rows, int K, const int64_t *ptr, const int32_t *idx,
                      const double *val, const double *other, double alpha, double rbar,
                      const double *Lambda, const double *mu, const double *Z, double *X,
                      int nthreads)
{
    double *Lmu = malloc(sizeof(double) * K);
    if (!Lmu) return OR_NOMEM;
    for (int a = 0; a < K; ++a) {
        double s = 0.0;
        for (int c = 0; c < K; ++c) s += Lambda[a * K + c] * mu[c];
        Lmu[a] = s;
    }
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    half_job jobs[256];
    pthread_t th[256];
    int64_t chunk = (n_rows + nthreads - 1) / nthreads;
    int rc = OR_OK;
    for (int t = 0; t < nthreads; ++t) {
        half_job *j = &jobs[t];
        j->lo = t * chunk < n_rows ? t * chunk : n_rows;
        j->hi = (t + 1) * chunk < n_rows ? (t + 1) * chunk : n_rows;
        j->K = K; j->ptr = ptr; j->idx = idx; j->val = val; j->other = other;
        j->alpha = alpha; j->rbar = rbar; j->Lambda = Lambda; j->Lmu = Lmu; j->Z = Z; j->X = X;
        if (nthreads == 1) half_worker(j);
        else pthread_create(&th[t], NULL, half_worker, j);
    }
    for (int t = 0; t < nthreads; ++t) {
        if (nthreads > 1) pthread_join(th[t], NULL);
        if (jobs[t].rc != OR_OK && rc == OR_OK) rc = jobs[t].rc;
    }
    free(Lmu);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Hyper-parameters of one side (Algorithm 1, "sample hyper-parameters")      */
/* ------------------------------------------------------------------------ */

/* Normal-Wishart posterior given the n rows of X (n x K):
 *   xbar = (1/n) sum X_i,  S = sum (X_i - xbar)(X_i - xbar)^T  (two passes)
 *   beta* = beta0 + n,  nu* = nu0 + n,  mu* = (beta0 mu0 + n xbar) / beta*
 *   W*^{-1} = W0^{-1} + S + (beta0 n / beta*) (xbar - mu0)(xbar - mu0)^T */
int oracle_nw_posterior(int K, int64_t n, const double *X, const double *mu0, double beta0,
                        double nu0, const double *W0, double *mu_star, double *beta_star,
                        double *nu_star, double *W_star)
{
    double *xbar = calloc(K, sizeof(double));
    double *S = calloc((size_t)K * K, sizeof(double));
    double *W0inv = malloc(sizeof(double) * K * K);
    double *Pm = malloc(sizeof(double) * K * K);
    int rc = OR_OK;
    if (!xbar || !S || !W0inv || !Pm) { rc = OR_NOMEM; goto done; }
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < K; ++a) xbar[a] += X[i * K + a];
    if (n > 0)
        for (int a = 0; a < K; ++a) xbar[a] /= (double)n;
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < K; ++a)
            for (int c = 0; c < K; ++c)
                S[a * K + c] += (X[i * K + a] - xbar[a]) * (X[i * K + c] - xbar[c]);
    double bs = beta0 + (double)n;
    *beta_star = bs;
    *nu_star = nu0 + (double)n;
    for (int a = 0; a < K; ++a) mu_star[a] = (beta0 * mu0[a] + (double)n * xbar[a]) / bs;
    rc = oracle_spd_inverse(K, W0, W0inv);
    if (rc != OR_OK) goto done;
    double coef = beta0 * (double)n / bs;
    for (int a = 0; a < K; ++a)
        for (int c = 0; c < K; ++c)
            Pm[a * K + c] = W0inv[a * K + c] + S[a * K + c] +
                            coef * (xbar[a] - mu0[a]) * (xbar[c] - mu0[c]);
    symmetrize(K, Pm);
    rc = oracle_spd_inverse(K, Pm, W_star);
    if (rc != OR_OK) goto done;
    symmetrize(K, W_star);
done:
    free(xbar); free(S); free(W0inv); free(Pm);
    return rc;
}

/* Draw (mu, Lambda) from the posterior with the given draws:
 *   Bartlett: A lower, A_kk = sqrt(chi2[k]), A_kl = zb[k(k-1)/2 + l] (k > l),
 *   Lambda = L_W A A^T L_W^T with L_W = chol(W*);
 *   mu = mu* + chol(beta* Lambda)^{-T} zm. */
int oracle_nw(int K, int64_t n, const double *X, const double *mu0, double beta0, double nu0,
              const double *W0, const double *chi2, const double *zb, const double *zm,
              double *Lambda, double *mu)
{
    double *mus = malloc(sizeof(double) * K);
    double *Ws = malloc(sizeof(double) * K * K);
    double *LW = malloc(sizeof(double) * K * K);
    double *A = calloc((size_t)K * K, sizeof(double));
    double *T = calloc((size_t)K * K, sizeof(double));
    double *BL = malloc(sizeof(double) * K * K);
    double *Lc = malloc(sizeof(double) * K * K);
    double *d = malloc(sizeof(double) * K);
    double bs, ns;
    int rc = OR_OK;
    if (!mus || !Ws || !LW || !A || !T || !BL || !Lc || !d) { rc = OR_NOMEM; goto done; }
    rc = oracle_nw_posterior(K, n, X, mu0, beta0, nu0, W0, mus, &bs, &ns, Ws);
    if (rc != OR_OK) goto done;
    rc = oracle_cholesky(K, Ws, LW);
    if (rc != OR_OK) goto done;
    for (int k = 0; k < K; ++k) {
        A[k * K + k] = sqrt(chi2[k]);
        for (int l = 0; l < k; ++l) A[k * K + l] = zb[k * (k - 1) / 2 + l];
    }
    /* T = L_W A */
    for (int a = 0; a < K; ++a)
        for (int c = 0; c < K; ++c) {
            double s = 0.0;
            for (int m = 0; m < K; ++m) s += LW[a * K + m] * A[m * K + c];
            T[a * K + c] = s;
        }
    /* Lambda = T T^T */
    for (int a = 0; a < K; ++a)
        for (int c = 0; c < K; ++c) {
            double s = 0.0;
            for (int m = 0; m < K; ++m) s += T[a * K + m] * T[c * K + m];
            Lambda[a * K + c] = s;
        }
    symmetrize(K, Lambda);
    for (int a = 0; a < K * K; ++a) BL[a] = bs * Lambda[a];
    rc = oracle_cholesky(K, BL, Lc);
    if (rc != OR_OK) goto done;
    backward_solve(K, Lc, zm, d);
    for (int a = 0; a < K; ++a) mu[a] = mus[a] + d[a];
done:
    free(mus); free(Ws); free(LW); free(A); free(T); free(BL); free(Lc); free(d);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Whole sampler (Algorithm 1)                                               */
/* ------------------------------------------------------------------------ */

int64_t oracle_tape_block_len(int64_t n_rows, int K)
{
    return (int64_t)K + (int64_t)K * (K - 1) / 2 + K + n_rows * K;
}

/* Runs `n_sweeps` sweeps from the state in U (M x K) and V (N x K), which are
 * overwritten.  Per sweep s: hypers of U from U, all users, hypers of V from
 * V, all movies, then for s >= burnin every test point's prediction
 * u_i . v_j + rbar is added to pred_sum (and pred_cnt incremented).
 * `sweep0` is the index of the first sweep (for burn-in across calls).
 * hyper_out (optional): the last sweep's [Lambda_U, mu_U, Lambda_V, mu_V]. */
int oracle_gibbs(int64_t M, int64_t N, int K,
                 const int64_t *row_ptr, const int32_t *col_idx, const double *row_val,
                 const int64_t *col_ptr, const int32_t *row_idx, const double *col_val,
                 double alpha, double rbar, const double *mu0, double beta0, double nu0,
                 const double *W0, const double *tape, int n_sweeps, int sweep0, int burnin,
                 double *U, double *V, int64_t n_test, const int32_t *trow,
                 const int32_t *tcol, double *pred_sum, int64_t *pred_cnt,
                 double *hyper_out, int nthreads)
{
    double *LamU = malloc(sizeof(double) * K * K), *muU = malloc(sizeof(double) * K);
    double *LamV = malloc(sizeof(double) * K * K), *muV = malloc(sizeof(double) * K);
    int rc = OR_OK;
    if (!LamU || !muU || !LamV || !muV) { rc = OR_NOMEM; goto done; }
    const int64_t hu = (int64_t)K + (int64_t)K * (K - 1) / 2 + K;
    const double *t = tape;
    for (int s = 0; s < n_sweeps; ++s) {
        /* users */
        rc = oracle_nw(K, M, U, mu0, beta0, nu0, W0, t, t + K, t + K + K * (K - 1) / 2,
                       LamU, muU);
        if (rc != OR_OK) goto done;
        rc = oracle_half_sweep(M, K, row_ptr, col_idx, row_val, V, alpha, rbar, LamU, muU,
                               t + hu, U, nthreads);
        if (rc != OR_OK) goto done;
        t += hu + M * K;
        /* movies */
        rc = oracle_nw(K, N, V, mu0, beta0, nu0, W0, t, t + K, t + K + K * (K - 1) / 2,
                       LamV, muV);
        if (rc != OR_OK) goto done;
        rc = oracle_half_sweep(N, K, col_ptr, row_idx, col_val, U, alpha, rbar, LamV, muV,
                               t + hu, V, nthreads);
        if (rc != OR_OK) goto done;
        t += hu + N * K;
        /* predictions */
        if (sweep0 + s >= burnin && n_test > 0) {
            for (int64_t q = 0; q < n_test; ++q) {
                double p = rbar;
                for (int a = 0; a < K; ++a)
                    p += U[(int64_t)trow[q] * K + a] * V[(int64_t)tcol[q] * K + a];
                pred_sum[q] += p;
            }
            *pred_cnt += 1;
        }
    }
    if (hyper_out) {
        memcpy(hyper_out, LamU, sizeof(double) * K * K);
        memcpy(hyper_out + K * K, muU, sizeof(double) * K);
        memcpy(hyper_out + K * K + K, LamV, sizeof(double) * K * K);
        memcpy(hyper_out + 2 * K * K + K, muV, sizeof(double) * K);
    }
done:
    free(LamU); free(muU); free(LamV); free(muV);
    return rc;
}

/* Predictions u_i . v_j + rbar for arbitrary pairs. */
void oracle_predict(int K, int64_t n, const int32_t *rows, const int32_t *cols,
                    const double *U, const double *V, double rbar, double *out)
{
    for (int64_t q = 0; q < n; ++q) {
        double p = rbar;
        for (int a = 0; a < K; ++a) p += U[(int64_t)rows[q] * K + a] * V[(int64_t)cols[q] * K + a];
        out[q] = p;
    }
}

/* ------------------------------------------------------------------------ */
/* Fold-in of new users against stored posterior samples                     */
/* ------------------------------------------------------------------------ */

/* For request r and sample s: the new user's conditional mean
 *   m_s = (Lambda_s + alpha sum_j v_j v_j^T)^{-1} (Lambda_s mu_s + alpha sum_j (r_j - rbar) v_j)
 * with v_j rows of Vs[s]; then pred_q = rbar + (1/S) sum_s m_s . Vs[s][q].
 * mean_out (optional): n_req x S x K conditional means. */
int oracle_foldin(int S, int64_t N, int K, double alpha, double rbar, const double *Vs,
                  const double *Lam, const double *mu, int64_t n_req, const int64_t *req_ptr,
                  const int32_t *cols, const double *vals, const int64_t *q_ptr,
                  const int32_t *q_cols, double *out, double *mean_out)
{
    double *Lmu = malloc(sizeof(double) * K);
    double *m = malloc(sizeof(double) * K);
    double *zero = calloc(K, sizeof(double));
    double *draw = malloc(sizeof(double) * K);
    int rc = OR_OK;
    if (!Lmu || !m || !zero || !draw) { rc = OR_NOMEM; goto done; }
    for (int64_t r = 0; r < n_req; ++r) {
        for (int64_t q = q_ptr[r]; q < q_ptr[r + 1]; ++q) out[q] = 0.0;
        for (int s = 0; s < S; ++s) {
            const double *Ls = Lam + (int64_t)s * K * K;
            const double *Vsm = Vs + (int64_t)s * N * K;
            for (int a = 0; a < K; ++a) {
                double acc = 0.0;
                for (int c = 0; c < K; ++c) acc += Ls[a * K + c] * mu[(int64_t)s * K + c];
                Lmu[a] = acc;
            }
            rc = oracle_row_update(K, req_ptr[r + 1] - req_ptr[r], cols + req_ptr[r],
                                   vals + req_ptr[r], Vsm, alpha, rbar, Ls, Lmu, zero, draw, m);
            if (rc != OR_OK) goto done;
            if (mean_out) memcpy(mean_out + (r * S + s) * K, m, sizeof(double) * K);
            for (int64_t q = q_ptr[r]; q < q_ptr[r + 1]; ++q) {
                double p = 0.0;
                for (int a = 0; a < K; ++a) p += m[a] * Vsm[(int64_t)q_cols[q] * K + a];
                out[q] += p;
            }
        }
        for (int64_t q = q_ptr[r]; q < q_ptr[r + 1]; ++q) out[q] = rbar + out[q] / (double)S;
    }
done:
    free(Lmu); free(m); free(zero); free(draw);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Counter-based draws (Philox4x32-10, Box-Muller, Marsaglia-Tsang)          */
/* ------------------------------------------------------------------------ */

/* Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11): each round
 * multiplies words 0 and 2 by two fixed odd constants, swaps the high and low
 * halves into new positions with the key mixed in by xor; the key advances
 * by two Weyl constants between rounds. */
void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 53-bit uniform in (0,1) from two words: a gives the high 32 bits, the top
 * 21 bits of b the rest; offset by half a unit so 0 and 1 never occur. */
static double u53(uint32_t a, uint32_t b)
{
    uint64_t m = ((uint64_t)a << 21) | (uint64_t)(b >> 11);
    return ((double)m + 0.5) * 0x1.0p-53;
}

static void philox_words(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                         uint32_t w[4])
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    oracle_philox4x32_10(ctr, key, w);
}

/* Box-Muller pair from one Philox block: u1 from words (0,1), u2 from (2,3). */
static void bm_pair(const uint32_t w[4], double *z0, double *z1)
{
    double u1 = u53(w[0], w[1]);
    double u2 = u53(w[2], w[3]);
    double rad = sqrt(-2.0 * log(u1));
    double th = 6.283185307179586476925286766559 * u2;
    *z0 = rad * cos(th);
    *z1 = rad * sin(th);
}

/* Row normals of half-sweep h: normal k of row r is half (k % 2) of the
 * Box-Muller pair from counter (k/2, r, h, 0). */
void oracle_philox_row_normals(uint64_t seed, uint32_t h, int64_t n_rows, int K, double *out)
{
    for (int64_t r = 0; r < n_rows; ++r)
        for (int p = 0; 2 * p < K; ++p) {
            uint32_t w[4];
            double z0, z1;
            philox_words(seed, (uint32_t)p, (uint32_t)r, h, 0u, w);
            bm_pair(w, &z0, &z1);
            out[r * K + 2 * p] = z0;
            if (2 * p + 1 < K) out[r * K + 2 * p + 1] = z1;
        }
}

/* Standard normal number q of stream `tag` of half-sweep h. */
static double stream_normal(uint64_t seed, uint32_t h, uint32_t tag, uint32_t q)
{
    uint32_t w[4];
    double z0, z1;
    philox_words(seed, q / 2u, 0u, h, tag, w);
    bm_pair(w, &z0, &z1);
    return (q & 1u) ? z1 : z0;
}

/* Gamma(shape a, scale 1) by Marsaglia and Tsang (ACM TOMS 26(3), 2000):
 * d = a - 1/3, c = 1/sqrt(9d); propose v = (1 + c x)^3 with x normal and
 * accept when log u < x^2/2 + d - d v + d log v.  For a < 1, draw with
 * shape a + 1 and scale by u^{1/a}.  Attempt t of draw k of half-sweep h
 * takes its normal from counter (t, k, h, 3) and its uniform from
 * (t, k, h, 4); the shape boost uniform comes from (0, k, h, 5). */
static double mt_gamma(uint64_t seed, uint32_t h, uint32_t k, double a)
{
    double boost = 1.0;
    if (a < 1.0) {
        uint32_t w[4];
        philox_words(seed, 0u, k, h, 5u, w);
        boost = pow(u53(w[0], w[1]), 1.0 / a);
        a += 1.0;
    }
    double d = a - 1.0 / 3.0;
    double c = 1.0 / sqrt(9.0 * d);
    for (uint32_t t = 0;; ++t) {
        uint32_t w[4];
        double x, unused;
        philox_words(seed, t, k, h, 3u, w);
        bm_pair(w, &x, &unused);
        double v = 1.0 + c * x;
        if (v <= 0.0) continue;
        v = v * v * v;
        philox_words(seed, t, k, h, 4u, w);
        double u = u53(w[0], w[1]);
        if (log(u) < 0.5 * x * x + d - d * v + d * log(v)) return boost * d * v;
    }
}

/* Fills one half-sweep's tape block (layout as in the header comment) from
 * the counter-based streams: chi2[k] = 2 Gamma((nu0 + n - k)/2) with draw
 * index k; Bartlett normals from stream 1, mean normals from stream 2, row
 * normals from stream 0. */
void oracle_philox_block(uint64_t seed, uint32_t h, int64_t n_rows, int K, double nu0,
                         double *out)
{
    double nus = nu0 + (double)n_rows;
    for (int k = 0; k < K; ++k) out[k] = 2.0 * mt_gamma(seed, h, (uint32_t)k, 0.5 * (nus - k));
    int nb = K * (K - 1) / 2;
    for (int q = 0; q < nb; ++q) out[K + q] = stream_normal(seed, h, 1u, (uint32_t)q);
    for (int q = 0; q < K; ++q) out[K + nb + q] = stream_normal(seed, h, 2u, (uint32_t)q);
    oracle_philox_row_normals(seed, h, n_rows, K, out + K + nb + K);
}

/* Whole tape for sweeps sweep0 .. sweep0 + n_sweeps - 1 (half-sweep index
 * h = 2 s for users, 2 s + 1 for movies). */
void oracle_philox_tape(uint64_t seed, int sweep0, int n_sweeps, int64_t M, int64_t N, int K,
                        double nu0, double *out)
{
    for (int s = sweep0; s < sweep0 + n_sweeps; ++s) {
        oracle_philox_block(seed, (uint32_t)(2 * s), M, K, nu0, out);
        out += oracle_tape_block_len(M, K);
        oracle_philox_block(seed, (uint32_t)(2 * s + 1), N, K, nu0, out);
        out += oracle_tape_block_len(N, K);
    }
}

/* Bulk Gamma draws for statistical tests of the sampler above. */
void oracle_gamma_draws(uint64_t seed, uint32_t h, double a, int64_t n, double *out)
{
    for (int64_t k = 0; k < n; ++k) out[k] = mt_gamma(seed, h, (uint32_t)k, a);
}

/* Bulk normals of stream `tag` for statistical tests. */
void oracle_stream_normals(uint64_t seed, uint32_t h, uint32_t tag, int64_t n, double *out)
{
    for (int64_t q = 0; q < n; ++q) out[q] = stream_normal(seed, h, tag, (uint32_t)q);
}
