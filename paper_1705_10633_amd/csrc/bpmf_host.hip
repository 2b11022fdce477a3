// bpmf_host.hip -- implementation of the C ABI declared in include/bpmf.h.
//
// Host-side plan of a sampler: validates the problem, carves the caller's
// workspace, orders rows by rating count, and enqueues per sweep (paper:
// Algorithm 1, users' half first):
//   stats(U) -> hyper(U) -> rows(U | V) [-> FP64 recompute of flagged rows]
//   stats(V) -> hyper(V) -> rows(V | U) [-> ...] -> predictions -> counter
// With a device generator the whole sweep can be captured once as a HIP
// graph and replayed; the kernels read the sweep counter from device memory.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/bpmf.h"
#include "common.hpp"
#include "plan.hpp"

namespace bpmf {
size_t rows_f64_lds_bytes(int K);
hipError_t launch_advance_burnin(DevState *state, int burnin, hipStream_t s);
hipError_t launch_foldin(int S, int K, int64_t N, double alpha, double rbar, const float *Vs,
                         const double *Lam, const double *mu, int64_t n_req, const int64_t *req_ptr,
                         const int32_t *cols, const float *vals, const int64_t *q_ptr,
                         const int32_t *q_cols, int64_t n_queries, float *partial, float *out,
                         hipStream_t st);
int64_t foldin_noalloc_max_partials();
hipError_t foldin_noalloc_scratch(float **out);
hipError_t launch_sum_values(const void *vals, int is_f64, int64_t n, double *partials, int nblk,
                             hipStream_t s);
hipError_t launch_mean_from_sum(const double *accum, const int64_t *perm, int64_t n,
                                const DevState *state, double *out, hipStream_t s);
hipError_t prepare_rows_f64(int K);
}  // namespace bpmf

using namespace bpmf;

static thread_local std::string g_last_error;

void bpmf::set_last_error(const std::string &msg) { g_last_error = msg; }

static bpmf_status fail(bpmf_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

#define HIP_OK(expr)                                                                       \
    do {                                                                                   \
        hipError_t _e = (expr);                                                            \
        if (_e != hipSuccess)                                                              \
            return fail(BPMF_E_HIP, std::string(#expr) + ": " + hipGetErrorString(_e));    \
    } while (0)

static const size_t kAlign = 256;

struct WsLayout {
    size_t total = 0;
    size_t add(size_t bytes)
    {
        size_t off = (total + kAlign - 1) / kAlign * kAlign;
        total = off + bytes;
        return off;
    }
};

struct Offsets {
    size_t state, partials[2], sums[2], lam[2], mu[2], lmu[2], lamf[2], lmuf[2], lamt[2], lamacc[2], lchol[2], nwd[2], mu0, w0inv,
        order[2], rowtab[2], recoff[2], rec[2], ctab[2], part[2], fblist[2], shadow[2], valsf[2], accum, trows, tcols, tperm, reduce;
    size_t total;
};

static int padded_k(int K) { return K <= 32 ? 32 : (K <= 64 ? 64 : 128); }

// Pieces of heavy rows per side (workspace reserved up front): rows with at
// least heavy_min_ratings() ratings are cut into pieces of at least 512.
static constexpr int64_t kMaxPieces = 2048;

// Mixed-precision row kernels: one wavefront per row for K <= 64 (FP32 or
// BF16 gathers); a four-wavefront workgroup per row for 64 < K <= 128 (BF16
// gathers only).  Other cases use FP64 row arithmetic on FP32 storage.
static bool mixed_supported(int K, int precision)
{
    return K <= 64 || (precision == BPMF_BF16 && K <= 128);
}

// Rows with at most this many ratings take the rank-one kernel (K <= 64): m
// updates cost about m K steps of a few instructions per lane, against a
// Cholesky of K steps with up to K instructions each plus the Gram pipeline.
static int64_t rank1_limit(int K)
{
    const int64_t lim = K <= 32 ? 3 : 2;
    return std::min<int64_t>(lim, rank1_max_ratings());
}

// The launch shape with the built-in choices filled in for the fields left at 0.
struct LaunchShape {
    int64_t heavy_min, piece_min, rank1_max;
    int heavy_split, rank1_split;
    int variant;  // kernel variant of the K <= 64 row kernel (1..3)
};

static LaunchShape resolve_shape(const bpmf_launch_shape *sh, int K)
{
    LaunchShape r{heavy_min_ratings(), 512, rank1_limit(K), 0, 0, 1};
    if (!sh) return r;
    if (sh->heavy_min_ratings) r.heavy_min = sh->heavy_min_ratings;
    if (sh->piece_min_ratings) r.piece_min = sh->piece_min_ratings;
    // -1: no row qualifies, not even rows without ratings
    if (sh->rank1_max_ratings) r.rank1_max = sh->rank1_max_ratings < 0 ? -1 : sh->rank1_max_ratings;
    r.heavy_split = sh->heavy_split;
    r.rank1_split = sh->rank1_split;
    if (sh->kernel_variant) r.variant = sh->kernel_variant;
    return r;
}

static Offsets layout(const bpmf_ratings *R, const bpmf_params *p, int64_t n_test)
{
    Offsets o;
    WsLayout w;
    const int K = p->K;
    const int64_t n[2] = {R->M, R->N};
    const bool mixed = p->precision != BPMF_FP64;
    const bool mk = mixed && mixed_supported(K, p->precision);
    o.state = w.add(sizeof(DevState));
    const int slots = stats_slots(K, p->precision == BPMF_FP64 ? 1 : 0);
    for (int s = 0; s < 2; ++s) {
        const int nc = stats_chunks(n[s], n[1 - s], K, slots);
        o.partials[s] = w.add(sizeof(double) * (size_t)nc * (K + K * (K + 1) / 2));
        o.sums[s] = w.add(sizeof(double) * (size_t)(K + K * (K + 1) / 2));
        o.lam[s] = w.add(sizeof(double) * K * K);
        o.mu[s] = w.add(sizeof(double) * K);
        o.lmu[s] = w.add(sizeof(double) * K);
        o.lamf[s] = w.add(sizeof(float) * K * K);
        o.lmuf[s] = w.add(sizeof(float) * K);
        o.lamt[s] = w.add(sizeof(float) * (size_t)padded_k(K) * (padded_k(K) + 3) / 2);
        o.lamacc[s] = w.add((mk && K <= 64) ? sizeof(float) * 3 * 16 * 64 : 0);
        o.lchol[s] = w.add((mk && K <= 64) ? sizeof(float) * (size_t)padded_k(K) * (padded_k(K) + 4) : 0);
        o.nwd[s] = w.add(sizeof(double) * (size_t)(2 * K + K * (K - 1) / 2));
        o.order[s] = w.add(sizeof(int32_t) * n[s]);
        // launch table: the rows, or (with heavy rows) their pieces and then the other rows
        const bool pieces = mk && K <= 64;
        const int64_t n_entries = n[s] + (pieces ? kMaxPieces : 0);
        o.rowtab[s] = w.add(sizeof(int4) * n_entries);
        // BF16 packed rating records: each entry padded to whole chunks, so at
        // most nnz + n_entries (chunk - 1) ratings, 8 bytes each
        const bool recs = mk && p->precision == BPMF_BF16;
        const int64_t chunk = bf16_chunk(padded_k(K));
        o.recoff[s] = w.add(recs ? sizeof(int64_t) * n_entries : 0);
        o.rec[s] = w.add(recs ? 8 * (size_t)(R->nnz + n_entries * (chunk - 1) + 4) : 0);
        o.ctab[s] = w.add(pieces ? sizeof(int4) * kMaxPieces / 2 : 0);
        o.part[s] = w.add(pieces ? sizeof(float) * (size_t)kMaxPieces * piece_floats(padded_k(K)) : 0);
        o.fblist[s] = w.add(mk ? sizeof(int32_t) * n[s] : 0);
        // BF16 copy plus one all-zero row (the gather target past a row's end)
        o.shadow[s] = w.add((mk && p->precision == BPMF_BF16) ? sizeof(uint16_t) * (n[s] + 1) * padded_k(K) : 0);
        o.valsf[s] = w.add((mixed && R->val_is_f64) ? sizeof(float) * R->nnz : 0);
    }
    o.mu0 = w.add(sizeof(double) * K);
    o.w0inv = w.add(sizeof(double) * K * K);
    o.accum = w.add(sizeof(double) * std::max<int64_t>(n_test, 0));
    o.trows = w.add(sizeof(int32_t) * std::max<int64_t>(n_test, 0));
    o.tcols = w.add(sizeof(int32_t) * std::max<int64_t>(n_test, 0));
    o.tperm = w.add(sizeof(int64_t) * std::max<int64_t>(n_test, 0));
    o.reduce = w.add(sizeof(double) * 1024);
    o.total = w.total + kAlign;
    return o;
}

struct bpmf_ctx {
    bpmf_ratings R;
    int K, KP, precision, burnin, use_graph;
    double alpha, beta0, nu0, rbar;
    uint64_t seed;
    void *dU, *dV;
    char *ws;
    Offsets off;
    DevState *state;
    HyperDev hyp[2];
    int n_chunks[2];
    // tails of the row order: rows for the rank-one kernels (n_small), of
    // which the last n_tiny (at most one rating, K <= 32) take the one-lane kernel
    int64_t n_small[2] = {0, 0}, n_tiny[2] = {0, 0};
    // head of the row order: heavy rows cut into pieces (K <= 64); the launch
    // table holds n_pieces pieces and then the rows from slot n_heavy on
    int64_t n_heavy[2] = {0, 0}, n_pieces[2] = {0, 0};
    // entries of the launch table per side (pieces and rows)
    int64_t n_entries[2] = {0, 0};
    bool records = false;  // BF16 mode: the row kernels read packed rating records
    int variant = 1;       // kernel variant of the K <= 64 row kernel
    int64_t n_test;
    const int32_t *test_rows, *test_cols;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipStream_t cap_stream = nullptr;
    bool broken = false;
    // per-kernel timing
    bool timing = false;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
    std::vector<hipEvent_t> pool;
    double t_ms[BPMF_TIMING_CLASSES] = {0};
    int64_t t_n[BPMF_TIMING_CLASSES] = {0};
    bool x_f64() const { return precision == BPMF_FP64; }
    template <class T> T *at(size_t o) const { return (T *)(ws + o); }
};

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------
static bpmf_status check_params(const bpmf_ratings *R, const bpmf_params *p)
{
    if (!R || !p) return fail(BPMF_E_INVALID, "NULL ratings or params");
    if (p->K < 1 || p->K > 128) return fail(BPMF_E_INVALID, "K must be in 1..128");
    if (p->precision < BPMF_FP64 || p->precision > BPMF_BF16)
        return fail(BPMF_E_INVALID, "unknown precision");
    if (!(p->alpha > 0.0) || !std::isfinite(p->alpha)) return fail(BPMF_E_INVALID, "alpha must be > 0");
    if (!(p->beta0 > 0.0) || !std::isfinite(p->beta0)) return fail(BPMF_E_INVALID, "beta0 must be > 0");
    if (!(p->nu0 > p->K - 1) || !std::isfinite(p->nu0)) return fail(BPMF_E_INVALID, "nu0 must be > K - 1");
    if (!p->mu0 || !p->W0) return fail(BPMF_E_INVALID, "mu0 and W0 are required");
    if (p->burnin < 0) return fail(BPMF_E_INVALID, "burnin must be >= 0");
    if (const bpmf_launch_shape *sh = p->shape) {
        if (sh->heavy_min_ratings != 0 && sh->heavy_min_ratings < 64)
            return fail(BPMF_E_INVALID, "shape.heavy_min_ratings must be 0 or >= 64");
        if (sh->piece_min_ratings != 0 && sh->piece_min_ratings < 64)
            return fail(BPMF_E_INVALID, "shape.piece_min_ratings must be 0 or >= 64");
        if (sh->heavy_split < -1 || sh->heavy_split > 1 || sh->rank1_split < -1 || sh->rank1_split > 1)
            return fail(BPMF_E_INVALID, "shape.heavy_split and shape.rank1_split must be -1, 0 or 1");
        if (sh->kernel_variant < 0 || sh->kernel_variant > 3)
            return fail(BPMF_E_INVALID, "shape.kernel_variant must be 0..3");
        if (sh->rank1_max_ratings < -1 || sh->rank1_max_ratings > rank1_max_ratings())
            return fail(BPMF_E_INVALID, "shape.rank1_max_ratings must be -1, 0 or 1.." +
                                            std::to_string(rank1_max_ratings()));
    }
    if (R->M < 1 || R->N < 1 || R->nnz < 0) return fail(BPMF_E_INVALID, "M, N must be >= 1, nnz >= 0");
    if (R->M > INT32_MAX || R->N > INT32_MAX) return fail(BPMF_E_INVALID, "M and N must fit in int32");
    // the BF16 gathers address rows with 32-bit byte offsets
    if (p->precision == BPMF_BF16 && (R->M >= (1 << 24) || R->N >= (1 << 24)))
        return fail(BPMF_E_INVALID, "BF16 precision needs M and N below 2^24");
    if (!R->d_row_ptr || !R->d_col_ptr) return fail(BPMF_E_INVALID, "NULL row_ptr/col_ptr");
    if (R->nnz > 0 && (!R->d_col_idx || !R->d_row_val || !R->d_row_idx || !R->d_col_val))
        return fail(BPMF_E_INVALID, "NULL index or value array");
    for (int i = 0; i < p->K; ++i)
        if (!std::isfinite(p->mu0[i])) return fail(BPMF_E_INVALID, "mu0 not finite");
    for (int i = 0; i < p->K; ++i)
        for (int j = 0; j < p->K; ++j)
            if (p->W0[(size_t)i * p->K + j] != p->W0[(size_t)j * p->K + i])
                return fail(BPMF_E_NOT_SPD, "W0 is not symmetric");
    std::vector<double> W(p->W0, p->W0 + (size_t)p->K * p->K), L;
    if (!host_cholesky(p->K, W, L)) return fail(BPMF_E_NOT_SPD, "W0 is not positive definite");
    return BPMF_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *bpmf_status_string(bpmf_status s)
{
    switch (s) {
    case BPMF_OK: return "ok";
    case BPMF_E_INVALID: return "invalid argument";
    case BPMF_E_NOT_SPD: return "matrix not symmetric positive definite";
    case BPMF_E_WORKSPACE: return "workspace too small";
    case BPMF_E_STATE: return "invalid context state";
    case BPMF_E_HIP: return "HIP runtime error";
    case BPMF_E_NOMEM: return "host allocation failed";
    }
    return "unknown status";
}

const char *bpmf_last_error(void) { return g_last_error.c_str(); }

const char *bpmf_version(void) { return "bpmf-gfx950 0.1"; }

bpmf_status bpmf_workspace_size(const bpmf_ratings *R, const bpmf_params *p, int64_t n_test, size_t *bytes)
{
    bpmf_status st = check_params(R, p);
    if (st != BPMF_OK) return st;
    if (!bytes) return fail(BPMF_E_INVALID, "NULL bytes");
    if (n_test < 0) return fail(BPMF_E_INVALID, "n_test < 0");
    *bytes = layout(R, p, n_test).total;
    return BPMF_OK;
}

bpmf_status bpmf_init(bpmf_ctx **out, const bpmf_ratings *R, const bpmf_params *p, void *d_U,
                      void *d_V, void *d_ws, size_t ws_bytes, int64_t n_test,
                      const int32_t *d_test_rows, const int32_t *d_test_cols, void *stream)
{
    if (!out) return fail(BPMF_E_INVALID, "NULL ctx output");
    *out = nullptr;
    bpmf_status st = check_params(R, p);
    if (st != BPMF_OK) return st;
    if (!d_U || !d_V) return fail(BPMF_E_INVALID, "NULL U or V");
    if (n_test < 0 || (n_test > 0 && (!d_test_rows || !d_test_cols)))
        return fail(BPMF_E_INVALID, "bad test set");
    Offsets off = layout(R, p, n_test);
    if (!d_ws || ws_bytes < off.total)
        return fail(BPMF_E_WORKSPACE, "workspace needs " + std::to_string(off.total) + " bytes");
    hipStream_t s = (hipStream_t)stream;
    const int K = p->K;
    const int64_t n[2] = {R->M, R->N};

    // structure: pointer arrays always, indices when asked
    std::vector<int64_t> ptr[2] = {std::vector<int64_t>(R->M + 1), std::vector<int64_t>(R->N + 1)};
    HIP_OK(hipMemcpyAsync(ptr[0].data(), R->d_row_ptr, sizeof(int64_t) * (R->M + 1), hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(ptr[1].data(), R->d_col_ptr, sizeof(int64_t) * (R->N + 1), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    for (int sd = 0; sd < 2; ++sd) {
        if (ptr[sd][0] != 0 || ptr[sd][n[sd]] != R->nnz)
            return fail(BPMF_E_INVALID, "pointer array must run from 0 to nnz");
        for (int64_t i = 0; i < n[sd]; ++i)
            if (ptr[sd][i + 1] < ptr[sd][i]) return fail(BPMF_E_INVALID, "pointer array decreases");
    }
    if (p->validate && R->nnz > 0) {
        std::vector<int32_t> ci(R->nnz), ri(R->nnz);
        const size_t vb = R->val_is_f64 ? 8 : 4;
        std::vector<char> rv(R->nnz * vb), cv(R->nnz * vb);
        HIP_OK(hipMemcpyAsync(ci.data(), R->d_col_idx, 4 * R->nnz, hipMemcpyDeviceToHost, s));
        HIP_OK(hipMemcpyAsync(ri.data(), R->d_row_idx, 4 * R->nnz, hipMemcpyDeviceToHost, s));
        HIP_OK(hipMemcpyAsync(rv.data(), R->d_row_val, vb * R->nnz, hipMemcpyDeviceToHost, s));
        HIP_OK(hipMemcpyAsync(cv.data(), R->d_col_val, vb * R->nnz, hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        std::string why;
        if (!check_structure(ptr[0], ci, R->N, why)) return fail(BPMF_E_INVALID, "CSR: " + why);
        if (!check_structure(ptr[1], ri, R->M, why)) return fail(BPMF_E_INVALID, "CSC: " + why);
        // CSR == CSC: walk CSR in column-major order via per-column cursors
        std::vector<int64_t> cur(ptr[1].begin(), ptr[1].end() - 1);
        for (int64_t i = 0; i < R->M; ++i)
            for (int64_t t = ptr[0][i]; t < ptr[0][i + 1]; ++t) {
                const int64_t c = ci[t];
                const int64_t u = cur[c]++;
                if (u >= ptr[1][c + 1] || ri[u] != i || std::memcmp(&rv[t * vb], &cv[u * vb], vb) != 0)
                    return fail(BPMF_E_INVALID, "CSR and CSC differ at row " + std::to_string(i));
            }
        for (int64_t t = 0; t < R->nnz; ++t) {
            double x = R->val_is_f64 ? ((double *)rv.data())[t] : ((float *)rv.data())[t];
            if (!std::isfinite(x)) return fail(BPMF_E_INVALID, "non-finite rating value");
        }
    }

    bpmf_ctx *c = new (std::nothrow) bpmf_ctx();
    if (!c) return fail(BPMF_E_NOMEM, "context allocation");
    c->R = *R;
    c->K = K;
    c->KP = padded_k(K);
    c->precision = p->precision;
    c->burnin = p->burnin;
    c->use_graph = p->use_graph;
    c->alpha = p->alpha;
    c->beta0 = p->beta0;
    c->nu0 = p->nu0;
    c->seed = p->seed;
    c->dU = d_U;
    c->dV = d_V;
    c->ws = (char *)(((uintptr_t)d_ws + kAlign - 1) / kAlign * kAlign);
    c->off = off;
    c->state = c->at<DevState>(off.state);
    c->n_test = n_test;
    c->test_rows = d_test_rows;
    c->test_cols = d_test_cols;
    const int slots = stats_slots(K, p->precision == BPMF_FP64 ? 1 : 0);
    for (int sd = 0; sd < 2; ++sd) {
        c->n_chunks[sd] = stats_chunks(n[sd], n[1 - sd], K, slots);
        c->hyp[sd].Lambda = c->at<double>(off.lam[sd]);
        c->hyp[sd].mu = c->at<double>(off.mu[sd]);
        c->hyp[sd].Lmu = c->at<double>(off.lmu[sd]);
        c->hyp[sd].Lambda_f = c->at<float>(off.lamf[sd]);
        c->hyp[sd].Lmu_f = c->at<float>(off.lmuf[sd]);
        c->hyp[sd].Lambda_tri = c->at<float>(off.lamt[sd]);
        c->hyp[sd].alpha = p->alpha;
        c->hyp[sd].acc16 = (p->precision == BPMF_BF16 && padded_k(K) == 64) ? 1 : 0;
        c->hyp[sd].Lambda_acc = (mixed_supported(K, p->precision) && p->precision != BPMF_FP64 && K <= 64)
                                    ? c->at<float>(off.lamacc[sd]) : nullptr;
        c->hyp[sd].Lchol = (mixed_supported(K, p->precision) && p->precision != BPMF_FP64 && K <= 64)
                               ? c->at<float>(off.lchol[sd]) : nullptr;
    }
    auto bail = [&](bpmf_status e) { delete c; return e; };
#define HIP_OK_C(expr)                                                                      \
    do {                                                                                    \
        hipError_t _e = (expr);                                                             \
        if (_e != hipSuccess) return bail(fail(BPMF_E_HIP, std::string(#expr) + ": " + hipGetErrorString(_e))); \
    } while (0)

    HIP_OK_C(prepare_rows_f64(K));
    HIP_OK_C(prepare_nw());
    HIP_OK_C(launch_fill_zero(c->ws, off.total - kAlign, s));

    // mean rating
    double rbar = p->mean_rating;
    if (std::isnan(rbar)) {
        if (R->nnz == 0) {
            rbar = 0.0;
        } else {
            const int nblk = 1024;
            HIP_OK_C(launch_sum_values(R->d_row_val, R->val_is_f64, R->nnz, c->at<double>(off.reduce), nblk, s));
            std::vector<double> part(nblk);
            HIP_OK_C(hipMemcpyAsync(part.data(), c->at<double>(off.reduce), sizeof(double) * nblk, hipMemcpyDeviceToHost, s));
            HIP_OK_C(hipStreamSynchronize(s));
            double sum = 0.0;
            for (double v : part) sum += v;
            rbar = sum / (double)R->nnz;
        }
    }
    c->rbar = rbar;

    const LaunchShape shape = resolve_shape(p->shape, K);
    c->records = p->precision == BPMF_BF16 && mixed_supported(K, p->precision);
    c->variant = shape.variant;
    // row order (rating count descending, ties by index) and launch table
    for (int sd = 0; sd < 2; ++sd) {
        const PlanShape ps{shape.heavy_min, shape.piece_min, shape.rank1_max, shape.heavy_split, shape.rank1_split};
        const SidePlan sp = plan_side(ptr[sd], n[sd], R->nnz, ps, c->hyp[sd].Lchol != nullptr, K, kMaxPieces,
                                      c->records ? bf16_chunk(c->KP) : 0);
        static_assert(sizeof(PlanEntry) == sizeof(int4), "launch-table entries are the kernels' int4");
        HIP_OK_C(hipMemcpyAsync(c->at<int32_t>(off.order[sd]), sp.order.data(), sizeof(int32_t) * n[sd],
                                hipMemcpyHostToDevice, s));
        c->n_small[sd] = sp.n_small;
        c->n_tiny[sd] = sp.n_tiny;
        c->n_heavy[sd] = sp.n_heavy;
        c->n_pieces[sd] = sp.n_pieces;
        c->n_entries[sd] = (int64_t)sp.tab.size();
        const std::vector<PlanEntry> &tab = sp.tab, &ctab = sp.ctab;
        HIP_OK_C(hipMemcpyAsync(c->at<int4>(off.rowtab[sd]), tab.data(), sizeof(PlanEntry) * tab.size(),
                                hipMemcpyHostToDevice, s));
        if (c->records)
            HIP_OK_C(hipMemcpyAsync(c->at<int64_t>(off.recoff[sd]), sp.recoff.data(),
                                    sizeof(int64_t) * sp.recoff.size(), hipMemcpyHostToDevice, s));
        if (!ctab.empty())
            HIP_OK_C(hipMemcpyAsync(c->at<int4>(off.ctab[sd]), ctab.data(), sizeof(int4) * ctab.size(),
                                    hipMemcpyHostToDevice, s));
        HIP_OK_C(hipStreamSynchronize(s));
    }
    // held-out pairs sorted by user (then movie) so that predictions reuse rows
    if (n_test > 0) {
        std::vector<int32_t> tr(n_test), tc(n_test);
        HIP_OK_C(hipMemcpyAsync(tr.data(), d_test_rows, 4 * n_test, hipMemcpyDeviceToHost, s));
        HIP_OK_C(hipMemcpyAsync(tc.data(), d_test_cols, 4 * n_test, hipMemcpyDeviceToHost, s));
        HIP_OK_C(hipStreamSynchronize(s));
        for (int64_t t = 0; t < n_test; ++t)
            if (tr[t] < 0 || tr[t] >= R->M || tc[t] < 0 || tc[t] >= R->N)
                return bail(fail(BPMF_E_INVALID, "test pair out of range at " + std::to_string(t)));
        std::vector<int64_t> perm(n_test);
        std::iota(perm.begin(), perm.end(), 0);
        std::stable_sort(perm.begin(), perm.end(), [&](int64_t a, int64_t b) {
            return tr[a] != tr[b] ? tr[a] < tr[b] : tc[a] < tc[b];
        });
        std::vector<int32_t> sr(n_test), sc(n_test);
        for (int64_t t = 0; t < n_test; ++t) {
            sr[t] = tr[perm[t]];
            sc[t] = tc[perm[t]];
        }
        HIP_OK_C(hipMemcpyAsync(c->at<int32_t>(off.trows), sr.data(), 4 * n_test, hipMemcpyHostToDevice, s));
        HIP_OK_C(hipMemcpyAsync(c->at<int32_t>(off.tcols), sc.data(), 4 * n_test, hipMemcpyHostToDevice, s));
        HIP_OK_C(hipMemcpyAsync(c->at<int64_t>(off.tperm), perm.data(), 8 * n_test, hipMemcpyHostToDevice, s));
        HIP_OK_C(hipStreamSynchronize(s));
    }
    // priors
    std::vector<double> W0(p->W0, p->W0 + (size_t)K * K), W0inv;
    if (!host_spd_inverse(K, W0, W0inv)) return bail(fail(BPMF_E_NOT_SPD, "W0 is not positive definite"));
    HIP_OK_C(hipMemcpyAsync(c->at<double>(off.mu0), p->mu0, sizeof(double) * K, hipMemcpyHostToDevice, s));
    HIP_OK_C(hipMemcpyAsync(c->at<double>(off.w0inv), W0inv.data(), sizeof(double) * K * K, hipMemcpyHostToDevice, s));
    // FP32 copies of the ratings for the mixed kernels
    if (p->precision != BPMF_FP64 && R->val_is_f64) {
        HIP_OK_C(launch_f64_to_f32((const double *)R->d_row_val, c->at<float>(off.valsf[0]), R->nnz, s));
        HIP_OK_C(launch_f64_to_f32((const double *)R->d_col_val, c->at<float>(off.valsf[1]), R->nnz, s));
    }
    // packed rating records of the BF16 row kernels
    if (c->records)
        for (int sd = 0; sd < 2; ++sd) {
            SideArgs a{};
            a.n_other = sd == 0 ? R->N : R->M;
            a.idx = sd == 0 ? R->d_col_idx : R->d_row_idx;
            a.val = R->val_is_f64 ? (const void *)c->at<float>(off.valsf[sd]) : (sd == 0 ? R->d_row_val : R->d_col_val);
            a.rowtab = c->at<int4>(off.rowtab[sd]);
            a.recoff = c->at<int64_t>(off.recoff[sd]);
            HIP_OK_C(launch_build_records(a, c->n_entries[sd], bf16_chunk(c->KP), (float)rbar,
                                          c->at<uint4>(off.rec[sd]), s));
        }
    // BF16 copies of the initial factors
    if (p->precision == BPMF_BF16 && mixed_supported(K, p->precision)) {
        HIP_OK_C(launch_to_bf16((const float *)d_U, R->M, K, c->KP, c->at<uint16_t>(off.shadow[0]), s));
        HIP_OK_C(launch_to_bf16((const float *)d_V, R->N, K, c->KP, c->at<uint16_t>(off.shadow[1]), s));
    }
    HIP_OK_C(hipStreamSynchronize(s));
#undef HIP_OK_C
    *out = c;
    return BPMF_OK;
}

}  // extern "C"

static hipEvent_t take_event(bpmf_ctx *c)
{
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Launch timing: time_begin records a start event (timing enabled only),
// time_end records the stop event and queues the pair under a kernel class.
static hipEvent_t time_begin(bpmf_ctx *c, hipStream_t s)
{
    if (!c->timing) return nullptr;
    hipEvent_t a = take_event(c);
    if (a) hipEventRecord(a, s);
    return a;
}

static void time_end(bpmf_ctx *c, int cls, hipEvent_t a, hipStream_t s)
{
    if (!c->timing || !a) return;
    hipEvent_t b = take_event(c);
    if (!b) return;
    hipEventRecord(b, s);
    c->pending.push_back({cls, {a, b}});
}

static DrawSrc draws_for(bpmf_ctx *c, int side, const double *tape_block)
{
    const int K = c->K;
    DrawSrc d;
    d.tape_nw = tape_block;
    d.tape_rows = tape_block ? tape_block + K + K * (K - 1) / 2 + K : nullptr;
    d.seed = c->seed;
    d.sweep = &c->state->sweep;
    d.side = side;
    return d;
}

// Hyper-parameters of both sides from their current factors (stream s):
// the statistics of U and V in one launch, one reduction, and one launch
// with a workgroup per side for the Normal-Wishart draws.
static bpmf_status enqueue_hyper(bpmf_ctx *c, const DrawSrc &d0, const DrawSrc &d1, hipStream_t s)
{
    const int K = c->K;
    StatsSides ss;
    ss.X[0] = c->dU;
    ss.X[1] = c->dV;
    ss.n[0] = c->R.M;
    ss.n[1] = c->R.N;
    // with device draws the statistics launch also draws the Normal-Wishart
    // randoms (two extra blocks), and the hyper step reads them like a tape
    const bool pre = !d0.tape_nw;
    ss.with_draws = pre ? 1 : 0;
    ss.nu0 = c->nu0;
    for (int sd = 0; sd < 2; ++sd) {
        ss.partials[sd] = c->at<double>(c->off.partials[sd]);
        ss.n_chunks[sd] = c->n_chunks[sd];
        ss.draw_out[sd] = c->at<double>(c->off.nwd[sd]);
        ss.draws[sd] = sd == 0 ? d0 : d1;
    }
    double *const sums[2] = {c->at<double>(c->off.sums[0]), c->at<double>(c->off.sums[1])};
    hipEvent_t t0 = time_begin(c, s);
    HIP_OK(launch_stats(ss, c->x_f64() ? 1 : 0, K, s));
    HIP_OK(launch_stats_reduce(ss, sums, K, s));
    time_end(c, 0, t0, s);
    NwSide nw[2];
    const DrawSrc *d[2] = {&d0, &d1};
    for (int sd = 0; sd < 2; ++sd) {
        nw[sd].sums = sums[sd];
        nw[sd].n = ss.n[sd];
        nw[sd].draws = *d[sd];
        if (pre) nw[sd].draws.tape_nw = ss.draw_out[sd];
        nw[sd].hyp = c->hyp[sd];
    }
    t0 = time_begin(c, s);
    HIP_OK(launch_nw(nw, K, c->at<double>(c->off.mu0), c->beta0, c->nu0, c->at<double>(c->off.w0inv), c->state, s));
    time_end(c, 1, t0, s);
    return BPMF_OK;
}

// Row updates of one side given the other side (stream s).
static bpmf_status enqueue_rows(bpmf_ctx *c, int side, const DrawSrc &d, hipStream_t s)
{
    const int K = c->K;
    const bpmf_ratings &R = c->R;
    const int64_t n = side == 0 ? R.M : R.N;
    const bool f64 = c->precision == BPMF_FP64;
    const bool mixed_kernel = !f64 && mixed_supported(K, c->precision);
    SideArgs a;
    a.n_rows = n;
    a.n_other = side == 0 ? R.N : R.M;
    a.ptr = side == 0 ? R.d_row_ptr : R.d_col_ptr;
    a.idx = side == 0 ? R.d_col_idx : R.d_row_idx;
    const void *vals_orig = side == 0 ? R.d_row_val : R.d_col_val;
    a.X = side == 0 ? c->dU : c->dV;
    a.other = side == 0 ? c->dV : c->dU;
    a.order = c->at<int32_t>(c->off.order[side]);
    a.rowtab = c->at<int4>(c->off.rowtab[side]);
    a.rec = c->records ? c->at<uint4>(c->off.rec[side]) : nullptr;
    a.recoff = c->records ? c->at<int64_t>(c->off.recoff[side]) : nullptr;
    a.shadow_stride = c->KP;
    hipEvent_t t0;
    if (f64) {
        a.val = vals_orig;
        a.val_is_f64 = R.val_is_f64;
        a.other_bf16 = nullptr;
        a.X_bf16 = nullptr;
        t0 = time_begin(c, s);
        HIP_OK(launch_rows_f64(a, K, c->alpha, c->rbar, c->hyp[side], d, nullptr, nullptr, n, 0, c->state, s));
        time_end(c, 2 + side, t0, s);
        return BPMF_OK;
    }
    const bool bf16 = c->precision == BPMF_BF16 && mixed_kernel;
    a.val = R.val_is_f64 ? (const void *)c->at<float>(c->off.valsf[side]) : vals_orig;
    a.val_is_f64 = 0;
    a.other_bf16 = bf16 ? c->at<uint16_t>(c->off.shadow[1 - side]) : nullptr;
    a.X_bf16 = bf16 ? c->at<uint16_t>(c->off.shadow[side]) : nullptr;
    if (!mixed_kernel) {
        // K > 64: FP64 arithmetic on FP32 storage
        t0 = time_begin(c, s);
        HIP_OK(launch_rows_f64(a, K, c->alpha, c->rbar, c->hyp[side], d, nullptr, nullptr, n, 1, c->state, s));
        time_end(c, 2 + side, t0, s);
        return BPMF_OK;
    }
    int32_t *fbl = c->at<int32_t>(c->off.fblist[side]);
    if (K <= 64) {
        // order slots: [0, nh) heavy rows (as np pieces, then one combine
        // entry each), [nh, n - ns) one wavefront per row, [n - ns, n - nt)
        // rank-one updates, [n - nt, n) one lane per row
        const int64_t nh = c->n_heavy[side], np = c->n_pieces[side], ns = c->n_small[side], nt = c->n_tiny[side];
        PieceArgs pc;
        pc.part = c->at<float>(c->off.part[side]);
        pc.ctab = c->at<int4>(c->off.ctab[side]);
        pc.combine = 0;
        t0 = time_begin(c, s);
        HIP_OK(launch_rows_mixed(a, K, c->KP, bf16 ? 1 : 0, c->alpha, c->rbar, c->hyp[side], d, fbl, c->state, pc,
                                 np + (n - ns - nh), c->variant, s));
        time_end(c, 2 + side, t0, s);
        if (nh > 0) {
            pc.combine = 1;
            t0 = time_begin(c, s);
            HIP_OK(launch_rows_mixed(a, K, c->KP, bf16 ? 1 : 0, c->alpha, c->rbar, c->hyp[side], d, fbl, c->state,
                                     pc, nh, c->variant, s));
            time_end(c, 8, t0, s);
        }
        if (ns > 0) {
            t0 = time_begin(c, s);
            HIP_OK(launch_rows_rank1(a, K, c->KP, bf16 ? 1 : 0, c->alpha, c->rbar, c->hyp[side], d, fbl, c->state,
                                     n - ns, n - nt, R.nnz, s));
            HIP_OK(launch_rows_tiny(a, K, bf16 ? 1 : 0, c->alpha, c->rbar, c->hyp[side], d, fbl, c->state, n - nt, n,
                                    R.nnz, s));
            time_end(c, 7, t0, s);
        }
    } else {
        t0 = time_begin(c, s);
        HIP_OK(launch_rows_mixed128(a, K, c->alpha, c->rbar, c->hyp[side], d, fbl, c->state, s));
        time_end(c, 2 + side, t0, s);
    }
    t0 = time_begin(c, s);
    HIP_OK(launch_rows_f64(a, K, c->alpha, c->rbar, c->hyp[side], d, c->at<int32_t>(c->off.fblist[side]),
                           &c->state->fb_count[side], n, 1, c->state, s));
    time_end(c, 4, t0, s);
    return BPMF_OK;
}

// One sweep, in Algorithm 1's order with users first: the hyper-parameters
// of both sides (each from its own factors, so they are computed together),
// the users' rows, the movies' rows, the held-out predictions.
static bpmf_status enqueue_sweep(bpmf_ctx *c, const double *tape, hipStream_t s)
{
    const int K = c->K;
    const int64_t hb = (int64_t)K + (int64_t)K * (K - 1) / 2 + K;
    const DrawSrc d0 = draws_for(c, 0, tape);
    const DrawSrc d1 = draws_for(c, 1, tape ? tape + hb + c->R.M * K : nullptr);
    bpmf_status st = enqueue_hyper(c, d0, d1, s);
    if (st != BPMF_OK) return st;
    st = enqueue_rows(c, 0, d0, s);
    if (st != BPMF_OK) return st;
    st = enqueue_rows(c, 1, d1, s);
    if (st != BPMF_OK) return st;
    if (c->n_test > 0) {
        hipEvent_t t0 = time_begin(c, s);
        HIP_OK(launch_predict(c->dU, c->dV, c->x_f64() ? 1 : 0, K, c->rbar, c->n_test,
                              c->at<int32_t>(c->off.trows), c->at<int32_t>(c->off.tcols), nullptr,
                              c->at<double>(c->off.accum), c->state, c->burnin, s));
        time_end(c, 5, t0, s);
    }
    hipEvent_t t1 = time_begin(c, s);
    HIP_OK(launch_advance_burnin(c->state, c->burnin, s));
    time_end(c, 6, t1, s);
    return BPMF_OK;
}

extern "C" {

bpmf_status bpmf_sweep(bpmf_ctx *c, int32_t n_sweeps, const double *d_tape, int64_t tape_len, void *stream)
{
    if (!c || c->broken) return fail(BPMF_E_STATE, "context is NULL or unusable");
    if (n_sweeps < 0) return fail(BPMF_E_INVALID, "n_sweeps < 0");
    hipStream_t s = (hipStream_t)stream;
    const int K = c->K;
    const int64_t hb = (int64_t)K + (int64_t)K * (K - 1) / 2 + K;
    const int64_t sweep_len = 2 * hb + (c->R.M + c->R.N) * K;
    if (d_tape) {
        if (tape_len != (int64_t)n_sweeps * sweep_len)
            return fail(BPMF_E_INVALID, "tape length " + std::to_string(tape_len) + " != " +
                                            std::to_string((int64_t)n_sweeps * sweep_len));
        for (int i = 0; i < n_sweeps; ++i) {
            bpmf_status st = enqueue_sweep(c, d_tape + (int64_t)i * sweep_len, s);
            if (st != BPMF_OK) { c->broken = true; return st; }
        }
        return BPMF_OK;
    }
    if (!c->use_graph || c->timing) {
        for (int i = 0; i < n_sweeps; ++i) {
            bpmf_status st = enqueue_sweep(c, nullptr, s);
            if (st != BPMF_OK) { c->broken = true; return st; }
        }
        return BPMF_OK;
    }
    if (!c->gexec) {
        HIP_OK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        HIP_OK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
        bpmf_status st = enqueue_sweep(c, nullptr, c->cap_stream);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
        if (st != BPMF_OK) { c->broken = true; return st; }
        if (e != hipSuccess) { c->broken = true; return fail(BPMF_E_HIP, std::string("graph capture: ") + hipGetErrorString(e)); }
        c->graph = g;
        HIP_OK(hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0));
    }
    for (int i = 0; i < n_sweeps; ++i) HIP_OK(hipGraphLaunch(c->gexec, s));
    return BPMF_OK;
}

bpmf_status bpmf_predict(bpmf_ctx *c, int64_t n, const int32_t *d_rows, const int32_t *d_cols, double *d_out, void *stream)
{
    if (!c || c->broken) return fail(BPMF_E_STATE, "context is NULL or unusable");
    if (n < 0 || (n > 0 && (!d_rows || !d_cols || !d_out))) return fail(BPMF_E_INVALID, "bad predict arguments");
    HIP_OK(launch_predict(c->dU, c->dV, c->x_f64() ? 1 : 0, c->K, c->rbar, n, d_rows, d_cols, d_out, nullptr, c->state, 0, (hipStream_t)stream));
    return BPMF_OK;
}

bpmf_status bpmf_test_predictions(bpmf_ctx *c, double *d_mean, int64_t *h_count, void *stream)
{
    if (!c || c->broken) return fail(BPMF_E_STATE, "context is NULL or unusable");
    hipStream_t s = (hipStream_t)stream;
    if (c->n_test > 0) {
        if (!d_mean) return fail(BPMF_E_INVALID, "NULL d_mean");
        HIP_OK(launch_mean_from_sum(c->at<double>(c->off.accum), c->at<int64_t>(c->off.tperm), c->n_test,
                                    c->state, d_mean, s));
    }
    DevState h;
    HIP_OK(hipMemcpyAsync(&h, c->state, sizeof(DevState), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (h_count) *h_count = h.pred_count;
    return BPMF_OK;
}

bpmf_status bpmf_get_hyper(bpmf_ctx *c, double *h_out, void *stream)
{
    if (!c || c->broken) return fail(BPMF_E_STATE, "context is NULL or unusable");
    if (!h_out) return fail(BPMF_E_INVALID, "NULL output");
    hipStream_t s = (hipStream_t)stream;
    const int K = c->K;
    for (int sd = 0; sd < 2; ++sd) {
        double *o = h_out + sd * (K * K + K);
        HIP_OK(hipMemcpyAsync(o, c->hyp[sd].Lambda, sizeof(double) * K * K, hipMemcpyDeviceToHost, s));
        HIP_OK(hipMemcpyAsync(o + K * K, c->hyp[sd].mu, sizeof(double) * K, hipMemcpyDeviceToHost, s));
    }
    HIP_OK(hipStreamSynchronize(s));
    return BPMF_OK;
}

bpmf_status bpmf_get_info(bpmf_ctx *c, bpmf_info *info, void *stream)
{
    if (!c || c->broken) return fail(BPMF_E_STATE, "context is NULL or unusable");
    if (!info) return fail(BPMF_E_INVALID, "NULL info");
    hipStream_t s = (hipStream_t)stream;
    DevState h;
    HIP_OK(hipMemcpyAsync(&h, c->state, sizeof(DevState), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    info->sweeps_done = h.sweep;
    info->fallback_rows = h.fallback_rows;
    info->nonfinite_rows = h.nonfinite_rows;
    info->mean_rating = c->rbar;
    info->K = c->K;
    info->precision = c->precision;
    for (int sd = 0; sd < 2; ++sd) {
        info->rank1_rows[sd] = c->n_small[sd];
        info->heavy_rows[sd] = c->n_heavy[sd];
        info->pieces[sd] = c->n_pieces[sd];
    }
    info->kernel_variant = (c->precision != BPMF_FP64 && c->K <= 64) ? c->variant : 0;
    return BPMF_OK;
}

bpmf_status bpmf_snapshot(bpmf_ctx *c, float *d_V_slot, double *d_Lambda_slot, double *d_mu_slot, void *stream)
{
    if (!c || c->broken) return fail(BPMF_E_STATE, "context is NULL or unusable");
    if (!d_V_slot || !d_Lambda_slot || !d_mu_slot) return fail(BPMF_E_INVALID, "NULL slot");
    hipStream_t s = (hipStream_t)stream;
    const int K = c->K;
    HIP_OK(launch_copy_f32_from(c->dV, c->x_f64() ? 1 : 0, c->R.N * K, d_V_slot, s));
    HIP_OK(hipMemcpyAsync(d_Lambda_slot, c->hyp[0].Lambda, sizeof(double) * K * K, hipMemcpyDeviceToDevice, s));
    HIP_OK(hipMemcpyAsync(d_mu_slot, c->hyp[0].mu, sizeof(double) * K, hipMemcpyDeviceToDevice, s));
    return BPMF_OK;
}

static size_t state_bytes(bpmf_ctx *c)
{
    const size_t xb = c->x_f64() ? 8 : 4;
    const int K = c->K;
    return sizeof(DevState) + xb * (size_t)(c->R.M + c->R.N) * K + 2 * sizeof(double) * (K * K + 2 * K) +
           sizeof(double) * (size_t)c->n_test;
}

bpmf_status bpmf_state_size(bpmf_ctx *c, size_t *bytes)
{
    if (!c || c->broken) return fail(BPMF_E_STATE, "context is NULL or unusable");
    if (!bytes) return fail(BPMF_E_INVALID, "NULL bytes");
    *bytes = state_bytes(c);
    return BPMF_OK;
}

static bpmf_status state_copy(bpmf_ctx *c, char *h, bool save, hipStream_t s)
{
    const size_t xb = c->x_f64() ? 8 : 4;
    const int K = c->K;
    auto cp = [&](void *dev, size_t n) -> hipError_t {
        hipError_t e = save ? hipMemcpyAsync(h, dev, n, hipMemcpyDeviceToHost, s)
                            : hipMemcpyAsync(dev, h, n, hipMemcpyHostToDevice, s);
        h += n;
        return e;
    };
    HIP_OK(cp(c->state, sizeof(DevState)));
    HIP_OK(cp(c->dU, xb * c->R.M * K));
    HIP_OK(cp(c->dV, xb * c->R.N * K));
    for (int sd = 0; sd < 2; ++sd) {
        HIP_OK(cp(c->hyp[sd].Lambda, sizeof(double) * K * K));
        HIP_OK(cp(c->hyp[sd].mu, sizeof(double) * K));
        HIP_OK(cp(c->hyp[sd].Lmu, sizeof(double) * K));
    }
    if (c->n_test > 0) HIP_OK(cp(c->at<double>(c->off.accum), sizeof(double) * c->n_test));
    if (!save) {
        for (int sd = 0; sd < 2; ++sd) {
            HIP_OK(launch_f64_to_f32(c->hyp[sd].Lambda, c->hyp[sd].Lambda_f, (int64_t)K * K, s));
            HIP_OK(launch_f64_to_f32(c->hyp[sd].Lmu, c->hyp[sd].Lmu_f, K, s));
            HIP_OK(launch_lambda_tri(c->hyp[sd], K, c->KP, s));
        }
        if (c->precision == BPMF_BF16 && mixed_supported(K, c->precision)) {
            HIP_OK(launch_to_bf16((const float *)c->dU, c->R.M, K, c->KP, c->at<uint16_t>(c->off.shadow[0]), s));
            HIP_OK(launch_to_bf16((const float *)c->dV, c->R.N, K, c->KP, c->at<uint16_t>(c->off.shadow[1]), s));
        }
    }
    HIP_OK(hipStreamSynchronize(s));
    return BPMF_OK;
}

bpmf_status bpmf_state_save(bpmf_ctx *c, void *h_buf, size_t bytes, void *stream)
{
    if (!c || c->broken) return fail(BPMF_E_STATE, "context is NULL or unusable");
    if (!h_buf || bytes < state_bytes(c)) return fail(BPMF_E_INVALID, "state buffer too small");
    return state_copy(c, (char *)h_buf, true, (hipStream_t)stream);
}

bpmf_status bpmf_state_restore(bpmf_ctx *c, const void *h_buf, size_t bytes, void *stream)
{
    if (!c || c->broken) return fail(BPMF_E_STATE, "context is NULL or unusable");
    if (!h_buf || bytes < state_bytes(c)) return fail(BPMF_E_INVALID, "state buffer too small");
    return state_copy(c, (char *)h_buf, false, (hipStream_t)stream);
}

bpmf_status bpmf_set_timing(bpmf_ctx *c, int32_t enable)
{
    if (!c || c->broken) return fail(BPMF_E_STATE, "context is NULL or unusable");
    c->timing = enable != 0;
    return BPMF_OK;
}

bpmf_status bpmf_get_timing(bpmf_ctx *c, bpmf_timing *out, int32_t reset)
{
    if (!c || c->broken) return fail(BPMF_E_STATE, "context is NULL or unusable");
    if (!out) return fail(BPMF_E_INVALID, "NULL output");
    for (auto &p : c->pending) {
        HIP_OK(hipEventSynchronize(p.second.second));
        float ms = 0.0f;
        HIP_OK(hipEventElapsedTime(&ms, p.second.first, p.second.second));
        c->t_ms[p.first] += ms;
        c->t_n[p.first] += 1;
        c->pool.push_back(p.second.first);
        c->pool.push_back(p.second.second);
    }
    c->pending.clear();
    for (int i = 0; i < BPMF_TIMING_CLASSES; ++i) {
        out->ms[i] = c->t_ms[i];
        out->launches[i] = c->t_n[i];
        if (reset) {
            c->t_ms[i] = 0.0;
            c->t_n[i] = 0;
        }
    }
    return BPMF_OK;
}

bpmf_status bpmf_destroy(bpmf_ctx *c)
{
    if (!c) return BPMF_OK;
    for (auto &p : c->pending) {
        hipEventDestroy(p.second.first);
        hipEventDestroy(p.second.second);
    }
    for (hipEvent_t e : c->pool) hipEventDestroy(e);
    if (c->gexec) hipGraphExecDestroy(c->gexec);
    if (c->graph) hipGraphDestroy(c->graph);
    if (c->cap_stream) hipStreamDestroy(c->cap_stream);
    delete c;
    return BPMF_OK;
}

bpmf_status bpmf_foldin_workspace_size(const bpmf_foldin_model *m, int64_t n_queries, size_t *bytes)
{
    if (!m || !bytes) return fail(BPMF_E_INVALID, "NULL argument");
    if (m->S < 1 || n_queries < 0) return fail(BPMF_E_INVALID, "S must be >= 1, n_queries >= 0");
    *bytes = sizeof(float) * (size_t)m->S * (size_t)std::max<int64_t>(n_queries, 1);
    return BPMF_OK;
}

static bpmf_status check_foldin_model(const bpmf_foldin_model *m)
{
    if (!m) return fail(BPMF_E_INVALID, "NULL model");
    if (m->S < 1 || m->K < 1 || m->K > 64 || m->N < 1) return fail(BPMF_E_INVALID, "fold-in needs S >= 1, 1 <= K <= 64, N >= 1");
    if (!m->d_V || !m->d_Lambda || !m->d_mu) return fail(BPMF_E_INVALID, "NULL model arrays");
    if (!(m->alpha > 0.0)) return fail(BPMF_E_INVALID, "alpha must be > 0");
    return BPMF_OK;
}

int64_t bpmf_foldin_noalloc_max_partials(void) { return foldin_noalloc_max_partials(); }

bpmf_status bpmf_foldin_noalloc(const bpmf_foldin_model *m, int64_t n_req, const int64_t *d_req_ptr,
                                const int32_t *d_cols, const float *d_vals, const int64_t *d_q_ptr,
                                const int32_t *d_q_cols, int64_t n_queries, float *d_out, void *stream)
{
    bpmf_status st = check_foldin_model(m);
    if (st != BPMF_OK) return st;
    if (n_req < 0 || n_queries < 0) return fail(BPMF_E_INVALID, "negative sizes");
    if ((int64_t)m->S * n_queries > foldin_noalloc_max_partials())
        return fail(BPMF_E_INVALID, "S * n_queries = " + std::to_string((int64_t)m->S * n_queries) +
                                        " exceeds the " + std::to_string(foldin_noalloc_max_partials()) +
                                        " partials of the library's fold-in array");
    if (n_req == 0) return BPMF_OK;
    if (!d_req_ptr || !d_q_ptr || (n_queries > 0 && (!d_q_cols || !d_out)))
        return fail(BPMF_E_INVALID, "NULL request arrays");
    float *partial = nullptr;
    HIP_OK(foldin_noalloc_scratch(&partial));
    HIP_OK(launch_foldin(m->S, m->K, m->N, m->alpha, m->mean_rating, m->d_V, m->d_Lambda, m->d_mu, n_req,
                         d_req_ptr, d_cols, d_vals, d_q_ptr, d_q_cols, n_queries, partial, d_out,
                         (hipStream_t)stream));
    return BPMF_OK;
}

bpmf_status bpmf_foldin(const bpmf_foldin_model *m, int64_t n_req, const int64_t *d_req_ptr,
                        const int32_t *d_cols, const float *d_vals, const int64_t *d_q_ptr,
                        const int32_t *d_q_cols, int64_t n_queries, float *d_out, void *d_ws,
                        size_t ws_bytes, void *stream)
{
    bpmf_status st = check_foldin_model(m);
    if (st != BPMF_OK) return st;
    if (n_req < 0 || n_queries < 0) return fail(BPMF_E_INVALID, "negative sizes");
    if (n_req == 0) return BPMF_OK;
    if (!d_req_ptr || !d_q_ptr || (n_queries > 0 && (!d_q_cols || !d_out)))
        return fail(BPMF_E_INVALID, "NULL request arrays");
    size_t need = 0;
    bpmf_foldin_workspace_size(m, n_queries, &need);
    if (!d_ws || ws_bytes < need) return fail(BPMF_E_WORKSPACE, "fold-in workspace needs " + std::to_string(need) + " bytes");
    HIP_OK(launch_foldin(m->S, m->K, m->N, m->alpha, m->mean_rating, m->d_V, m->d_Lambda, m->d_mu, n_req,
                         d_req_ptr, d_cols, d_vals, d_q_ptr, d_q_cols, n_queries, (float *)d_ws, d_out,
                         (hipStream_t)stream));
    return BPMF_OK;
}

}  // extern "C"
