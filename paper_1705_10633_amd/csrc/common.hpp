// common.hpp -- shared declarations of the HIP kernels and the host library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace bpmf {

// Sets the thread-local message returned by bpmf_last_error().
void set_last_error(const std::string &msg);

// Where a half-sweep's standard normals come from: a tape block (row-major
// n x K doubles) or the device counter-based generator at half-sweep
// h = 2 * (*sweep) + side.
struct DrawSrc {
    const double *tape_rows;   // NULL -> counter-based generator
    const double *tape_nw;     // [K chi2][K(K-1)/2 Bartlett][K mean normals] or NULL
    uint64_t seed;
    const int64_t *sweep;      // device sweep counter
    int32_t side;              // 0 users, 1 movies
};

__device__ __forceinline__ uint32_t half_sweep_index(const DrawSrc &d)
{
    return (uint32_t)(2 * (*d.sweep) + d.side);
}

// Device-resident counters of a sampler.
struct DevState {
    int64_t sweep;            // sweeps completed
    int64_t pred_count;       // sweeps entered into the test-prediction mean
    int64_t fallback_rows;    // cumulative FP64 recomputes
    int64_t nonfinite_rows;   // cumulative non-finite FP64 rows
    int32_t fb_count[2];      // rows queued for FP64 recompute in the current half-sweep
    int32_t pad[2];
};

// Hyper-parameters of one side, FP64 with FP32 copies for the mixed kernels.
struct HyperDev {
    double *Lambda;  // K x K
    double *mu;      // K
    double *Lmu;     // K  (Lambda mu)
    float *Lambda_f; // K x K
    float *Lmu_f;    // K
    // FP32 Lambda as the mixed row kernel's packed lower triangle of the
    // padded size KP (row r at r (r + 1) / 2, identity in the padding), KP (KP + 3) / 2 floats
    float *Lambda_tri;
    // FP32 Lambda / alpha in the K <= 64 row kernel's Gram accumulator
    // layout, or NULL: entry (t * 16 + e) * 64 + l is Lambda[r][c] / alpha of
    // lower 32 x 32 tile t ((0,0), (1,0), (1,1)), r = 32 a + 8 (e / 4) +
    // 4 (l / 32) + e % 4, c = 32 b + l % 32 (identity in the padding); the
    // row kernel's accumulators start from it
    float *Lambda_acc;
    int32_t acc16;   // Lambda_acc in the 16 x 16 tile layout (BF16, KP = 64)
    double alpha;    // the sampler's alpha
    // chol(Lambda) in FP32 for the rank-one row paths (K <= 64), or NULL:
    // KP x KP row-major (lower; identity in the padding), then KP floats each
    // of 1 / L_ii, L^T mu (= L^{-1} Lambda mu), Lambda_ii (0 in the padding)
    // and 1 / 0 flags of the live components
    float *Lchol;
};

// One half-sweep: rows of one side against the other side's factors.
struct SideArgs {
    int64_t n_rows;
    int64_t n_other;        // rows of the other side (its BF16 copy has one more, all zeros)
    const int64_t *ptr;
    const int32_t *idx;
    const void *val;        // float or double ratings
    int32_t val_is_f64;
    const void *other;      // master of the other side (double in FP64 mode, else float)
    const uint16_t *other_bf16;  // BF16 copy of the other side (row stride KP), BF16 mode
    void *X;                // master of this side (output)
    uint16_t *X_bf16;       // BF16 copy of this side (output), or NULL
    int32_t shadow_stride;  // row stride of the BF16 copies
    const int32_t *order;   // rows in processing order (nnz descending)
    // per order slot {row, rating count, first rating (low, high word)}: one
    // 16-byte load instead of the order entry and then the row pointers
    const int4 *rowtab;
    // BF16 mode: the ratings of each launch-table entry as packed records,
    // one 32-byte record per 4 ratings: {4 column indices} then the offsets
    // r' = r - rbar of the 4 ratings as two BF16 parts hi = bf16(r'),
    // lo = bf16(r' - hi), packed {hi0 | hi1 << 16, hi2 | hi3 << 16,
    // lo0 | lo1 << 16, lo2 | lo3 << 16}.  Every entry is padded to a multiple
    // of the kernel's chunk with records of the all-zero row and r' = 0, so
    // the gathers need no bounds.  Entry e starts at record recoff[e]
    // (uint4 rec[2 * recoff[e]]).  NULL outside BF16 mode.
    const uint4 *rec;
    const int64_t *recoff;
};

// Ratings per chunk of the BF16 row kernels, which each entry's records are
// padded to: KP = 32 and 128: 64; KP = 64: 32.
__host__ __device__ constexpr int bf16_chunk(int KP) { return KP == 64 ? 32 : 64; }

// Masked loads are written as an unconditional load (from a clamped, valid
// index) scaled or blended by the mask, so the compiler does not put each
// load behind its own branch (which also waits for every load in flight).
__device__ __forceinline__ int blend_idx(bool ok, int v, int other)
{
    const int m = -(int)ok;
    return (v & m) | (other & ~m);
}

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f)
{
    // one v_cvt_pk_bf16_f32 on gfx950: round to nearest even, NaN stays NaN
    const __bf16 h = (__bf16)f;
    uint16_t u;
    __builtin_memcpy(&u, &h, 2);
    return u;
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h)
{
    return __uint_as_float(((uint32_t)h) << 16);
}

// ---------------------------------------------------------------------------
// Launchers (defined in the .hip files; all return hipError_t of the launch)
// ---------------------------------------------------------------------------
// Both sides of a sweep's hyper-parameter step (0 users, 1 movies).
struct StatsSides {
    const void *X[2];      // factor matrices (FP64 or FP32)
    int64_t n[2];          // rows
    double *partials[2];   // per-chunk partial sums
    int n_chunks[2];
    // Optional (K <= 64, device draws): two more blocks draw each side's
    // Normal-Wishart randoms into draw_out[side] in the tape layout
    // [K chi^2][K(K-1)/2 Bartlett normals][K mean normals].
    double *draw_out[2];
    DrawSrc draws[2];
    double nu0;
    int with_draws;
};
struct NwSide {
    const double *sums;    // sum x (K) then sum x x^T (packed lower, K(K+1)/2)
    int64_t n;
    DrawSrc draws;
    HyperDev hyp;
};
hipError_t launch_stats(const StatsSides &ss, int x_is_f64, int K, hipStream_t s);
int stats_chunks(int64_t n, int64_t n_other, int K, int slots);
int stats_slots(int K, int x_is_f64);
hipError_t launch_stats_reduce(const StatsSides &ss, double *const sums[2], int K, hipStream_t s);
hipError_t launch_nw(const NwSide sides[2], int K, const double *mu0, double beta0, double nu0,
                     const double *W0inv, DevState *state, hipStream_t s);
hipError_t launch_rows_f64(const SideArgs &a, int K, double alpha, double rbar,
                           HyperDev hyp, DrawSrc draws, const int32_t *list,
                           const int32_t *list_count, int64_t max_rows, int x_is_f32,
                           DevState *state, hipStream_t s);
hipError_t launch_rows_mixed128(const SideArgs &a, int K, double alpha, double rbar, HyperDev hyp,
                                DrawSrc draws, int32_t *fb_list, DevState *state, hipStream_t s);
// Pieces of heavy rows (see rows_mixed_kernel): per piece, the partial Gram
// tiles in accumulator layout plus the right-hand side, floats per piece (the
// stride; the 16 x 16 tile layout uses 40 x 64 + 64 of them):
__host__ __device__ constexpr int piece_floats(int KP) { return (KP == 64 ? 3 : 1) * 16 * 64 + 64; }

// Position of Lambda[r][c] (both < 64) in the accumulator layout of
// HyperDev::Lambda_acc (-1 for an upper tile): lower 32 x 32 tiles, or with
// g16 the ten lower 16 x 16 tiles (the K <= 64 BF16 row kernel's layout for
// KP = 64; see GramAcc).
__host__ __device__ inline int lambda_acc_index(int r, int c, bool g16)
{
    if (g16) {
        const int a = r >> 4, b = c >> 4;
        if (a < b) return -1;
        const int rr = r & 15;
        return (4 * (a * (a + 1) / 2 + b) + (rr & 3)) * 64 + 16 * (rr >> 2) + (c & 15);
    }
    const int ta = r >> 5, tb = c >> 5;
    if (ta < tb) return -1;
    const int t = ta == 0 ? 0 : (tb == 0 ? 1 : 2);
    const int rr = r & 31;
    return (t * 16 + 4 * (rr >> 3) + (rr & 3)) * 64 + 32 * ((rr >> 2) & 1) + (c & 31);
}
struct PieceArgs {
    float *part;        // piece partial sums
    const int4 *ctab;   // combine launch: per heavy row {row, first piece, piece count, 0}
    int32_t combine;    // 0: the launch table a.rowtab (pieces then rows); 1: combine
};
// n_entries entries of a.rowtab (pieces have row < 0), or with pc.combine
// n_entries heavy rows from pc.ctab.
// variant: bpmf_launch_shape::kernel_variant resolved (1..3; KP = 64 only).
hipError_t launch_rows_mixed(const SideArgs &a, int K, int KP, int bf16, double alpha,
                             double rbar, HyperDev hyp, DrawSrc draws, int32_t *fb_list,
                             DevState *state, PieceArgs pc, int64_t n_entries, int variant, hipStream_t s);
// Rows with at least this many ratings are cut into pieces (K <= 64).
int heavy_min_ratings();
// Rows in order slots [slot0, slot1), each with at most rank1_max_ratings()
// ratings, by rank-one updates of chol(Lambda) (K <= 64, hyp.Lchol set).
int rank1_max_ratings();
// Rows in order slots [slot0, slot1) with at most one rating, K <= 32: one
// lane per row, closed-form factor of I + p p^T.
hipError_t launch_rows_tiny(const SideArgs &a, int K, int bf16, double alpha, double rbar, HyperDev hyp,
                            DrawSrc draws, int32_t *fb_list, DevState *state, int64_t slot0, int64_t slot1,
                            int64_t nnz, hipStream_t s);
hipError_t launch_rows_rank1(const SideArgs &a, int K, int KP, int bf16, double alpha, double rbar, HyperDev hyp,
                             DrawSrc draws, int32_t *fb_list, DevState *state, int64_t slot0, int64_t slot1,
                             int64_t nnz, hipStream_t s);
// Packed rating records (SideArgs::rec) of n_entries launch-table entries of
// a.rowtab, each padded to a multiple of `chunk` ratings.
hipError_t launch_build_records(const SideArgs &a, int64_t n_entries, int chunk, float rbar, uint4 *rec,
                                hipStream_t s);
hipError_t launch_predict(const void *U, const void *V, int x_is_f64, int K, double rbar,
                          int64_t n, const int32_t *rows, const int32_t *cols, double *out,
                          double *accum, const DevState *state, int burnin, hipStream_t s);
hipError_t launch_advance_burnin(DevState *state, int burnin, hipStream_t s);
hipError_t launch_lambda_tri(HyperDev hyp, int K, int KP, hipStream_t s);
hipError_t prepare_nw();
hipError_t launch_to_bf16(const float *X, int64_t n, int K, int stride, uint16_t *out,
                          hipStream_t s);
hipError_t launch_f64_to_f32(const double *in, float *out, int64_t n, hipStream_t s);
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s);
hipError_t launch_copy_f32_from(const void *X, int x_is_f64, int64_t n, float *out,
                                hipStream_t s);

}  // namespace bpmf
