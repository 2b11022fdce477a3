// plan.hpp -- host-side planning of a sampler, plain C++17 (no HIP): the
// structure checks of the rating matrix, the host Cholesky used for W0, and
// the launch table of a side (rows ordered by rating count, heavy rows cut
// into pieces, the rank-one tail, the packed-record offsets).  Kept free of
// device types so the same code can be built with host sanitizers.
#pragma once
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <numeric>
#include <string>
#include <vector>

namespace bpmf {

// One launch-table entry, laid out as the kernels' int4:
// rows: {row, rating count, first rating (low, high word)};
// pieces of a heavy row: {-(piece index) - 1, count, first rating (low, high)};
// combine table: {row, first piece, piece count, 0}.
struct PlanEntry {
    int32_t x, y, z, w;
};

inline bool host_cholesky(int n, const std::vector<double> &A, std::vector<double> &L)
{
    L.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j <= i; ++j) {
            double s = A[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) s -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
            if (i == j) {
                if (!(s > 0.0) || !std::isfinite(s)) return false;
                L[(size_t)i * n + i] = std::sqrt(s);
            } else {
                L[(size_t)i * n + j] = s / L[(size_t)j * n + j];
            }
        }
    return true;
}

inline bool host_spd_inverse(int n, const std::vector<double> &A, std::vector<double> &inv)
{
    std::vector<double> L;
    if (!host_cholesky(n, A, L)) return false;
    // inv = L^{-T} L^{-1}; first Li = L^{-1}
    std::vector<double> Li((size_t)n * n, 0.0);
    for (int c = 0; c < n; ++c) {
        Li[(size_t)c * n + c] = 1.0 / L[(size_t)c * n + c];
        for (int i = c + 1; i < n; ++i) {
            double s = 0.0;
            for (int m = c; m < i; ++m) s += L[(size_t)i * n + m] * Li[(size_t)m * n + c];
            Li[(size_t)i * n + c] = -s / L[(size_t)i * n + i];
        }
    }
    inv.assign((size_t)n * n, 0.0);
    for (int a = 0; a < n; ++a)
        for (int c = 0; c <= a; ++c) {
            double s = 0.0;
            for (int m = a; m < n; ++m) s += Li[(size_t)m * n + a] * Li[(size_t)m * n + c];
            inv[(size_t)a * n + c] = s;
            inv[(size_t)c * n + a] = s;
        }
    return true;
}

// Pointer array ptr[0..n] with indices idx: starts at 0, nondecreasing,
// indices in [0, n_other) and strictly increasing within a row.
inline bool check_structure(const std::vector<int64_t> &ptr, const std::vector<int32_t> &idx, int64_t n_other,
                            std::string &why)
{
    if (ptr.empty() || ptr[0] != 0) { why = "pointer array must start at 0"; return false; }
    if (ptr.back() > (int64_t)idx.size()) { why = "pointer array runs past the indices"; return false; }
    for (size_t i = 0; i + 1 < ptr.size(); ++i) {
        if (ptr[i + 1] < ptr[i]) { why = "pointer array decreases at " + std::to_string(i); return false; }
        for (int64_t t = ptr[i]; t < ptr[i + 1]; ++t) {
            if (idx[t] < 0 || idx[t] >= n_other) { why = "index out of range in row " + std::to_string(i); return false; }
            if (t > ptr[i] && idx[t] <= idx[t - 1]) { why = "indices not strictly increasing in row " + std::to_string(i); return false; }
        }
    }
    return true;
}

// The launch shape with every field resolved (see bpmf_launch_shape).
struct PlanShape {
    int64_t heavy_min, piece_min, rank1_max;
    int heavy_split, rank1_split;
};

struct SidePlan {
    std::vector<int32_t> order;     // rows by rating count, descending (ties by index)
    std::vector<PlanEntry> tab;     // pieces of the heavy rows, then rows order[n_heavy ..]
    std::vector<PlanEntry> ctab;    // per heavy row: {row, first piece, piece count, 0}
    std::vector<int64_t> recoff;    // first packed record of every tab entry (when records are used)
    int64_t n_small = 0;            // rows at the end of the order for the rank-one kernels
    int64_t n_tiny = 0;             // of which the last ones (at most one rating, K <= 32) one lane each
    int64_t n_heavy = 0;            // rows at the start of the order cut into pieces
    int64_t n_pieces = 0;
    int64_t rec_groups = 0;         // 4-rating records in all
};

// The launch table of one side with n rows (pointer array ptr, nnz ratings of
// the whole matrix).  rank1 = 0: no rank-one kernels (and no heavy pieces) at
// this K and precision.  rec_chunk > 0: packed records, each entry padded to
// a multiple of rec_chunk ratings.
inline SidePlan plan_side(const std::vector<int64_t> &ptr, int64_t n, int64_t nnz, const PlanShape &shape,
                          bool rank1, int K, int64_t max_pieces, int64_t rec_chunk)
{
    SidePlan sp;
    sp.order.resize(n);
    std::iota(sp.order.begin(), sp.order.end(), 0);
    auto cnt = [&](int32_t r) { return ptr[r + 1] - ptr[r]; };
    std::stable_sort(sp.order.begin(), sp.order.end(), [&](int32_t a, int32_t b) { return cnt(a) > cnt(b); });
    const std::vector<int32_t> &ord = sp.order;
    int64_t nh = 0;
    if (rank1) {
        const int64_t lim = shape.rank1_max;
        int64_t m = 0, t = 0;
        while (m < n && cnt(ord[n - 1 - m]) <= lim) {
            if (cnt(ord[n - 1 - m]) <= 1) ++t;
            ++m;
        }
        // a short tail finishes inside the full kernel's launch anyway;
        // a separate launch pays off once it is a sizeable share of the rows
        const bool small_launch = shape.rank1_split > 0 ? m > 0
                                  : (shape.rank1_split == 0 && (m >= 16384 || 16 * m >= n));
        if (!small_launch) m = 0;
        if (small_launch) {
            sp.n_small = m;
            sp.n_tiny = K <= 32 ? t : 0;
        }
        // heavy rows: worth the extra combine launch when they hold a
        // sizeable share of the ratings (otherwise they finish inside the
        // one-wavefront launch anyway)
        int64_t hv = 0, hnnz = 0;
        while (hv < n - m && hv < max_pieces / 2 && cnt(ord[hv]) >= shape.heavy_min) {
            hnnz += cnt(ord[hv]);
            ++hv;
        }
        if (shape.heavy_split > 0 || (shape.heavy_split == 0 && 10 * hnnz >= nnz)) nh = hv;
    }
    if (nh > 0) {
        int64_t hnnz = 0;
        for (int64_t q = 0; q < nh; ++q) hnnz += cnt(ord[q]);
        // sum over rows of ceil(nnz / psz) <= hnnz / psz + nh <= max_pieces
        const int64_t psz = std::max<int64_t>(shape.piece_min, (hnnz + max_pieces - nh - 1) / (max_pieces - nh));
        for (int64_t q = 0; q < nh; ++q) {
            const int64_t b = ptr[ord[q]], e = ptr[ord[q] + 1];
            sp.ctab.push_back({ord[q], (int32_t)sp.tab.size(), 0, 0});
            for (int64_t x = b; x < e; x += psz) {
                const int64_t c = std::min<int64_t>(psz, e - x);
                sp.tab.push_back({-(int32_t)sp.tab.size() - 1, (int32_t)c, (int32_t)(uint32_t)(uint64_t)x,
                                  (int32_t)(uint32_t)((uint64_t)x >> 32)});
            }
            sp.ctab.back().z = (int32_t)sp.tab.size() - sp.ctab.back().y;
        }
    }
    sp.n_heavy = nh;
    sp.n_pieces = (int64_t)sp.tab.size();
    for (int64_t q = nh; q < n; ++q) {
        const int64_t b = ptr[ord[q]];
        sp.tab.push_back({ord[q], (int32_t)cnt(ord[q]), (int32_t)(uint32_t)(uint64_t)b,
                          (int32_t)(uint32_t)((uint64_t)b >> 32)});
    }
    if (rec_chunk > 0) {
        sp.recoff.resize(sp.tab.size());
        int64_t g = 0;
        for (size_t e = 0; e < sp.tab.size(); ++e) {
            sp.recoff[e] = g;
            g += (sp.tab[e].y + rec_chunk - 1) / rec_chunk * (rec_chunk / 4);
        }
        sp.rec_groups = g;
    }
    return sp;
}

}  // namespace bpmf
