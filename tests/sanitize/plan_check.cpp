// Host-sanitizer check of the sampler's planning code (plan.hpp): built with
// -fsanitize=address,undefined by tests/test_sanitizers.py and run on the CPU.
// Random rating-count patterns (rows without ratings, one-rating tails, heavy
// rows) under every launch-shape choice; every invariant the kernels rely on
// is checked, and the structure checks and the host Cholesky get valid and
// corrupted inputs.  Exit status 0 when everything holds.
#include <cstdio>
#include <cstdlib>
#include <random>

#include "plan.hpp"

using namespace bpmf;

static int failures = 0;
#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++failures;                                                 \
        }                                                               \
    } while (0)

static void check_plan(const std::vector<int64_t> &ptr, int64_t n, const PlanShape &sh, bool rank1, int K,
                       int64_t max_pieces, int64_t chunk)
{
    const int64_t nnz = ptr[n];
    const SidePlan sp = plan_side(ptr, n, nnz, sh, rank1, K, max_pieces, chunk);
    CHECK((int64_t)sp.order.size() == n);
    std::vector<int> seen(n, 0);
    for (int32_t r : sp.order) {
        CHECK(r >= 0 && r < n);
        if (r >= 0 && r < n) seen[r]++;
    }
    for (int64_t r = 0; r < n; ++r) CHECK(seen[r] == 1);
    for (int64_t q = 1; q < n; ++q)
        CHECK(ptr[sp.order[q - 1] + 1] - ptr[sp.order[q - 1]] >= ptr[sp.order[q] + 1] - ptr[sp.order[q]]);
    CHECK(sp.n_pieces <= max_pieces);
    CHECK(sp.n_heavy + sp.n_small <= n);
    CHECK(sp.n_tiny <= sp.n_small);
    CHECK((int64_t)sp.tab.size() == sp.n_pieces + n - sp.n_heavy);
    // pieces cover each heavy row's ratings exactly, in order
    CHECK((int64_t)sp.ctab.size() == sp.n_heavy);
    for (int64_t h = 0; h < (int64_t)sp.ctab.size(); ++h) {
        const PlanEntry &c = sp.ctab[h];
        CHECK(c.x == sp.order[h]);
        int64_t at = ptr[c.x];
        for (int32_t p = c.y; p < c.y + c.z; ++p) {
            const PlanEntry &e = sp.tab[p];
            CHECK(e.x == -p - 1);
            const int64_t first = (int64_t)(((uint64_t)(uint32_t)e.w << 32) | (uint32_t)e.z);
            CHECK(first == at);
            at += e.y;
        }
        CHECK(at == ptr[c.x + 1]);
    }
    // the rows after the pieces: the order from n_heavy on, with their ratings
    for (int64_t q = sp.n_heavy; q < n; ++q) {
        const PlanEntry &e = sp.tab[sp.n_pieces + q - sp.n_heavy];
        CHECK(e.x == sp.order[q]);
        const int64_t first = (int64_t)(((uint64_t)(uint32_t)e.w << 32) | (uint32_t)e.z);
        CHECK(first == ptr[e.x] && e.y == ptr[e.x + 1] - ptr[e.x]);
    }
    // rank-one tail: only rows within the limit
    for (int64_t q = n - sp.n_small; q < n; ++q) CHECK(ptr[sp.order[q] + 1] - ptr[sp.order[q]] <= sh.rank1_max);
    if (chunk > 0) {
        CHECK(sp.recoff.size() == sp.tab.size());
        int64_t g = 0;
        for (size_t e = 0; e < sp.tab.size(); ++e) {
            CHECK(sp.recoff[e] == g);
            g += (sp.tab[e].y + chunk - 1) / chunk * (chunk / 4);
        }
        CHECK(sp.rec_groups == g);
        // the workspace bound the library reserves for the records
        CHECK(4 * sp.rec_groups <= nnz + (int64_t)sp.tab.size() * (chunk - 1) + 4);
    }
}

int main()
{
    std::mt19937_64 rng(12345);
    const int64_t max_pieces = 2048;
    for (int trial = 0; trial < 60; ++trial) {
        const int64_t n = 1 + (int64_t)(rng() % 3000);
        std::vector<int64_t> ptr(n + 1, 0);
        for (int64_t r = 0; r < n; ++r) {
            const int kind = (int)(rng() % 10);
            const int64_t c = kind < 2 ? 0 : kind < 5 ? 1 + (int64_t)(rng() % 3) : kind < 9 ? (int64_t)(rng() % 300)
                                                                             : 1000 + (int64_t)(rng() % 9000);
            ptr[r + 1] = ptr[r] + c;
        }
        for (int K : {10, 32, 64, 128})
            for (int hs : {-1, 0, 1})
                for (int rs : {-1, 0, 1})
                    for (int64_t lim : {-1, 1, 3})
                        for (int64_t hmin : {64, 2048}) {
                            const PlanShape sh{hmin, 64 + (int64_t)(rng() % 1000), lim, hs, rs};
                            const int64_t chunk = K == 64 ? 32 : 64;
                            check_plan(ptr, n, sh, K <= 64, K, max_pieces, (trial & 1) ? chunk : 0);
                        }
    }
    // structure checks
    {
        std::vector<int64_t> ptr = {0, 2, 2, 5};
        std::vector<int32_t> idx = {1, 3, 0, 2, 4};
        std::string why;
        CHECK(check_structure(ptr, idx, 5, why));
        std::vector<int32_t> bad = idx;
        bad[1] = 1;  // duplicate
        CHECK(!check_structure(ptr, bad, 5, why));
        bad = idx;
        bad[4] = 5;  // out of range
        CHECK(!check_structure(ptr, bad, 5, why));
        std::vector<int64_t> dec = {0, 3, 2, 5};
        CHECK(!check_structure(dec, idx, 5, why));
        std::vector<int64_t> past = {0, 2, 2, 6};
        CHECK(!check_structure(past, idx, 5, why));
    }
    // host Cholesky and SPD inverse
    for (int n : {1, 2, 7, 64, 128}) {
        std::normal_distribution<double> nd;
        std::vector<double> X((size_t)n * 2 * n), A((size_t)n * n, 0.0), L, inv;
        for (double &x : X) x = nd(rng);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double s = i == j ? 0.5 : 0.0;
                for (int k = 0; k < 2 * n; ++k) s += X[(size_t)i * 2 * n + k] * X[(size_t)j * 2 * n + k] / (2 * n);
                A[(size_t)i * n + j] = s;
            }
        CHECK(host_cholesky(n, A, L));
        CHECK(host_spd_inverse(n, A, inv));
        double err = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double s = 0.0;
                for (int k = 0; k < n; ++k) s += A[(size_t)i * n + k] * inv[(size_t)k * n + j];
                err = std::max(err, std::fabs(s - (i == j ? 1.0 : 0.0)));
            }
        CHECK(err < 1e-8);
        A[0] = -1.0;
        CHECK(!host_cholesky(n, A, L));
    }
    if (failures) std::fprintf(stderr, "%d checks failed\n", failures);
    else std::printf("plan checks passed\n");
    return failures ? 1 : 0;
}
