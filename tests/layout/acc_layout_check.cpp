// The Normal-Wishart step writes Lambda / alpha through lambda_acc_index; the
// K <= 64 row kernel reads accumulator element i of lane l as the entry the
// matrix cores leave there.  This checks, on the CPU, that the two agree for
// both layouts and that the writer's map covers every slot exactly once.
#include "common.hpp"

#include <cstdio>
#include <vector>

using bpmf::lambda_acc_index;

// entry (r, c) of accumulator element i of lane l, as the row kernel holds it
static void element_entry(bool g16, int i, int l, int &r, int &c)
{
    if (g16) {
        // ten lower 16 x 16 tiles, t = a (a + 1) / 2 + b; element 4 t + v of
        // lane l: (16 a + 4 (l / 16) + v, 16 b + l % 16)
        const int t = i / 4, v = i % 4;
        int a = 0;
        while ((a + 1) * (a + 2) / 2 <= t) ++a;
        const int b = t - a * (a + 1) / 2;
        r = 16 * a + 4 * (l / 16) + v;
        c = 16 * b + l % 16;
    } else {
        // lower 32 x 32 tiles (0,0), (1,0), (1,1); element 16 t + e of lane l:
        // (32 ta + 8 (e / 4) + 4 (l / 32) + e % 4, 32 tb + l % 32)
        const int t = i / 16, e = i % 16;
        const int ta = t == 0 ? 0 : 1, tb = t == 2 ? 1 : 0;
        r = 32 * ta + 8 * (e / 4) + 4 * (l / 32) + e % 4;
        c = 32 * tb + l % 32;
    }
}

int main()
{
    int bad = 0;
    for (int g = 0; g < 2; ++g) {
        const bool g16 = g == 1;
        const int n = g16 ? 40 : 48, slots = n * 64;
        std::vector<int> hits(slots, 0);
        int mapped = 0;
        for (int r = 0; r < 64; ++r)
            for (int c = 0; c < 64; ++c) {
                const int q = lambda_acc_index(r, c, g16);
                const bool upper_tile = g16 ? (r >> 4) < (c >> 4) : (r >> 5) < (c >> 5);
                if (upper_tile != (q < 0)) {
                    std::printf("g16=%d (%d,%d): index %d for %s tile\n", g, r, c, q, upper_tile ? "an upper" : "a lower");
                    ++bad;
                }
                if (q < 0) continue;
                if (q >= slots) {
                    std::printf("g16=%d (%d,%d): index %d out of range\n", g, r, c, q);
                    ++bad;
                    continue;
                }
                ++hits[q];
                ++mapped;
            }
        for (int q = 0; q < slots; ++q)
            if (hits[q] != 1) {
                std::printf("g16=%d slot %d written %d times\n", g, q, hits[q]);
                ++bad;
            }
        for (int i = 0; i < n; ++i)
            for (int l = 0; l < 64; ++l) {
                int r, c;
                element_entry(g16, i, l, r, c);
                if (lambda_acc_index(r, c, g16) != i * 64 + l) {
                    std::printf("g16=%d element %d lane %d: entry (%d,%d) maps to %d\n", g, i, l, r, c,
                                lambda_acc_index(r, c, g16));
                    ++bad;
                }
            }
        std::printf("g16=%d: %d entries on %d slots\n", g, mapped, slots);
    }
    if (bad) {
        std::printf("%d layout mismatches\n", bad);
        return 1;
    }
    std::printf("layout checks passed\n");
    return 0;
}
