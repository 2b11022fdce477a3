// rng.hpp -- device counter-based draws for the Gibbs sampler.
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as
// easy as 1, 2, 3", SC'11): ten rounds; each round forms the 64-bit products
// of counter words 0 and 2 with two fixed odd multipliers, and the new
// counter is (hi(w2*M1) ^ w1 ^ k0, lo(w2*M1), hi(w0*M0) ^ w3 ^ k1, lo(w0*M0));
// the key is bumped by the two Weyl constants after every round.
//
// Counter assignment (key = the 64-bit seed):
//   row normals     (pair p, row r, half-sweep h, 0): normals 2p and 2p+1 of row r
//   Bartlett normals(q/2, 0, h, 1), mean normals (q/2, 0, h, 2)
//   gamma attempt t of draw k: normal from (t, k, h, 3), uniform from (t, k, h, 4);
//   shape boost uniform (0, k, h, 5)
// Uniforms carry 53 bits: the first word gives the high 32 bits, the top 21
// bits of the second word the rest, offset by half a unit (never 0 or 1).
// Normals come in Box-Muller pairs: radius from the uniform of words (0,1),
// angle from the uniform of words (2,3).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bpmf {

struct u32x4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ u32x4 philox4x32_10(u32x4 c, uint64_t seed)
{
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)c.x * 0xD2511F53u;
        uint64_t p1 = (uint64_t)c.z * 0xCD9E8D57u;
        u32x4 n;
        n.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
        n.y = (uint32_t)p1;
        n.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
        n.w = (uint32_t)p0;
        c = n;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

__device__ __forceinline__ double uniform53(uint32_t hi, uint32_t lo)
{
    uint64_t m = ((uint64_t)hi << 21) | (uint64_t)(lo >> 11);
    return ((double)m + 0.5) * 0x1.0p-53;
}

// The same uniform rounded to FP32 with relative error below 2^-23: the high
// word contributes x * 2^-32 and the remaining 21 bits x * 2^-53.
__device__ __forceinline__ float uniform53_f32(uint32_t hi, uint32_t lo)
{
    float a = (float)hi * 0x1.0p-32f;
    float b = ((float)(lo >> 11) + 0.5f) * 0x1.0p-53f;
    return a + b;
}

__device__ __forceinline__ void box_muller_f64(u32x4 w, double &z0, double &z1)
{
    double u1 = uniform53(w.x, w.y);
    double u2 = uniform53(w.z, w.w);
    double rad = sqrt(-2.0 * log(u1));
    double s, c;
    sincospi(2.0 * u2, &s, &c);
    z0 = rad * c;
    z1 = rad * s;
}

// -log(u) for the 53-bit uniform u of (hi, lo), to a few FP32 ulps over all
// of (0, 1).  Rounding u itself to FP32 costs up to 2^-25 / (1 - u) of
// relative accuracy near u = 1, so for v = 1 - u < 1/8 the series
// -log(u) = sum_k v^k / k is used instead, with v the exact complement (the
// uniform of the inverted 53 bits) rounded to FP32; nine terms leave a
// truncation error below v^9 / 10 < 2^-27 relative.  Both forms are
// evaluated and one is selected, so no lane waits for a branch.
__device__ __forceinline__ float neglog_uniform53_f32(uint32_t hi, uint32_t lo)
{
    const float u = uniform53_f32(hi, lo);
    const float v = uniform53_f32(~hi, ~lo);
    float s = 1.0f / 9.0f;
    s = fmaf(s, v, 1.0f / 8.0f);
    s = fmaf(s, v, 1.0f / 7.0f);
    s = fmaf(s, v, 1.0f / 6.0f);
    s = fmaf(s, v, 1.0f / 5.0f);
    s = fmaf(s, v, 1.0f / 4.0f);
    s = fmaf(s, v, 1.0f / 3.0f);
    s = fmaf(s, v, 0.5f);
    s = fmaf(s, v, 1.0f);
    const float lg = -logf(u);
    return v < 0.125f ? v * s : lg;
}

__device__ __forceinline__ void box_muller_f32(u32x4 w, float &z0, float &z1)
{
    float u2 = uniform53_f32(w.z, w.w);
    float rad = sqrtf(2.0f * neglog_uniform53_f32(w.x, w.y));
    float s, c;
    sincospif(2.0f * u2, &s, &c);
    z0 = rad * c;
    z1 = rad * s;
}

__device__ __forceinline__ u32x4 ctr4(uint32_t a, uint32_t b, uint32_t c, uint32_t d)
{
    u32x4 r;
    r.x = a; r.y = b; r.z = c; r.w = d;
    return r;
}

// Standard normal number q of stream `tag` (1 = Bartlett, 2 = mean) of half-sweep h.
__device__ __forceinline__ double stream_normal_f64(uint64_t seed, uint32_t h, uint32_t tag,
                                                    uint32_t q)
{
    double z0, z1;
    box_muller_f64(philox4x32_10(ctr4(q >> 1, 0u, h, tag), seed), z0, z1);
    return (q & 1u) ? z1 : z0;
}

// Gamma(a, 1) by Marsaglia and Tsang (ACM TOMS 26(3), 2000): with d = a - 1/3
// and c = 1/sqrt(9 d), propose v = (1 + c x)^3 for a standard normal x and
// accept when log u < x^2/2 + d - d v + d log v; for a < 1 use shape a + 1
// and multiply by u^(1/a).  Each attempt uses its own counters, so the draw
// is a pure function of (seed, h, k).
__device__ inline double gamma_mt(uint64_t seed, uint32_t h, uint32_t k, double a)
{
    double boost = 1.0;
    if (a < 1.0) {
        u32x4 w = philox4x32_10(ctr4(0u, k, h, 5u), seed);
        boost = pow(uniform53(w.x, w.y), 1.0 / a);
        a += 1.0;
    }
    const double d = a - 1.0 / 3.0;
    const double c = 1.0 / sqrt(9.0 * d);
    for (uint32_t t = 0; t < 1000000u; ++t) {
        double x, unused;
        box_muller_f64(philox4x32_10(ctr4(t, k, h, 3u), seed), x, unused);
        double v = 1.0 + c * x;
        if (v <= 0.0) continue;
        v = v * v * v;
        u32x4 w = philox4x32_10(ctr4(t, k, h, 4u), seed);
        double u = uniform53(w.x, w.y);
        if (log(u) < 0.5 * x * x + d - d * v + d * log(v)) return boost * d * v;
    }
    return boost * d;  // unreachable in practice (acceptance rate > 95%)
}

}  // namespace bpmf
