// Host-only stand-in for the HIP runtime header: just enough for the layout
// helpers of csrc/common.hpp to compile as plain C++ for a CPU check (no
// kernel is compiled or run).
#pragma once
#include <cstdint>
#include <cstring>
#define __host__
#define __device__
#define __global__
#define __forceinline__ inline
typedef int hipError_t;
typedef void *hipStream_t;
struct int4 { int x, y, z, w; };
struct uint4 { unsigned x, y, z, w; };
struct int2 { int x, y; };
struct float4 { float x, y, z, w; };
inline float __uint_as_float(uint32_t u) { float f; std::memcpy(&f, &u, 4); return f; }
inline uint32_t __float_as_uint(float f) { uint32_t u; std::memcpy(&u, &f, 4); return u; }
