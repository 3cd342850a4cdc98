// Device-side helpers shared by the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qs_internal.h"

namespace qs {

template <typename T> struct C2;
template <> struct C2<double> { using type = double2; };
template <> struct C2<float> { using type = float2; };

constexpr int kBlock = 256;
// 16 resident blocks of 4 waves per CU on 256 CUs: every grid-stride kernel
// is capped here so that each CU holds a fixed share of the waves.
constexpr uint64_t kMaxGrid = 256 * 16;

inline int grid_for(uint64_t items, int items_per_thread)
{
    const uint64_t per_block = (uint64_t)kBlock * items_per_thread;
    uint64_t blocks = (items + per_block - 1) / per_block;
    if (blocks < 1) blocks = 1;
    if (blocks > kMaxGrid) blocks = kMaxGrid;
    return (int)blocks;
}

// Insert the bits listed in `b` (ascending final positions) into i; the
// inserted bits take the values of b.ones.
__device__ __forceinline__ uint64_t expand(uint64_t i, const BitInsert& b)
{
    for (int k = 0; k < b.count; ++k) {
        const int p = b.pos[k];
        const uint64_t lo = i & ((1ull << p) - 1ull);
        i = ((i >> p) << (p + 1)) | lo;
    }
    return i | b.ones;
}

// out = a * x + b * y for complex a, b (interleaved re/im in T[2]).
template <typename T, typename V>
__device__ __forceinline__ V cmac2(T ar, T ai, V x, T br, T bi, V y)
{
    V r;
    r.x = ar * x.x - ai * x.y + br * y.x - bi * y.y;
    r.y = ar * x.y + ai * x.x + br * y.y + bi * y.x;
    return r;
}

template <typename T, typename V>
__device__ __forceinline__ V cmul(T ar, T ai, V x)
{
    V r;
    r.x = ar * x.x - ai * x.y;
    r.y = ar * x.y + ai * x.x;
    return r;
}

// (x, y) <- U (x, y) with U row-major interleaved in m[8].
template <typename T, typename V>
__device__ __forceinline__ void apply2(const T* m, V& x, V& y)
{
    const V nx = cmac2<T, V>(m[0], m[1], x, m[2], m[3], y);
    const V ny = cmac2<T, V>(m[4], m[5], x, m[6], m[7], y);
    x = nx;
    y = ny;
}

// Neumaier accumulator in double.
struct NSum {
    double s, c;
};

__device__ __forceinline__ void nadd(NSum& a, double v)
{
    const double t = a.s + v;
    a.c += (fabs(a.s) >= fabs(v)) ? ((a.s - t) + v) : ((v - t) + a.s);
    a.s = t;
}

// Merge two compensated sums (Knuth TwoSum on the leading parts).
__device__ __forceinline__ NSum nmerge(NSum a, NSum b)
{
    const double t = a.s + b.s;
    const double bb = t - a.s;
    const double e = (a.s - (t - bb)) + (b.s - bb);
    NSum r;
    r.s = t;
    r.c = a.c + b.c + e;
    return r;
}

}  // namespace qs
