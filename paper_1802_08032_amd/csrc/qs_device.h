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

// Streaming kernels move 256 bytes per thread per step (16 complex128 or 32
// complex64 amplitudes) and issue all loads before the first store.  A
// workgroup step of PS = kBlock * per items covers two half-runs of PS/2
// items spaced PS apart, and consecutive loads alternate between them.
// Measured on MI355X for in-place read/write of 64 GiB: ~6.1 TB/s with this
// order, ~5.3-5.6 TB/s for one contiguous run read in order, ~5.2 TB/s for
// runs 128 KiB or more apart, ~5.0 TB/s with 2-4 amplitudes per thread.
template <typename T>
constexpr int kPer = 256 / (2 * (int)sizeof(T));

// First item of workgroup step s; steps 2k and 2k+1 together cover
// [2k PS, (2k+2) PS).
__device__ __forceinline__ uint64_t step_base(uint64_t s, uint64_t ps)
{
    return (s >> 1) * 2 * ps + (s & 1) * (ps / 2);
}

// Item of this thread's j-th element in the step starting at `base`.
__device__ __forceinline__ uint64_t step_item(uint64_t base, int j, uint64_t ps)
{
    return base + (uint64_t)(j & 1) * ps + (uint64_t)(j >> 1) * kBlock + threadIdx.x;
}

template <typename V> struct VecOf;
template <> struct VecOf<double2> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct VecOf<float2> { typedef float type __attribute__((ext_vector_type(2))); };

// Non-temporal load / store of one amplitude (each is touched once per pass).
template <typename V>
__device__ __forceinline__ V ldnt(const V* p)
{
    using E = typename VecOf<V>::type;
    const E e = __builtin_nontemporal_load((const E*)p);
    V v;
    v.x = e.x;
    v.y = e.y;
    return v;
}

template <typename V>
__device__ __forceinline__ void stnt(V* p, V v)
{
    using E = typename VecOf<V>::type;
    E e;
    e.x = v.x;
    e.y = v.y;
    __builtin_nontemporal_store(e, (E*)p);
}
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
