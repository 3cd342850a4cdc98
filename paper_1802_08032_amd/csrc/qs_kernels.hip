// gfx950 kernels for one operation per pass: the amplitude-pair update of
// Eq. 1 (Sec. II.B.1) for state vectors, the 4-element group update that
// fuses the two passes of Eq. 2 for density matrices, the channel updates,
// probability reductions and measurement collapse.
//
// Layout: interleaved complex (double2 / float2), qubit q = bit q of the
// index.  Every kernel loops over 64-bit indices with a grid capped at 16
// blocks per CU; the streaming kernels take kPer amplitudes per thread per
// step (see qs_device.h).
#include <algorithm>

#include "qs_device.h"

namespace qs {

BitInsert make_insert(const int* positions, int count, uint64_t ones)
{
    BitInsert b;
    b.count = count;
    int tmp[64];
    for (int k = 0; k < count; ++k) tmp[k] = positions[k];
    std::sort(tmp, tmp + count);
    for (int k = 0; k < count; ++k) b.pos[k] = tmp[k];
    b.ones = ones;
    return b;
}

namespace {

// ---------------------------------------------------------------------------
// Initialisation: every amplitude 0 except `index`, which is (re, im).
template <typename T, int U>
__global__ __launch_bounds__(kBlock) void k_init_basis(typename C2<T>::type* __restrict__ amp,
                                                       uint64_t len, uint64_t index, T re, T im)
{
    using V = typename C2<T>::type;
    static_assert(U % 2 == 0, "the step order alternates two half-runs");
    const uint64_t ps = (uint64_t)kBlock * U;
    for (uint64_t s = blockIdx.x; step_base(s, ps) < len; s += gridDim.x) {
        const uint64_t c = step_base(s, ps);
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint64_t i = step_item(c, j, ps);
            if (i >= len) continue;
            V v;  // plain stores: measured faster than non-temporal ones for write-only streams
            v.x = (i == index) ? re : T(0);
            v.y = (i == index) ? im : T(0);
            amp[i] = v;
        }
    }
}

// ---------------------------------------------------------------------------
// Eq. 1 pair update for targets whose pair partner lies in another wavefront
// row (t >= 6): each lane owns a pair (a, a + 2^t); 64 consecutive lanes
// touch two contiguous 1 KiB (c128) runs.  `ins` inserts a 0 at t and a 1
// at every control of at least kLineBits; lower controls are the bits of
// `lowmask`, tested per pair.
template <typename T, int P>
__global__ __launch_bounds__(kBlock) void k_gate_pair(typename C2<T>::type* __restrict__ amp,
                                                      uint64_t npairs, uint64_t tb, BitInsert ins,
                                                      uint64_t lowmask, Mat2<T> u)
{
    using V = typename C2<T>::type;
    static_assert(P % 2 == 0, "the step order alternates two half-runs");
    const uint64_t ps = (uint64_t)kBlock * P;
    for (uint64_t s = blockIdx.x; step_base(s, ps) < npairs; s += gridDim.x) {
        const uint64_t c = step_base(s, ps);
        uint64_t a[P];
        V x[P], y[P];
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const uint64_t i = step_item(c, j, ps);
            a[j] = expand(i < npairs ? i : npairs - 1, ins);  // a clamped lane only reads
        }
        // all low halves, then all high halves: each run of loads alternates
        // between the step's two half-runs
#pragma unroll
        for (int j = 0; j < P; ++j) x[j] = ldnt(amp + a[j]);
#pragma unroll
        for (int j = 0; j < P; ++j) y[j] = ldnt(amp + a[j] + tb);
#pragma unroll
        for (int j = 0; j < P; ++j) {
            // controls below the line size are tested per pair: unselected
            // pairs are written back unchanged, so every store is a full line
            V nx = x[j], ny = y[j];
            apply2<T, V>(u.m, nx, ny);
            const bool ok = (a[j] & lowmask) == lowmask;
            // component-wise selects: a select of whole vector structs puts
            // the arrays in scratch memory
            x[j].x = ok ? nx.x : x[j].x;
            x[j].y = ok ? nx.y : x[j].y;
            y[j].x = ok ? ny.x : y[j].x;
            y[j].y = ok ? ny.y : y[j].y;
        }
#pragma unroll
        for (int j = 0; j < P; ++j)
            if (step_item(c, j, ps) < npairs) stnt(amp + a[j], x[j]);
#pragma unroll
        for (int j = 0; j < P; ++j)
            if (step_item(c, j, ps) < npairs) stnt(amp + a[j] + tb, y[j]);
    }
}

// Cross-lane exchange with lane ^ 2^TT inside a wavefront of 64 lanes:
// DPP quad permutes for 1 and 2, ds_swizzle bit mode for 4, 8, 16 and a
// backwards permute for 32.  All lanes must be active.
template <int TT>
__device__ __forceinline__ int lane_xor(int v, int lane)
{
    if constexpr (TT == 0) return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);
    else if constexpr (TT == 1) return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);
    else if constexpr (TT == 2) return __builtin_amdgcn_ds_swizzle(v, 0x101F);
    else if constexpr (TT == 3) return __builtin_amdgcn_ds_swizzle(v, 0x201F);
    else if constexpr (TT == 4) return __builtin_amdgcn_ds_swizzle(v, 0x401F);
    else return __builtin_amdgcn_ds_bpermute((lane ^ 32) << 2, v);
}

template <int TT>
__device__ __forceinline__ double xchg(double v, int lane)
{
    const long long b = __double_as_longlong(v);
    const int lo = lane_xor<TT>((int)(b & 0xffffffffll), lane);
    const int hi = lane_xor<TT>((int)(b >> 32), lane);
    return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}

template <int TT>
__device__ __forceinline__ float xchg(float v, int lane)
{
    return __int_as_float(lane_xor<TT>(__float_as_int(v), lane));
}

// Eq. 1 for targets t < 6: each lane loads ONE amplitude of a contiguous
// 64-amplitude chunk, fetches its pair partner from lane ^ 2^t in registers
// and writes its own new value, so loads and stores stay fully contiguous.
// Controls at bits >= 6 are folded into the chunk index (`hi`); controls at
// bits < 6 become a lane mask.
template <typename T, int TT, int U>
__global__ __launch_bounds__(kBlock) void k_gate_low(typename C2<T>::type* __restrict__ amp,
                                                     uint64_t nchunks, BitInsert hi,
                                                     uint32_t lowmask, Mat2<T> u)
{
    static_assert(U % 2 == 0, "the step order alternates two half-runs");
    using V = typename C2<T>::type;
    const int lane = threadIdx.x & 63;
    const bool up = (lane >> TT) & 1;
    const bool ok = ((uint32_t)lane & lowmask) == lowmask;
    // A lane whose controls at or above the 128-byte line are not all set
    // holds a whole line the gate leaves unchanged: it loads and stores
    // nothing.  Its pair partner (lane ^ 2^TT; the target is never a
    // control) has the same control bits, so no active lane reads it.
    constexpr uint32_t kLine = sizeof(T) == 8 ? 3 : 4;
    const uint32_t linemask = lowmask & ~((1u << kLine) - 1);
    const bool act = ((uint32_t)lane & linemask) == linemask;
    // new = s * self + p * partner
    const T sr = up ? u.m[6] : u.m[0], si = up ? u.m[7] : u.m[1];
    const T pr = up ? u.m[4] : u.m[2], pi = up ? u.m[5] : u.m[3];
    // chunks play the role of items: a workgroup step of PS = 4 * kPer
    // chunks is two half-runs PS apart, alternated as in step_item (with
    // the 4 waves in place of the threads)
    const int w = threadIdx.x >> 6;
    const uint64_t ps = (uint64_t)(kBlock / 64) * U;
    auto chunk = [&](uint64_t base, int j) {
        return base + (uint64_t)(j & 1) * ps + (uint64_t)(j >> 1) * (kBlock / 64) + w;
    };
    for (uint64_t s = blockIdx.x; step_base(s, ps) < nchunks; s += gridDim.x) {
        const uint64_t c0 = step_base(s, ps);
        V v[U];
        uint64_t e[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint64_t c = chunk(c0, j);
            e[j] = (expand(c < nchunks ? c : nchunks - 1, hi) << 6) | (uint64_t)lane;
            v[j].x = T(0);
            v[j].y = T(0);
            if (act) v[j] = ldnt(amp + e[j]);
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            // the chunk test is uniform over the wave, so every lane joins the exchange
            V p;
            p.x = xchg<TT>(v[j].x, lane);
            p.y = xchg<TT>(v[j].y, lane);
            const V r = cmac2<T, V>(sr, si, v[j], pr, pi, p);
            // active lanes whose controls below the line are not all set
            // store their value unchanged, so that every store covers whole
            // lines
            V o;
            o.x = ok ? r.x : v[j].x;
            o.y = ok ? r.y : v[j].y;
            if (act && chunk(c0, j) < nchunks) stnt(amp + e[j], o);
        }
    }
}

// Multi-controlled NOT: swap each pair whose controls are set (controls
// below kLineBits tested per pair, as in k_gate_pair).
template <typename T, int P>
__global__ __launch_bounds__(kBlock) void k_not(typename C2<T>::type* __restrict__ amp,
                                                uint64_t npairs, uint64_t tb, BitInsert ins, uint64_t lowmask)
{
    using V = typename C2<T>::type;
    static_assert(P % 2 == 0, "the step order alternates two half-runs");
    const uint64_t ps = (uint64_t)kBlock * P;
    for (uint64_t s = blockIdx.x; step_base(s, ps) < npairs; s += gridDim.x) {
        const uint64_t c = step_base(s, ps);
        uint64_t a[P];
        V x[P], y[P];
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const uint64_t i = step_item(c, j, ps);
            a[j] = expand(i < npairs ? i : npairs - 1, ins);  // a clamped lane only reads
        }
        // all low halves, then all high halves: each run of loads alternates
        // between the step's two half-runs
#pragma unroll
        for (int j = 0; j < P; ++j) x[j] = ldnt(amp + a[j]);
#pragma unroll
        for (int j = 0; j < P; ++j) y[j] = ldnt(amp + a[j] + tb);
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const bool ok = (a[j] & lowmask) == lowmask;  // unselected pairs keep their order
            const T x0 = x[j].x, x1 = x[j].y;
            x[j].x = ok ? y[j].x : x0;
            x[j].y = ok ? y[j].y : x1;
            y[j].x = ok ? x0 : y[j].x;
            y[j].y = ok ? x1 : y[j].y;
        }
#pragma unroll
        for (int j = 0; j < P; ++j)
            if (step_item(c, j, ps) < npairs) stnt(amp + a[j], x[j]);
#pragma unroll
        for (int j = 0; j < P; ++j)
            if (step_item(c, j, ps) < npairs) stnt(amp + a[j] + tb, y[j]);
    }
}

// Diagonal phase on the amplitudes whose `ins.ones` bits are all set,
// except those that also have every bit of `skip` set (skip != 0).
template <typename T, int U>
__global__ __launch_bounds__(kBlock) void k_phase(typename C2<T>::type* __restrict__ amp,
                                                  uint64_t count, BitInsert ins, uint64_t lowmask,
                                                  uint64_t skip, T fr, T fi)
{
    static_assert(U % 2 == 0, "the step order alternates two half-runs");
    using V = typename C2<T>::type;
    const uint64_t ps = (uint64_t)kBlock * U;
    for (uint64_t s = blockIdx.x; step_base(s, ps) < count; s += gridDim.x) {
        const uint64_t c = step_base(s, ps);
        uint64_t e[U];
        bool on[U];
        V v[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint64_t i = step_item(c, j, ps);
            e[j] = expand(i < count ? i : count - 1, ins);
            on[j] = i < count;
            if (on[j]) v[j] = ldnt(amp + e[j]);
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            if (!on[j]) continue;
            // phase bits below kLineBits are tested per element; the others
            // are written back unchanged so that every store is a full line
            const bool hit = (e[j] & lowmask) == lowmask && !(skip != 0 && (e[j] & skip) == skip);
            const V m = cmul<T, V>(fr, fi, v[j]);
            V r;
            r.x = hit ? m.x : v[j].x;
            r.y = hit ? m.y : v[j].y;
            stnt(amp + e[j], r);
        }
    }
}

// ---------------------------------------------------------------------------
// Density matrix, Eq. 2 fused into one pass.  A group is the four entries
// (rho[r][c]) with row bit t = r and column bit t+N = c; the gate is
// rho -> (R ? U : I) rho (C ? U^dagger : I), R / C = row / column controls
// all set.  Columns multiplied by U^dagger is conj(U) on the column qubit.
template <typename T, int G>
__global__ __launch_bounds__(kBlock) void k_dm_gate(typename C2<T>::type* __restrict__ rho,
                                                    uint64_t ngroups, uint64_t tb, uint64_t cb,
                                                    BitInsert ins, uint64_t rmask, uint64_t cmask,
                                                    Mat2<T> u)
{
    using V = typename C2<T>::type;
    T uc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) uc[k] = (k & 1) ? -u.m[k] : u.m[k];
    static_assert(G % 2 == 0, "the step order alternates two half-runs");
    const uint64_t ps = (uint64_t)kBlock * G;
    for (uint64_t s = blockIdx.x; step_base(s, ps) < ngroups; s += gridDim.x) {
        const uint64_t c = step_base(s, ps);
        uint64_t b[G];
        bool R[G], Cc[G];
        V m00[G], m10[G], m01[G], m11[G];
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const uint64_t g = step_item(c, j, ps);
            b[j] = expand(g < ngroups ? g : ngroups - 1, ins);
            R[j] = g < ngroups && (b[j] & rmask) == rmask;
            Cc[j] = g < ngroups && (b[j] & cmask) == cmask;
            if (R[j] || Cc[j]) {
                m00[j] = ldnt(rho + b[j]);
                m10[j] = ldnt(rho + b[j] + tb);
                m01[j] = ldnt(rho + b[j] + cb);
                m11[j] = ldnt(rho + b[j] + tb + cb);
            }
        }
#pragma unroll
        for (int j = 0; j < G; ++j) {
            if (!R[j] && !Cc[j]) continue;
            if (R[j]) {  // U on the row index, for each column
                apply2<T, V>(u.m, m00[j], m10[j]);
                apply2<T, V>(u.m, m01[j], m11[j]);
            }
            if (Cc[j]) {  // conj(U) on the column index, for each row
                apply2<T, V>(uc, m00[j], m01[j]);
                apply2<T, V>(uc, m10[j], m11[j]);
            }
            stnt(rho + b[j], m00[j]);
            stnt(rho + b[j] + tb, m10[j]);
            stnt(rho + b[j] + cb, m01[j]);
            stnt(rho + b[j] + tb + cb, m11[j]);
        }
    }
}

// Channel closed forms on each 4-group (arithmetic in double).
//   dephasing p:     off-diagonals * (1 - 2p)
//   depolarising p:  r00 <- (1-2p/3) r00 + (2p/3) r11, r11 symmetric,
//                    off-diagonals * (1 - 4p/3)
//   damping g:       r00 <- r00 + g r11, r11 <- (1-g) r11,
//                    off-diagonals * sqrt(1-g)
// a, b: diagonal mixing (r00' = a r00 + b r11 ... per channel), f: off-diagonal factor.
template <typename T, int CH, int G>
__global__ __launch_bounds__(kBlock) void k_dm_channel(typename C2<T>::type* __restrict__ rho,
                                                       uint64_t ngroups, uint64_t tb, uint64_t cb,
                                                       BitInsert ins, double p0, double p1, double f)
{
    using V = typename C2<T>::type;
    static_assert(G % 2 == 0, "the step order alternates two half-runs");
    const uint64_t ps = (uint64_t)kBlock * G;
    for (uint64_t s = blockIdx.x; step_base(s, ps) < ngroups; s += gridDim.x) {
        const uint64_t c = step_base(s, ps);
        uint64_t b[G];
        V m00[G], m10[G], m01[G], m11[G];
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const uint64_t g = step_item(c, j, ps);
            b[j] = expand(g < ngroups ? g : ngroups - 1, ins);
            m10[j] = ldnt(rho + b[j] + tb);
            m01[j] = ldnt(rho + b[j] + cb);
            if constexpr (CH != QS_DEPHASING) {
                m00[j] = ldnt(rho + b[j]);
                m11[j] = ldnt(rho + b[j] + tb + cb);
            }
        }
#pragma unroll
        for (int j = 0; j < G; ++j) {
            if (step_item(c, j, ps) >= ngroups) continue;
            V n10, n01;
            n10.x = (T)(f * (double)m10[j].x);
            n10.y = (T)(f * (double)m10[j].y);
            n01.x = (T)(f * (double)m01[j].x);
            n01.y = (T)(f * (double)m01[j].y);
            stnt(rho + b[j] + tb, n10);
            stnt(rho + b[j] + cb, n01);
            if constexpr (CH != QS_DEPHASING) {
                const double a0 = m00[j].x, a1 = m00[j].y, d0 = m11[j].x, d1 = m11[j].y;
                V n00, n11;
                if constexpr (CH == QS_DEPOLARISING) {  // p0 = 1 - 2p/3, p1 = 2p/3
                    n00.x = (T)(p0 * a0 + p1 * d0);
                    n00.y = (T)(p0 * a1 + p1 * d1);
                    n11.x = (T)(p0 * d0 + p1 * a0);
                    n11.y = (T)(p0 * d1 + p1 * a1);
                } else {  // damping: p0 = gamma, p1 = 1 - gamma
                    n00.x = (T)(a0 + p0 * d0);
                    n00.y = (T)(a1 + p0 * d1);
                    n11.x = (T)(p1 * d0);
                    n11.y = (T)(p1 * d1);
                }
                stnt(rho + b[j], n00);
                stnt(rho + b[j] + tb + cb, n11);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Reductions: per-thread Neumaier sums in double, merged across the wave
// with cross-lane shuffles and across the block through LDS; one partial
// per block, folded by k_reduce_final.
__device__ __forceinline__ NSum wave_merge(NSum a)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        NSum o;
        o.s = __shfl_xor(a.s, off, 64);
        o.c = __shfl_xor(a.c, off, 64);
        a = nmerge(a, o);
    }
    return a;
}

__device__ __forceinline__ void block_store2(NSum s0, NSum s1, double* partials)
{
    __shared__ double sh[4][kBlock / 64];
    s0 = wave_merge(s0);
    s1 = wave_merge(s1);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[0][w] = s0.s;
        sh[1][w] = s0.c;
        sh[2][w] = s1.s;
        sh[3][w] = s1.c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        NSum a = {sh[0][0], sh[1][0]}, b = {sh[2][0], sh[3][0]};
        for (int k = 1; k < kBlock / 64; ++k) {
            a = nmerge(a, NSum{sh[0][k], sh[1][k]});
            b = nmerge(b, NSum{sh[2][k], sh[3][k]});
        }
        partials[4 * blockIdx.x + 0] = a.s;
        partials[4 * blockIdx.x + 1] = a.c;
        partials[4 * blockIdx.x + 2] = b.s;
        partials[4 * blockIdx.x + 3] = b.c;
    }
}

// Sum |alpha_i|^2 split by bit q of i (q < 0: everything in the first sum).
template <typename T, int U>
__global__ __launch_bounds__(kBlock) void k_prob_sv(const typename C2<T>::type* __restrict__ amp,
                                                    uint64_t len, int q, double* partials)
{
    static_assert(U % 2 == 0, "the step order alternates two half-runs");
    using V = typename C2<T>::type;
    NSum s0 = {0.0, 0.0}, s1 = {0.0, 0.0};
    const uint64_t ps = (uint64_t)kBlock * U;
    for (uint64_t s = blockIdx.x; step_base(s, ps) < len; s += gridDim.x) {
        const uint64_t c = step_base(s, ps);
        V v[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint64_t i = step_item(c, j, ps);
            v[j] = ldnt(amp + (i < len ? i : len - 1));
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint64_t i = step_item(c, j, ps);
            const double p = i < len ? (double)v[j].x * (double)v[j].x + (double)v[j].y * (double)v[j].y : 0.0;
            const bool one = (q >= 0) && ((i >> q) & 1);
            nadd(s0, one ? 0.0 : p);
            nadd(s1, one ? p : 0.0);
        }
    }
    block_store2(s0, s1, partials);
}

// Sum |alpha_i|^2 over the indices i whose bit q equals o, reading only
// those: item k stands for k with bit o inserted at position q.  With q at
// or above the line bits every 128-byte line lies in one half, so half the
// state is read.
template <typename T, int U>
__global__ __launch_bounds__(kBlock) void k_prob_half_sv(const typename C2<T>::type* __restrict__ amp,
                                                         uint64_t half, int q, int o, double* partials)
{
    static_assert(U % 2 == 0, "the step order alternates two half-runs");
    using V = typename C2<T>::type;
    NSum s0 = {0.0, 0.0}, s1 = {0.0, 0.0};
    const uint64_t ps = (uint64_t)kBlock * U;
    const uint64_t low = (1ull << q) - 1, bit = (uint64_t)o << q;
    for (uint64_t s = blockIdx.x; step_base(s, ps) < half; s += gridDim.x) {
        const uint64_t c = step_base(s, ps);
        V v[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint64_t k0 = step_item(c, j, ps);
            const uint64_t k = k0 < half ? k0 : half - 1;
            v[j] = ldnt(amp + (((k & ~low) << 1) | bit | (k & low)));
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const double p = step_item(c, j, ps) < half
                                 ? (double)v[j].x * (double)v[j].x + (double)v[j].y * (double)v[j].y
                                 : 0.0;
            nadd(s0, p);
        }
    }
    block_store2(s0, s1, partials);
}

// Sum Re rho[j][j] split by bit q of j (the diagonal is entry j (2^N + 1)).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_prob_dm(const typename C2<T>::type* __restrict__ rho,
                                                    uint64_t dim, int q, double* partials)
{
    NSum s0 = {0.0, 0.0}, s1 = {0.0, 0.0};
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t j = (uint64_t)blockIdx.x * kBlock + threadIdx.x; j < dim; j += stride) {
        const double p = (double)rho[j * (dim + 1)].x;
        const bool one = (q >= 0) && ((j >> q) & 1);
        nadd(s0, one ? 0.0 : p);
        nadd(s1, one ? p : 0.0);
    }
    block_store2(s0, s1, partials);
}

// out[j] = sum over rows i of part[i * cols + j], in row order (one thread
// per column, compensated): the fused readouts' per-workgroup sums.
__global__ __launch_bounds__(64) void k_sum_columns(const double* __restrict__ part, int rows, int cols,
                                                    double* __restrict__ out)
{
    const int j = blockIdx.x * 64 + threadIdx.x;
    if (j >= cols) return;
    NSum a = {0.0, 0.0};
    for (int i = 0; i < rows; ++i) nadd(a, part[(size_t)i * cols + j]);
    out[j] = a.s + a.c;
}

__global__ __launch_bounds__(kBlock) void k_reduce_final(const double* __restrict__ partials,
                                                         int nblocks, double* out)
{
    NSum s0 = {0.0, 0.0}, s1 = {0.0, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += kBlock) {
        s0 = nmerge(s0, NSum{partials[4 * b + 0], partials[4 * b + 1]});
        s1 = nmerge(s1, NSum{partials[4 * b + 2], partials[4 * b + 3]});
    }
    __shared__ double tmp[4 * 4];
    s0 = wave_merge(s0);
    s1 = wave_merge(s1);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        tmp[4 * w + 0] = s0.s;
        tmp[4 * w + 1] = s0.c;
        tmp[4 * w + 2] = s1.s;
        tmp[4 * w + 3] = s1.c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        NSum a = {tmp[0], tmp[1]}, b = {tmp[2], tmp[3]};
        for (int k = 1; k < kBlock / 64; ++k) {
            a = nmerge(a, NSum{tmp[4 * k + 0], tmp[4 * k + 1]});
            b = nmerge(b, NSum{tmp[4 * k + 2], tmp[4 * k + 3]});
        }
        out[0] = a.s + a.c;
        out[1] = b.s + b.c;
    }
}

// Collapse: keep amplitudes with bit q == outcome (scaled in double), zero
// the rest without reading them.
template <typename T, int U>
__global__ __launch_bounds__(kBlock) void k_collapse_sv(typename C2<T>::type* __restrict__ amp,
                                                        uint64_t len, int q, int outcome, double scale)
{
    static_assert(U % 2 == 0, "the step order alternates two half-runs");
    using V = typename C2<T>::type;
    const uint64_t ps = (uint64_t)kBlock * U;
    for (uint64_t s = blockIdx.x; step_base(s, ps) < len; s += gridDim.x) {
        const uint64_t c = step_base(s, ps);
        V v[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint64_t i = step_item(c, j, ps);
            v[j].x = T(0);
            v[j].y = T(0);
            if (i < len && (int)((i >> q) & 1) == outcome) v[j] = ldnt(amp + i);
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint64_t i = step_item(c, j, ps);
            if (i >= len) continue;
            V r;
            r.x = (T)(scale * (double)v[j].x);
            r.y = (T)(scale * (double)v[j].y);
            stnt(amp + i, r);
        }
    }
}

// Density-matrix collapse: keep rho[j][k] when bit q of j and of k both
// equal the outcome (bits q and q+N of the vector index), scaled by 1/p.
template <typename T, int U>
__global__ __launch_bounds__(kBlock) void k_collapse_dm(typename C2<T>::type* __restrict__ rho,
                                                        uint64_t len, int q, int N, int outcome,
                                                        double scale)
{
    static_assert(U % 2 == 0, "the step order alternates two half-runs");
    using V = typename C2<T>::type;
    const uint64_t ps = (uint64_t)kBlock * U;
    for (uint64_t s = blockIdx.x; step_base(s, ps) < len; s += gridDim.x) {
        const uint64_t c = step_base(s, ps);
        V v[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint64_t i = step_item(c, j, ps);
            v[j].x = T(0);
            v[j].y = T(0);
            const bool keep = (int)((i >> q) & 1) == outcome && (int)((i >> (q + N)) & 1) == outcome;
            if (i < len && keep) v[j] = ldnt(rho + i);
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint64_t i = step_item(c, j, ps);
            if (i >= len) continue;
            V r;
            r.x = (T)(scale * (double)v[j].x);
            r.y = (T)(scale * (double)v[j].y);
            stnt(rho + i, r);
        }
    }
}

// ---------------------------------------------------------------------------
// Measure-all.  The items j < count of a subspace sit at index
// fixed + (j << shift); item j falls in bin j mod 2^mbits (mbits <= 10).
// Each block writes 2^mbits Neumaier partials (sum, compensation) of
// |alpha|^2.  Steps are multiples of 1024 items, so with the alternating
// step order the thread's j-th element lies in bin ((j >> 1) & 3) * kBlock +
// tid (mod 2^mbits): four accumulators per thread, folded through LDS.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_hist_sv(const typename C2<T>::type* __restrict__ amp,
                                                    uint64_t count, int shift, uint64_t fixed, int mbits,
                                                    double* __restrict__ partials)
{
    using V = typename C2<T>::type;
    constexpr int U = kPer<T>;
    static_assert((kBlock * U / 2) % 1024 == 0, "steps must be whole multiples of 1024 bins");
    __shared__ double ls[4 * kBlock], lc[4 * kBlock];
    NSum acc[4] = {};
    const uint64_t ps = (uint64_t)kBlock * U;
    for (uint64_t s = blockIdx.x; step_base(s, ps) < count; s += gridDim.x) {
        const uint64_t c = step_base(s, ps);
        V v[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint64_t item = step_item(c, j, ps);
            v[j] = ldnt(amp + (fixed + ((item < count ? item : count - 1) << shift)));
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const double p = step_item(c, j, ps) < count
                                 ? (double)v[j].x * (double)v[j].x + (double)v[j].y * (double)v[j].y
                                 : 0.0;
            nadd(acc[(j >> 1) & 3], p);
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        ls[k * kBlock + threadIdx.x] = acc[k].s;
        lc[k * kBlock + threadIdx.x] = acc[k].c;
    }
    __syncthreads();
    const int nb = 1 << mbits;
    for (int b = threadIdx.x; b < nb; b += kBlock) {
        NSum a = {0.0, 0.0};
        for (int e = b; e < 4 * kBlock; e += nb) a = nmerge(a, NSum{ls[e], lc[e]});
        partials[2 * ((uint64_t)blockIdx.x * nb + b)] = a.s;
        partials[2 * ((uint64_t)blockIdx.x * nb + b) + 1] = a.c;
    }
}

// Fold the per-block partials of each bin; out[2b], out[2b+1] = (sum, compensation).
__global__ __launch_bounds__(kBlock) void k_hist_final(const double* __restrict__ partials, int nblocks,
                                                       int nb, double* __restrict__ out)
{
    const int b = blockIdx.x * kBlock + threadIdx.x;
    if (b >= nb) return;
    NSum a = {0.0, 0.0};
    for (int k = 0; k < nblocks; ++k)
        a = nmerge(a, NSum{partials[2 * ((uint64_t)k * nb + b)], partials[2 * ((uint64_t)k * nb + b) + 1]});
    out[2 * b] = a.s;
    out[2 * b + 1] = a.c;
}

// Real parts of the diagonal rho[j][j] (entry j (2^N + 1) of the vector).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_diag_dm(const typename C2<T>::type* __restrict__ rho, uint64_t dim,
                                                    double* __restrict__ out)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t j = (uint64_t)blockIdx.x * kBlock + threadIdx.x; j < dim; j += stride)
        out[j] = (double)rho[j * (dim + 1)].x;
}

// ---------------------------------------------------------------------------
// k-qubit groups.  Eq. 1 and the Eq. 2 identity hold for gates on several
// qubits (Sec. II.B.1): a group is the D = 2^k amplitudes that agree on
// every bit outside the target set, member r at base + the sum of
// tbit[j] = 2^targets[j] over the set bits j of r; the group is replaced by
// m times it (m: D x D complex, row-major, interleaved, read with uniform
// loads).  `ins` inserts a 0 at every target and a 1 at every control.  One
// thread holds one group and writes each output row as soon as it is formed
// (all D inputs are already in registers).
template <int K>
struct GroupBits {
    uint64_t tbit[K];
};

template <int K>
__device__ __forceinline__ uint64_t group_off(const GroupBits<K>& gb, int r)
{
    uint64_t o = 0;
#pragma unroll
    for (int j = 0; j < K; ++j)
        if ((r >> j) & 1) o += gb.tbit[j];
    return o;
}

template <typename T, int K>
__global__ __launch_bounds__(kBlock) void k_group_gate(typename C2<T>::type* __restrict__ amp,
                                                       uint64_t ngroups, BitInsert ins, GroupBits<K> gb,
                                                       const T* __restrict__ m)
{
    using V = typename C2<T>::type;
    constexpr int D = 1 << K;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t g = (uint64_t)blockIdx.x * kBlock + threadIdx.x; g < ngroups; g += stride) {
        const uint64_t b = expand(g, ins);
        V x[D];
#pragma unroll
        for (int j = 0; j < D; ++j) x[j] = ldnt(amp + b + group_off<K>(gb, j));
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const T* row = m + 2 * D * i;
            // one product or multiply-add per statement: every term is a
            // fused multiply-add
            T re = row[0] * x[0].x;
            T im = row[0] * x[0].y;
            re = -row[1] * x[0].y + re;
            im = row[1] * x[0].x + im;
#pragma unroll
            for (int j = 1; j < D; ++j) {
                re = row[2 * j] * x[j].x + re;
                re = -row[2 * j + 1] * x[j].y + re;
                im = row[2 * j] * x[j].y + im;
                im = row[2 * j + 1] * x[j].x + im;
            }
            V y;
            y.x = re;
            y.y = im;
            stnt(amp + b + group_off<K>(gb, i), y);
        }
    }
}

// ---------------------------------------------------------------------------
// Every amplitude set to (re, im).  Write-only.
template <typename T, int U>
__global__ __launch_bounds__(kBlock) void k_init_fill(typename C2<T>::type* __restrict__ amp, uint64_t len,
                                                      T re, T im)
{
    using V = typename C2<T>::type;
    static_assert(U % 2 == 0, "the step order alternates two half-runs");
    const uint64_t ps = (uint64_t)kBlock * U;
    V v;
    v.x = re;
    v.y = im;
    for (uint64_t s = blockIdx.x; step_base(s, ps) < len; s += gridDim.x) {
        const uint64_t c = step_base(s, ps);
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint64_t i = step_item(c, j, ps);
            if (i < len) amp[i] = v;
        }
    }
}

// rho[j][k] = psi_j conj(psi_k) at vector index j + 2^N k (Eq. 2 layout).
// Write-only on rho; psi (2^N amplitudes) is read through the caches.
template <typename T, int U>
__global__ __launch_bounds__(kBlock) void k_dm_from_pure(typename C2<T>::type* __restrict__ rho,
                                                         const typename C2<T>::type* __restrict__ psi, int N)
{
    using V = typename C2<T>::type;
    static_assert(U % 2 == 0, "the step order alternates two half-runs");
    const uint64_t len = 1ull << (2 * N), low = (1ull << N) - 1;
    const uint64_t ps = (uint64_t)kBlock * U;
    for (uint64_t s = blockIdx.x; step_base(s, ps) < len; s += gridDim.x) {
        const uint64_t c = step_base(s, ps);
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint64_t i = step_item(c, j, ps);
            if (i >= len) continue;
            const V a = psi[i & low], b = psi[i >> N];
            V v;  // a conj(b)
            v.x = a.x * b.x + a.y * b.y;
            v.y = a.y * b.x - a.x * b.y;
            stnt(rho + i, v);
        }
    }
}

// sum_i conj(a_i) b_i: real part in the first compensated sum, imaginary
// part in the second (products formed in double).
template <typename T, int U>
__global__ __launch_bounds__(kBlock) void k_inner_sv(const typename C2<T>::type* __restrict__ a,
                                                     const typename C2<T>::type* __restrict__ b, uint64_t len,
                                                     double* partials)
{
    static_assert(U % 2 == 0, "the step order alternates two half-runs");
    using V = typename C2<T>::type;
    NSum s0 = {0.0, 0.0}, s1 = {0.0, 0.0};
    const uint64_t ps = (uint64_t)kBlock * U;
    for (uint64_t s = blockIdx.x; step_base(s, ps) < len; s += gridDim.x) {
        const uint64_t c = step_base(s, ps);
        V x[U], y[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint64_t i0 = step_item(c, j, ps);
            const uint64_t i = i0 < len ? i0 : len - 1;
            x[j] = ldnt(a + i);
            y[j] = ldnt(b + i);
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const bool in = step_item(c, j, ps) < len;
            const double xr = x[j].x, xi = x[j].y, yr = y[j].x, yi = y[j].y;
            nadd(s0, in ? xr * yr + xi * yi : 0.0);
            nadd(s1, in ? xr * yi - xi * yr : 0.0);
        }
    }
    block_store2(s0, s1, partials);
}

// <psi| rho |psi> = sum_{j,k} conj(psi_j) rho[j][k] psi_k over the Eq. 2
// vector (entry j + 2^N k): real part in the first sum, imaginary part (zero
// for a Hermitian rho, up to rounding) in the second.
template <typename T, int U>
__global__ __launch_bounds__(kBlock) void k_fid_dm(const typename C2<T>::type* __restrict__ rho,
                                                   const typename C2<T>::type* __restrict__ psi, int N,
                                                   double* partials)
{
    static_assert(U % 2 == 0, "the step order alternates two half-runs");
    using V = typename C2<T>::type;
    NSum s0 = {0.0, 0.0}, s1 = {0.0, 0.0};
    const uint64_t len = 1ull << (2 * N), low = (1ull << N) - 1;
    const uint64_t ps = (uint64_t)kBlock * U;
    for (uint64_t s = blockIdx.x; step_base(s, ps) < len; s += gridDim.x) {
        const uint64_t c = step_base(s, ps);
        V r[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint64_t i0 = step_item(c, j, ps);
            r[j] = ldnt(rho + (i0 < len ? i0 : len - 1));
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint64_t i0 = step_item(c, j, ps);
            const uint64_t i = i0 < len ? i0 : len - 1;
            const V pj = psi[i & low], pk = psi[i >> N];
            // t = conj(psi_j) rho psi_k, in double
            const double ar = pj.x, ai = -(double)pj.y, rr = r[j].x, ri = r[j].y, br = pk.x, bi = pk.y;
            const double ur = ar * rr - ai * ri, ui = ar * ri + ai * rr;
            const bool in = i0 < len;
            nadd(s0, in ? ur * br - ui * bi : 0.0);
            nadd(s1, in ? ur * bi + ui * br : 0.0);
        }
    }
    block_store2(s0, s1, partials);
}

}  // namespace

// ===========================================================================
// Launchers

// Controls (and phase bits) below kLineBits select within a 128-byte line:
// the pair and phase kernels walk those bits too and test them per item, so
// that loads and stores stay contiguous.
template <typename T>
constexpr int kLineBits = sizeof(T) == 8 ? 3 : 4;

// Small registers take kSmallPer items (amplitudes, pairs or 4-groups) per
// thread per step instead of 256 bytes' worth, so that the grid still
// spreads over the CUs (below 512 blocks with the large steps).  The step
// order needs an even count.
constexpr int kSmallPer = 2;

inline bool wide(uint64_t items, int per) { return items >= (uint64_t)512 * kBlock * per; }

template <typename T>
hipError_t launch_init_basis(const Launch& L, void* amp, uint64_t len, uint64_t index, double re, double im)
{
    using V = typename C2<T>::type;
    if (wide(len, kPer<T>))
        hipLaunchKernelGGL((k_init_basis<T, kPer<T>>), dim3(grid_for(len, kPer<T>)), dim3(kBlock), 0, L.stream,
                           (V*)amp, len, index, (T)re, (T)im);
    else
        hipLaunchKernelGGL((k_init_basis<T, kSmallPer>), dim3(grid_for(len, kSmallPer)), dim3(kBlock), 0,
                           L.stream, (V*)amp, len, index, (T)re, (T)im);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_hist_sv(const Launch& L, const void* amp, int nbits, int shift, uint64_t fixed, int mbits,
                          double* partials, int max_blocks, double* dev_out)
{
    using V = typename C2<T>::type;
    const uint64_t count = 1ull << (nbits - shift);
    int grid = grid_for(count, kPer<T>);
    if (grid > max_blocks) grid = max_blocks;
    const int nb = 1 << mbits;
    hipLaunchKernelGGL(k_hist_sv<T>, dim3(grid), dim3(kBlock), 0, L.stream, (const V*)amp, count, shift, fixed,
                       mbits, partials);
    hipLaunchKernelGGL(k_hist_final, dim3((nb + kBlock - 1) / kBlock), dim3(kBlock), 0, L.stream, partials, grid,
                       nb, dev_out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_diag_dm(const Launch& L, const void* rho, int N, double* dev_out)
{
    using V = typename C2<T>::type;
    const uint64_t dim = 1ull << N;
    hipLaunchKernelGGL(k_diag_dm<T>, dim3(grid_for(dim, 1)), dim3(kBlock), 0, L.stream, (const V*)rho, dim,
                       dev_out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gate(const Launch& L, void* amp, int nbits, int t, const int* ctrls, int nc,
                       const Mat2<T>& u, int* klass)
{
    using V = typename C2<T>::type;
    if (t < 6 && nbits >= 6) {
        // chunk index = amplitude index >> 6; controls >= 6 are inserted as ones
        int hp[64];
        int nh = 0;
        uint64_t ones = 0;
        uint32_t lowmask = 0;
        for (int k = 0; k < nc; ++k) {
            if (ctrls[k] >= 6) {
                hp[nh++] = ctrls[k] - 6;
                ones |= 1ull << (ctrls[k] - 6);
            } else {
                lowmask |= 1u << ctrls[k];
            }
        }
        const BitInsert hi = make_insert(hp, nh, ones);
        const uint64_t nchunks = 1ull << (nbits - 6 - nh);
        // one wave-row of 64 lanes per chunk, U chunks per wave per step
        const bool big = wide(nchunks * 64, kPer<T>);
        const int grid = grid_for(nchunks * 64, big ? kPer<T> : kSmallPer);
        switch (t) {
#define QS_LOW(TT) case TT:                                                                              \
    if (big)                                                                                             \
        hipLaunchKernelGGL((k_gate_low<T, TT, kPer<T>>), dim3(grid), dim3(kBlock), 0, L.stream, (V*)amp, \
                           nchunks, hi, lowmask, u);                                                     \
    else                                                                                                 \
        hipLaunchKernelGGL((k_gate_low<T, TT, kSmallPer>), dim3(grid), dim3(kBlock), 0, L.stream, (V*)amp, \
                           nchunks, hi, lowmask, u);                                                     \
    break;
            QS_LOW(0) QS_LOW(1) QS_LOW(2) QS_LOW(3) QS_LOW(4) QS_LOW(5)
#undef QS_LOW
        }
        if (klass) *klass = QS_K_GATE_LOW;
        return hipGetLastError();
    }
    int pos[64];
    int np = 0;
    uint64_t ones = 0, lowmask = 0;
    for (int k = 0; k < nc; ++k) {
        if (ctrls[k] < kLineBits<T>) {
            lowmask |= 1ull << ctrls[k];
            continue;
        }
        pos[np++] = ctrls[k];
        ones |= 1ull << ctrls[k];
    }
    pos[np] = t;
    const BitInsert ins = make_insert(pos, np + 1, ones);
    const uint64_t npairs = 1ull << (nbits - 1 - np);
    if (wide(npairs, kPer<T> / 2))
        hipLaunchKernelGGL((k_gate_pair<T, kPer<T> / 2>), dim3(grid_for(npairs, kPer<T> / 2)), dim3(kBlock), 0, L.stream,
                           (V*)amp, npairs, 1ull << t, ins, lowmask, u);
    else
        hipLaunchKernelGGL((k_gate_pair<T, kSmallPer>), dim3(grid_for(npairs, kSmallPer)), dim3(kBlock), 0,
                           L.stream, (V*)amp, npairs, 1ull << t, ins, lowmask, u);
    if (klass) *klass = QS_K_GATE;
    return hipGetLastError();
}

template <typename T>
hipError_t launch_not(const Launch& L, void* amp, int nbits, int t, const int* ctrls, int nc)
{
    if (t < 6 && nbits >= 6) {
        // the in-wave exchange path of dense gates keeps every access a full
        // line; X costs a few multiply-adds there
        Mat2<T> x;
        for (int k = 0; k < 8; ++k) x.m[k] = (k == 2 || k == 4) ? T(1) : T(0);
        return launch_gate<T>(L, amp, nbits, t, ctrls, nc, x, nullptr);
    }
    using V = typename C2<T>::type;
    int pos[64];
    int np = 0;
    uint64_t ones = 0, lowmask = 0;
    for (int k = 0; k < nc; ++k) {
        if (ctrls[k] < kLineBits<T>) {
            lowmask |= 1ull << ctrls[k];
            continue;
        }
        pos[np++] = ctrls[k];
        ones |= 1ull << ctrls[k];
    }
    pos[np] = t;
    const BitInsert ins = make_insert(pos, np + 1, ones);
    const uint64_t npairs = 1ull << (nbits - 1 - np);
    if (wide(npairs, kPer<T> / 2))
        hipLaunchKernelGGL((k_not<T, kPer<T> / 2>), dim3(grid_for(npairs, kPer<T> / 2)), dim3(kBlock), 0, L.stream,
                           (V*)amp, npairs, 1ull << t, ins, lowmask);
    else
        hipLaunchKernelGGL((k_not<T, kSmallPer>), dim3(grid_for(npairs, kSmallPer)), dim3(kBlock), 0, L.stream,
                           (V*)amp, npairs, 1ull << t, ins, lowmask);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_phase(const Launch& L, void* amp, int nbits, uint64_t mask, uint64_t skip,
                        double fre, double fim)
{
    using V = typename C2<T>::type;
    int pos[64];
    int np = 0;
    const uint64_t lowmask = mask & ((1ull << kLineBits<T>) - 1);
    for (int q = kLineBits<T>; q < nbits; ++q)
        if ((mask >> q) & 1) pos[np++] = q;
    const BitInsert ins = make_insert(pos, np, mask & ~lowmask);
    const uint64_t count = 1ull << (nbits - np);
    if (wide(count, kPer<T>))
        hipLaunchKernelGGL((k_phase<T, kPer<T>>), dim3(grid_for(count, kPer<T>)), dim3(kBlock), 0, L.stream,
                           (V*)amp, count, ins, lowmask, skip, (T)fre, (T)fim);
    else
        hipLaunchKernelGGL((k_phase<T, kSmallPer>), dim3(grid_for(count, kSmallPer)), dim3(kBlock), 0, L.stream,
                           (V*)amp, count, ins, lowmask, skip, (T)fre, (T)fim);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_dm_gate(const Launch& L, void* rho, int N, int t, const int* ctrls, int nc,
                          const Mat2<T>& u)
{
    using V = typename C2<T>::type;
    const int pos[2] = {t, t + N};
    const BitInsert ins = make_insert(pos, 2, 0);
    uint64_t rmask = 0;
    for (int k = 0; k < nc; ++k) rmask |= 1ull << ctrls[k];
    const uint64_t ngroups = 1ull << (2 * N - 2);
    if (wide(ngroups, kPer<T> / 4))
        hipLaunchKernelGGL((k_dm_gate<T, kPer<T> / 4>), dim3(grid_for(ngroups, kPer<T> / 4)), dim3(kBlock), 0,
                           L.stream, (V*)rho, ngroups, 1ull << t, 1ull << (t + N), ins, rmask, rmask << N, u);
    else
        hipLaunchKernelGGL((k_dm_gate<T, kSmallPer>), dim3(grid_for(ngroups, kSmallPer)), dim3(kBlock), 0, L.stream,
                           (V*)rho, ngroups, 1ull << t, 1ull << (t + N), ins, rmask, rmask << N, u);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_dm_channel(const Launch& L, void* rho, int N, int t, int channel, double p)
{
    using V = typename C2<T>::type;
    const int pos[2] = {t, t + N};
    const BitInsert ins = make_insert(pos, 2, 0);
    const uint64_t ngroups = 1ull << (2 * N - 2);
    const bool big = wide(ngroups, kPer<T> / 4);
    const dim3 grid(grid_for(ngroups, big ? kPer<T> / 4 : kSmallPer)), block(kBlock);
    const uint64_t tb = 1ull << t, cb = 1ull << (t + N);
    switch (channel) {
    case QS_DEPHASING:
        if (big)
            hipLaunchKernelGGL((k_dm_channel<T, QS_DEPHASING, kPer<T> / 4>), grid, block, 0, L.stream, (V*)rho, ngroups,
                               tb, cb, ins, 0.0, 0.0, 1.0 - 2.0 * p);
        else
            hipLaunchKernelGGL((k_dm_channel<T, QS_DEPHASING, kSmallPer>), grid, block, 0, L.stream, (V*)rho, ngroups,
                               tb, cb, ins, 0.0, 0.0, 1.0 - 2.0 * p);
        break;
    case QS_DEPOLARISING:
        if (big)
            hipLaunchKernelGGL((k_dm_channel<T, QS_DEPOLARISING, kPer<T> / 4>), grid, block, 0, L.stream, (V*)rho, ngroups,
                               tb, cb, ins, 1.0 - 2.0 * p / 3.0, 2.0 * p / 3.0,
                           1.0 - 4.0 * p / 3.0);
        else
            hipLaunchKernelGGL((k_dm_channel<T, QS_DEPOLARISING, kSmallPer>), grid, block, 0, L.stream, (V*)rho, ngroups,
                               tb, cb, ins, 1.0 - 2.0 * p / 3.0, 2.0 * p / 3.0,
                           1.0 - 4.0 * p / 3.0);
        break;
    default:
        if (big)
            hipLaunchKernelGGL((k_dm_channel<T, QS_DAMPING, kPer<T> / 4>), grid, block, 0, L.stream, (V*)rho, ngroups,
                               tb, cb, ins, p, 1.0 - p, sqrt(1.0 - p));
        else
            hipLaunchKernelGGL((k_dm_channel<T, QS_DAMPING, kSmallPer>), grid, block, 0, L.stream, (V*)rho, ngroups,
                               tb, cb, ins, p, 1.0 - p, sqrt(1.0 - p));
        break;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_prob_sv(const Launch& L, const void* amp, int nbits, int q, double* partials,
                          double* dev_out)
{
    using V = typename C2<T>::type;
    const uint64_t len = 1ull << nbits;
    const bool big = wide(len, kPer<T>);
    int grid = grid_for(len, big ? kPer<T> : kSmallPer);
    if (grid > kReduceBlocks) grid = kReduceBlocks;
    if (big)
        hipLaunchKernelGGL((k_prob_sv<T, kPer<T>>), dim3(grid), dim3(kBlock), 0, L.stream, (const V*)amp, len, q,
                           partials);
    else
        hipLaunchKernelGGL((k_prob_sv<T, kSmallPer>), dim3(grid), dim3(kBlock), 0, L.stream, (const V*)amp, len, q,
                           partials);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kBlock), 0, L.stream, partials, grid, dev_out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_prob_half_sv(const Launch& L, const void* amp, int nbits, int q, int outcome, double* partials,
                               double* dev_out)
{
    using V = typename C2<T>::type;
    const uint64_t half = 1ull << (nbits - 1);
    const bool big = wide(half, kPer<T>);
    int grid = grid_for(half, big ? kPer<T> : kSmallPer);
    if (grid > kReduceBlocks) grid = kReduceBlocks;
    if (big)
        hipLaunchKernelGGL((k_prob_half_sv<T, kPer<T>>), dim3(grid), dim3(kBlock), 0, L.stream, (const V*)amp, half,
                           q, outcome, partials);
    else
        hipLaunchKernelGGL((k_prob_half_sv<T, kSmallPer>), dim3(grid), dim3(kBlock), 0, L.stream, (const V*)amp, half,
                           q, outcome, partials);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kBlock), 0, L.stream, partials, grid, dev_out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_prob_dm(const Launch& L, const void* rho, int N, int q, double* partials,
                          double* dev_out)
{
    using V = typename C2<T>::type;
    const uint64_t dim = 1ull << N;
    int grid = grid_for(dim, 1);
    if (grid > kReduceBlocks) grid = kReduceBlocks;
    hipLaunchKernelGGL(k_prob_dm<T>, dim3(grid), dim3(kBlock), 0, L.stream, (const V*)rho, dim, q,
                       partials);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kBlock), 0, L.stream, partials, grid, dev_out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_collapse_sv(const Launch& L, void* amp, int nbits, int q, int outcome, double scale)
{
    using V = typename C2<T>::type;
    const uint64_t len = 1ull << nbits;
    if (wide(len, kPer<T>))
        hipLaunchKernelGGL((k_collapse_sv<T, kPer<T>>), dim3(grid_for(len, kPer<T>)), dim3(kBlock), 0, L.stream,
                           (V*)amp, len, q, outcome, scale);
    else
        hipLaunchKernelGGL((k_collapse_sv<T, kSmallPer>), dim3(grid_for(len, kSmallPer)), dim3(kBlock), 0, L.stream,
                           (V*)amp, len, q, outcome, scale);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_collapse_dm(const Launch& L, void* rho, int N, int q, int outcome, double scale)
{
    using V = typename C2<T>::type;
    const uint64_t len = 1ull << (2 * N);
    if (wide(len, kPer<T>))
        hipLaunchKernelGGL((k_collapse_dm<T, kPer<T>>), dim3(grid_for(len, kPer<T>)), dim3(kBlock), 0, L.stream,
                           (V*)rho, len, q, N, outcome, scale);
    else
        hipLaunchKernelGGL((k_collapse_dm<T, kSmallPer>), dim3(grid_for(len, kSmallPer)), dim3(kBlock), 0, L.stream,
                           (V*)rho, len, q, N, outcome, scale);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_group_gate(const Launch& L, void* amp, int nbits, const int* targets, int k, const int* ctrls,
                             int nc, const T* dev_m)
{
    using V = typename C2<T>::type;
    int pos[64];
    int np = 0;
    uint64_t ones = 0;
    for (int j = 0; j < k; ++j) pos[np++] = targets[j];
    for (int j = 0; j < nc; ++j) {
        pos[np++] = ctrls[j];
        ones |= 1ull << ctrls[j];
    }
    const BitInsert ins = make_insert(pos, np, ones);
    const uint64_t ngroups = 1ull << (nbits - np);
    const int grid = grid_for(ngroups, 1);
    switch (k) {
#define QS_GROUP(KK) case KK: {                                                                        \
        GroupBits<KK> gb;                                                                              \
        for (int j = 0; j < KK; ++j) gb.tbit[j] = 1ull << targets[j];                                  \
        hipLaunchKernelGGL((k_group_gate<T, KK>), dim3(grid), dim3(kBlock), 0, L.stream, (V*)amp, ngroups, \
                           ins, gb, dev_m);                                                            \
        break;                                                                                         \
    }
        QS_GROUP(1) QS_GROUP(2) QS_GROUP(3) QS_GROUP(4) QS_GROUP(5)
#undef QS_GROUP
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_init_fill(const Launch& L, void* amp, uint64_t len, double re, double im)
{
    using V = typename C2<T>::type;
    if (wide(len, kPer<T>))
        hipLaunchKernelGGL((k_init_fill<T, kPer<T>>), dim3(grid_for(len, kPer<T>)), dim3(kBlock), 0, L.stream,
                           (V*)amp, len, (T)re, (T)im);
    else
        hipLaunchKernelGGL((k_init_fill<T, kSmallPer>), dim3(grid_for(len, kSmallPer)), dim3(kBlock), 0,
                           L.stream, (V*)amp, len, (T)re, (T)im);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_dm_from_pure(const Launch& L, void* rho, int N, const void* psi)
{
    using V = typename C2<T>::type;
    const uint64_t len = 1ull << (2 * N);
    if (wide(len, kPer<T>))
        hipLaunchKernelGGL((k_dm_from_pure<T, kPer<T>>), dim3(grid_for(len, kPer<T>)), dim3(kBlock), 0,
                           L.stream, (V*)rho, (const V*)psi, N);
    else
        hipLaunchKernelGGL((k_dm_from_pure<T, kSmallPer>), dim3(grid_for(len, kSmallPer)), dim3(kBlock), 0,
                           L.stream, (V*)rho, (const V*)psi, N);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_inner_sv(const Launch& L, const void* a, const void* b, int nbits, double* partials,
                           double* dev_out)
{
    using V = typename C2<T>::type;
    const uint64_t len = 1ull << nbits;
    constexpr int U = kPer<T> / 2;  // two streams per step
    int grid;
    if (wide(len, U)) {
        grid = std::min(grid_for(len, U), kReduceBlocks);
        hipLaunchKernelGGL((k_inner_sv<T, U>), dim3(grid), dim3(kBlock), 0, L.stream, (const V*)a, (const V*)b,
                           len, partials);
    } else {
        grid = std::min(grid_for(len, kSmallPer), kReduceBlocks);
        hipLaunchKernelGGL((k_inner_sv<T, kSmallPer>), dim3(grid), dim3(kBlock), 0, L.stream, (const V*)a,
                           (const V*)b, len, partials);
    }
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kBlock), 0, L.stream, partials, grid, dev_out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fid_dm(const Launch& L, const void* rho, int N, const void* psi, double* partials,
                         double* dev_out)
{
    using V = typename C2<T>::type;
    const uint64_t len = 1ull << (2 * N);
    int grid;
    if (wide(len, kPer<T>)) {
        grid = std::min(grid_for(len, kPer<T>), kReduceBlocks);
        hipLaunchKernelGGL((k_fid_dm<T, kPer<T>>), dim3(grid), dim3(kBlock), 0, L.stream, (const V*)rho,
                           (const V*)psi, N, partials);
    } else {
        grid = std::min(grid_for(len, kSmallPer), kReduceBlocks);
        hipLaunchKernelGGL((k_fid_dm<T, kSmallPer>), dim3(grid), dim3(kBlock), 0, L.stream, (const V*)rho,
                           (const V*)psi, N, partials);
    }
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kBlock), 0, L.stream, partials, grid, dev_out);
    return hipGetLastError();
}

#define QS_INSTANTIATE(T)                                                                              \
    template hipError_t launch_init_basis<T>(const Launch&, void*, uint64_t, uint64_t, double, double); \
    template hipError_t launch_hist_sv<T>(const Launch&, const void*, int, int, uint64_t, int, double*, int, \
                                          double*);                                                    \
    template hipError_t launch_diag_dm<T>(const Launch&, const void*, int, double*);                   \
    template hipError_t launch_gate<T>(const Launch&, void*, int, int, const int*, int, const Mat2<T>&, \
                                       int*);                                                          \
    template hipError_t launch_not<T>(const Launch&, void*, int, int, const int*, int);                \
    template hipError_t launch_phase<T>(const Launch&, void*, int, uint64_t, uint64_t, double, double); \
    template hipError_t launch_dm_gate<T>(const Launch&, void*, int, int, const int*, int,             \
                                          const Mat2<T>&);                                             \
    template hipError_t launch_dm_channel<T>(const Launch&, void*, int, int, int, double);             \
    template hipError_t launch_prob_sv<T>(const Launch&, const void*, int, int, double*, double*);     \
    template hipError_t launch_prob_half_sv<T>(const Launch&, const void*, int, int, int, double*, double*); \
    template hipError_t launch_prob_dm<T>(const Launch&, const void*, int, int, double*, double*);     \
    template hipError_t launch_collapse_sv<T>(const Launch&, void*, int, int, int, double);            \
    template hipError_t launch_collapse_dm<T>(const Launch&, void*, int, int, int, double); \
    template hipError_t launch_group_gate<T>(const Launch&, void*, int, const int*, int, const int*, int, \
                                             const T*);                                                \
    template hipError_t launch_init_fill<T>(const Launch&, void*, uint64_t, double, double);           \
    template hipError_t launch_dm_from_pure<T>(const Launch&, void*, int, const void*);                \
    template hipError_t launch_inner_sv<T>(const Launch&, const void*, const void*, int, double*, double*); \
    template hipError_t launch_fid_dm<T>(const Launch&, const void*, int, const void*, double*, double*);

QS_INSTANTIATE(double)
QS_INSTANTIATE(float)

hipError_t launch_sum_columns(const Launch& L, const double* part, int rows, int cols, double* out)
{
    if (rows < 1 || cols < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sum_columns, dim3((cols + 63) / 64), dim3(64), 0, L.stream, part, rows, cols, out);
    return hipGetLastError();
}

}  // namespace qs
