// Gate fusion for state vectors: a run of gates whose targets lie in a set S
// of K qubits is applied to every 2^K-amplitude tile (all amplitudes that
// agree on the qubits outside S) in one read and one write of HBM -- the
// GPU form of the cache blocking / gate fusion described in Sec. II.B.
//
// Tile layout.  A workgroup of 2^TB threads holds a tile of 2^K = 2^(TB+RB)
// amplitudes in registers, 2^RB per thread.  At any moment each local qubit
// of the tile is either a "thread bit" (selects the thread) or a "register
// bit" (selects the register inside the thread).  A gate whose target is a
// register bit is applied by every thread to its own registers; controls and
// diagonal phases may sit anywhere, since a thread knows the value of its
// thread bits and of the qubits outside S (fixed per tile).  When the next
// gates target thread bits, the tile is re-laid out through LDS (one write
// and one read of 2^K amplitudes) so that those qubits become register
// bits.  Lanes 0..63 always cover global qubits 0..5 when the tile is read
// from or written to HBM, so every global access is a contiguous 64-element
// run per wavefront.
//
// LDS addresses are a linear map over GF(2) of the local index (an XOR
// swizzle chosen per re-layout so that the 8 lanes of a 128-byte LDS cycle
// hit distinct banks in both the writing and the reading layout).  Each
// layout is handed to the kernel as the images of single thread / register
// bits, so the kernel only XORs precomputed values.
#include <string.h>

#include <algorithm>
#include <complex>
#include <memory>
#include <vector>

#include "qs_device.h"
#include "qs_host.h"
#include "qs_plan.h"

namespace qs {
namespace {

constexpr int kTBMax = 10;
constexpr int kRBMax = 5;

struct FPhase {
    uint32_t wthr[kTBMax], wreg[kRBMax];  // LDS images of the layout being left
    uint32_t rthr[kTBMax], rreg[kRBMax];  // LDS images of the layout entered
    int op_begin, op_end;
};

struct FPass {
    int nphases;
    int final_transpose;  // 1: re-lay out to the store layout before storing
    uint64_t ld_thr[kTBMax], ld_reg[kRBMax];  // HBM offsets of the load layout
    uint64_t st_thr[kTBMax], st_reg[kRBMax];  // HBM offsets of the store layout
    BitInsert outside;                        // inserts zeros at the tile's qubits
    FPhase ph[kPhMax];
    FPhase fin;
};

struct FOp {
    int kind;        // specialised op code (see apply_op)
    int rb;          // target register bit (dense / not / core)
    uint32_t rmask;  // register bits that must be 1
    uint32_t tmask;  // thread-index bits that must be 1
    uint64_t gmask;  // global qubits outside the tile that must be 1
    double m[8];     // dense matrix, phase factor in m[0], m[1], or core coefficient k in m[0], m[1]
    uint32_t aux;    // 4x4 ops: entry of the 4x4 matrix table
    uint32_t pad;
};

// In-register op application.  Conditions that are the same for the whole
// workgroup (controls outside the tile, register-bit controls) become scalar
// selects; only thread-bit controls need per-lane selects.  Every variant is
// straight-line code over compile-time register indices.

template <typename T>
__device__ __forceinline__ void load_mat(T (&m)[8], const FOp& op)
{
#pragma unroll
    for (int k = 0; k < 8; ++k) m[k] = (T)op.m[k];
}

// Identity element k of a row-major interleaved 2x2 matrix.
template <typename T>
__device__ __forceinline__ T ident(int k) { return (k == 0 || k == 6) ? T(1) : T(0); }

// Dense 2x2 on register bit RBIT.  MASKED: only pairs whose register index
// has every bit of rmask set (identity matrix elsewhere, chosen per pair).
template <typename T, int RB, int RBIT, bool MASKED>
__device__ __forceinline__ void dense_rb(typename C2<T>::type (&v)[1 << RB], const T (&m)[8], uint32_t rmask)
{
    using V = typename C2<T>::type;
#pragma unroll
    for (int r0 = 0; r0 < (1 << RB); ++r0) {
        if (r0 & (1 << RBIT)) continue;
        if constexpr (MASKED) {
            // the register-control test is the same for every lane: a scalar
            // branch skips the pairs it excludes
            if (((uint32_t)r0 & rmask) == rmask) apply2<T, V>(m, v[r0], v[r0 | (1 << RBIT)]);
        } else {
            apply2<T, V>(m, v[r0], v[r0 | (1 << RBIT)]);
        }
    }
}

// NOT on register bit RBIT: swap each pair where `sel` (per lane) and, when
// MASKED, the pair's register controls hold.  LANE = false: sel is true.
template <typename T, int RB, int RBIT, bool MASKED, bool LANE>
__device__ __forceinline__ void not_rb(typename C2<T>::type (&v)[1 << RB], uint32_t rmask, bool sel)
{
    using V = typename C2<T>::type;
#pragma unroll
    for (int r0 = 0; r0 < (1 << RB); ++r0) {
        if (r0 & (1 << RBIT)) continue;
        const int r1 = r0 | (1 << RBIT);
        if constexpr (MASKED) {  // uniform over the wave: skip excluded pairs by a branch
            if (((uint32_t)r0 & rmask) != rmask) continue;
        }
        const bool c = LANE ? sel : true;
        if constexpr (!LANE) {
            const V t = v[r0];
            v[r0] = v[r1];
            v[r1] = t;
        } else {
            const V a = v[r0], b = v[r1];
            v[r0].x = c ? b.x : a.x;
            v[r0].y = c ? b.y : a.y;
            v[r1].x = c ? a.x : b.x;
            v[r1].y = c ? a.y : b.y;
        }
    }
}

// Diagonal phase: multiply the registers whose index has every bit of rmask
// set by (fr, fi) (already 1 on lanes that fail their thread-bit controls).
template <typename T, int RB>
__device__ __forceinline__ void phase_op(typename C2<T>::type (&v)[1 << RB], T fr, T fi, uint32_t rmask)
{
    using V = typename C2<T>::type;
#pragma unroll
    for (int r = 0; r < (1 << RB); ++r)
        if (((uint32_t)r & rmask) == rmask) v[r] = cmul<T, V>(fr, fi, v[r]);  // uniform branch
}

// Op codes: the host specialises every op so that the device dispatches with
// one switch and each case is straight-line code.
//   code = 4 * rb + variant        dense gate (variant: bit 0 register controls,
//                                  bit 1 thread-bit controls)
//   code = 32 + 4 * rb + variant   NOT
//   code = 64 + lane               phase (lane: thread-bit controls present)
//   code = 96 + 4 * rb + variant   diagonal dense gate (u01 = u10 = 0)
//   code = 128 + 4 * rb            unit-diagonal core, amplitudes in place:
//                                  (a, b) <- (a + k b, b - conj(k) a)
//   code = 160 + 4 * rb            core with the pair exchanged:
//                                  (a, b) <- (k a + b, a - conj(k) b)
//   code = 192 + pair              4x4 on register bits (b1 < b2), pair index
//                                  of (b1, b2), matrix in the 4x4 table
//   code = 255                     nothing (a gate whose effect is deferred)
enum : int { kDense = 0, kNot = 32, kPhase = 64, kDiag = 96, kCoreA = 128, kCoreB = 160, kDense4 = 192, kNop = 255 };

// Register-bit pairs of the 4x4 ops, indexed by (b1 < b2) in lexical order.
constexpr int kPairB1[10] = {0, 0, 0, 0, 1, 1, 1, 2, 2, 3};
constexpr int kPairB2[10] = {1, 2, 3, 4, 2, 3, 4, 3, 4, 4};

template <typename T, int RB, int RBIT, bool EXCH>
__device__ __forceinline__ void core_case(typename C2<T>::type (&v)[1 << RB], const FOp& op)
{
    using V = typename C2<T>::type;
    const T kr = (T)op.m[0], ki = (T)op.m[1];
#pragma unroll
    for (int r0 = 0; r0 < (1 << RB); ++r0) {
        if (r0 & (1 << RBIT)) continue;
        const V a = v[r0], b = v[r0 | (1 << RBIT)];
        V na, nb;
        if constexpr (!EXCH) {  // a + k b, b - conj(k) a
            na.x = kr * b.x + a.x;
            na.x = -ki * b.y + na.x;
            na.y = kr * b.y + a.y;
            na.y = ki * b.x + na.y;
            nb.x = -kr * a.x + b.x;
            nb.x = -ki * a.y + nb.x;
            nb.y = -kr * a.y + b.y;
            nb.y = ki * a.x + nb.y;
        } else {  // k a + b, a - conj(k) b
            na.x = kr * a.x + b.x;
            na.x = -ki * a.y + na.x;
            na.y = kr * a.y + b.y;
            na.y = ki * a.x + na.y;
            nb.x = -kr * b.x + a.x;
            nb.x = -ki * b.y + nb.x;
            nb.y = -kr * b.y + a.y;
            nb.y = ki * b.x + nb.y;
        }
        v[r0] = na;
        v[r0 | (1 << RBIT)] = nb;
    }
}

// 4x4 complex matrix m (row-major, index bit(B1) + 2 bit(B2)) on every
// register quad.
template <typename T, int RB, int B1, int B2>
__device__ __forceinline__ void dense4_case(typename C2<T>::type (&v)[1 << RB], const T* __restrict__ m)
{
    using V = typename C2<T>::type;
#pragma unroll
    for (int r0 = 0; r0 < (1 << RB); ++r0) {
        if ((r0 >> B1) & 1 || (r0 >> B2) & 1) continue;
        const int r[4] = {r0, r0 | (1 << B1), r0 | (1 << B2), r0 | (1 << B1) | (1 << B2)};
        const V x[4] = {v[r[0]], v[r[1]], v[r[2]], v[r[3]]};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            // one product or multiply-add per statement
            T re = m[8 * i] * x[0].x;
            T im = m[8 * i] * x[0].y;
            re = -m[8 * i + 1] * x[0].y + re;
            im = m[8 * i + 1] * x[0].x + im;
#pragma unroll
            for (int j = 1; j < 4; ++j) {
                const T mr = m[2 * (4 * i + j)], mi = m[2 * (4 * i + j) + 1];
                re = mr * x[j].x + re;
                re = -mi * x[j].y + re;
                im = mr * x[j].y + im;
                im = mi * x[j].x + im;
            }
            v[r[i]].x = re;
            v[r[i]].y = im;
        }
    }
}

template <typename T, int RB, int RBIT, int VAR>
__device__ __forceinline__ void dense_case(typename C2<T>::type (&v)[1 << RB], const FOp& op, uint32_t tid)
{
    T m[8];
    load_mat<T>(m, op);
    if constexpr (VAR & 2) {
        const bool sel = (tid & op.tmask) == op.tmask;
#pragma unroll
        for (int k = 0; k < 8; ++k) m[k] = sel ? m[k] : ident<T>(k);
    }
    dense_rb<T, RB, RBIT, (VAR & 1) != 0>(v, m, op.rmask);
}

// Diagonal 2x2 on register bit RBIT: each amplitude of a pair is multiplied
// by its diagonal entry (half the work of a dense product).
template <typename T, int RB, int RBIT, int VAR>
__device__ __forceinline__ void diag_case(typename C2<T>::type (&v)[1 << RB], const FOp& op, uint32_t tid)
{
    using V = typename C2<T>::type;
    T d0r = (T)op.m[0], d0i = (T)op.m[1], d1r = (T)op.m[6], d1i = (T)op.m[7];
    if constexpr (VAR & 2) {
        const bool sel = (tid & op.tmask) == op.tmask;
        d0r = sel ? d0r : T(1);
        d0i = sel ? d0i : T(0);
        d1r = sel ? d1r : T(1);
        d1i = sel ? d1i : T(0);
    }
#pragma unroll
    for (int r0 = 0; r0 < (1 << RB); ++r0) {
        if (r0 & (1 << RBIT)) continue;
        if constexpr (VAR & 1) {  // register controls: uniform over the wave
            if (((uint32_t)r0 & op.rmask) != op.rmask) continue;
        }
        v[r0] = cmul<T, V>(d0r, d0i, v[r0]);
        v[r0 | (1 << RBIT)] = cmul<T, V>(d1r, d1i, v[r0 | (1 << RBIT)]);
    }
}

template <typename T, int RB, int RBIT, int VAR>
__device__ __forceinline__ void not_case(typename C2<T>::type (&v)[1 << RB], const FOp& op, uint32_t tid)
{
    const bool sel = (tid & op.tmask) == op.tmask;
    not_rb<T, RB, RBIT, (VAR & 1) != 0, (VAR & 2) != 0>(v, op.rmask, sel);
}

template <typename T, int RB, bool LANE>
__device__ __forceinline__ void phase_case(typename C2<T>::type (&v)[1 << RB], const FOp& op, uint32_t tid)
{
    T fr = (T)op.m[0], fi = (T)op.m[1];
    if constexpr (LANE) {
        const bool sel = (tid & op.tmask) == op.tmask;
        fr = sel ? fr : T(1);
        fi = sel ? fi : T(0);
    }
    phase_op<T, RB>(v, fr, fi, op.rmask);
}

template <typename T, int RB>
__device__ __forceinline__ void apply_op(typename C2<T>::type (&v)[1 << RB], const FOp& op, uint32_t tid,
                                         const T* __restrict__ m4tab)
{
    switch (op.kind) {
#define QS_DENSE(RBIT)                                                                   \
    case kDense + 4 * RBIT + 0: if constexpr (RB > RBIT) dense_case<T, RB, RBIT, 0>(v, op, tid); break; \
    case kDense + 4 * RBIT + 1: if constexpr (RB > RBIT) dense_case<T, RB, RBIT, 1>(v, op, tid); break; \
    case kDense + 4 * RBIT + 2: if constexpr (RB > RBIT) dense_case<T, RB, RBIT, 2>(v, op, tid); break; \
    case kDense + 4 * RBIT + 3: if constexpr (RB > RBIT) dense_case<T, RB, RBIT, 3>(v, op, tid); break; \
    case kNot + 4 * RBIT + 0: if constexpr (RB > RBIT) not_case<T, RB, RBIT, 0>(v, op, tid); break;     \
    case kNot + 4 * RBIT + 1: if constexpr (RB > RBIT) not_case<T, RB, RBIT, 1>(v, op, tid); break;     \
    case kNot + 4 * RBIT + 2: if constexpr (RB > RBIT) not_case<T, RB, RBIT, 2>(v, op, tid); break;     \
    case kNot + 4 * RBIT + 3: if constexpr (RB > RBIT) not_case<T, RB, RBIT, 3>(v, op, tid); break;     \
    case kDiag + 4 * RBIT + 0: if constexpr (RB > RBIT) diag_case<T, RB, RBIT, 0>(v, op, tid); break;   \
    case kDiag + 4 * RBIT + 1: if constexpr (RB > RBIT) diag_case<T, RB, RBIT, 1>(v, op, tid); break;   \
    case kDiag + 4 * RBIT + 2: if constexpr (RB > RBIT) diag_case<T, RB, RBIT, 2>(v, op, tid); break;   \
    case kDiag + 4 * RBIT + 3: if constexpr (RB > RBIT) diag_case<T, RB, RBIT, 3>(v, op, tid); break;
    QS_DENSE(0) QS_DENSE(1) QS_DENSE(2) QS_DENSE(3) QS_DENSE(4)
#undef QS_DENSE
#define QS_CORE(RBIT)                                                                                    \
    case kCoreA + 4 * RBIT: if constexpr (RB > RBIT) core_case<T, RB, RBIT, false>(v, op); break;        \
    case kCoreB + 4 * RBIT: if constexpr (RB > RBIT) core_case<T, RB, RBIT, true>(v, op); break;
    QS_CORE(0) QS_CORE(1) QS_CORE(2) QS_CORE(3) QS_CORE(4)
#undef QS_CORE
#define QS_D4(P)                                                                                         \
    case kDense4 + P:                                                                                    \
        if constexpr (RB > kPairB2[P]) dense4_case<T, RB, kPairB1[P], kPairB2[P]>(v, m4tab + 32 * op.aux); \
        break;
    QS_D4(0) QS_D4(1) QS_D4(2) QS_D4(3) QS_D4(4) QS_D4(5) QS_D4(6) QS_D4(7) QS_D4(8) QS_D4(9)
#undef QS_D4
    case kPhase + 0: phase_case<T, RB, false>(v, op, tid); break;
    case kPhase + 1: phase_case<T, RB, true>(v, op, tid); break;
    default: break;
    }
}

// XOR of img[b] over the set bits b of x (x < 2^NB).
template <int NB, typename U>
__device__ __forceinline__ U span(uint32_t x, const U* img)
{
    U s = 0;
#pragma unroll
    for (int b = 0; b < NB; ++b)
        if ((x >> b) & 1) s ^= img[b];
    return s;
}

template <int NB, typename U>
__device__ __forceinline__ U span_sum(uint32_t x, const U* img)
{
    U s = 0;
#pragma unroll
    for (int b = 0; b < NB; ++b)
        if ((x >> b) & 1) s += img[b];
    return s;
}

template <typename T, int TB, int RB>
__device__ __forceinline__ void relayout(typename C2<T>::type (&v)[1 << RB],
                                         typename C2<T>::type* lds, const FPhase& F, uint32_t tid)
{
    const uint32_t tw = span<TB, uint32_t>(tid, F.wthr);
    const uint32_t tr = span<TB, uint32_t>(tid, F.rthr);
#pragma unroll
    for (int r = 0; r < (1 << RB); ++r) lds[tw ^ span<RB, uint32_t>((uint32_t)r, F.wreg)] = v[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < (1 << RB); ++r) v[r] = lds[tr ^ span<RB, uint32_t>((uint32_t)r, F.rreg)];
    __syncthreads();
}

// One tile of a planned pass: load, apply every phase's ops with the
// re-layouts between them, store.  `base` = tile index with zeros at the
// tile's qubits.
template <typename T, int TB, int RB>
__device__ __forceinline__ void process_tile(typename C2<T>::type* __restrict__ amp, const FPass* __restrict__ P,
                                             const FOp* __restrict__ ops, const T* __restrict__ m4tab,
                                             uint64_t tile, typename C2<T>::type* lds, uint32_t tid,
                                             bool zero_init = false)
{
    using V = typename C2<T>::type;
    constexpr int E = 1 << RB;
    const uint64_t ld_t = span_sum<TB, uint64_t>(tid, P->ld_thr);
    const uint64_t st_t = span_sum<TB, uint64_t>(tid, P->st_thr);
    const int nph = P->nphases;
    const uint64_t base = expand(tile, P->outside);
    V v[E];
    if (zero_init) {  // the tile of |0..0>: nothing to read
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const uint64_t a = base + ld_t + span_sum<RB, uint64_t>((uint32_t)r, P->ld_reg);
            v[r].x = (a == 0) ? T(1) : T(0);
            v[r].y = T(0);
        }
    } else {
#pragma unroll
        for (int r = 0; r < E; ++r) v[r] = amp[base + ld_t + span_sum<RB, uint64_t>((uint32_t)r, P->ld_reg)];
    }
    for (int ph = 0; ph < nph; ++ph) {
        const FPhase& F = P->ph[ph];
        if (ph > 0) relayout<T, TB, RB>(v, lds, F, tid);
        for (int o = F.op_begin; o < F.op_end; ++o) {
            const FOp& op = ops[o];
            if ((base & op.gmask) != op.gmask) continue;  // same for the whole tile
            apply_op<T, RB>(v, op, tid, m4tab);
        }
    }
    if (P->final_transpose) relayout<T, TB, RB>(v, lds, P->fin, tid);
#pragma unroll
    for (int r = 0; r < E; ++r) amp[base + st_t + span_sum<RB, uint64_t>((uint32_t)r, P->st_reg)] = v[r];
}

template <typename T, int TB, int RB>
__global__ __launch_bounds__(1 << TB) void k_fused(typename C2<T>::type* __restrict__ amp,
                                                   const FPass* __restrict__ P,
                                                   const FOp* __restrict__ ops, const T* __restrict__ m4tab,
                                                   uint64_t ntiles)
{
    using V = typename C2<T>::type;
    __shared__ V lds[1 << (TB + RB)];
    for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x)
        process_tile<T, TB, RB>(amp, P, ops, m4tab, tile, lds, threadIdx.x);
}

// Batched registers.  Every register's circuit is planned into passes; the
// work of pass level p is the list of items (register, its pass p, range of
// tiles) over all registers that have a pass p.  One launch per level runs
// its items, each workgroup taking items in a grid-stride loop; the launch
// boundary is the only synchronisation between the passes of a register, so
// no workgroup ever waits for another.  Tiles of the first pass can be
// produced as |0..0> instead of being read (init).
struct BatchReg {
    void* amp;
    int n;
    int npasses;
    uint32_t pass0;  // first pass of the register in the pass array
    uint32_t pad;
};

struct BatchItem {
    uint32_t reg, pass, tile0, tile1;
};

template <typename T, int TB, int RB>
__global__ __launch_bounds__(1 << TB) void k_batch(const BatchReg* __restrict__ regs,
                                                   const BatchItem* __restrict__ items, int nitems,
                                                   const FPass* __restrict__ passes,
                                                   const FOp* __restrict__ ops, const T* __restrict__ m4tab,
                                                   int init)
{
    using V = typename C2<T>::type;
    __shared__ V lds[1 << (TB + RB)];
    const uint32_t tid = threadIdx.x;
    for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
        const BatchItem it = items[i];
        const BatchReg R = regs[it.reg];
        const FPass* P = passes + R.pass0 + it.pass;
        const bool zi = init && it.pass == 0;
        for (uint32_t tile = it.tile0; tile < it.tile1; ++tile)
            process_tile<T, TB, RB>((V*)R.amp, P, ops, m4tab, tile, lds, tid, zi);
    }
}

// Per-register probabilities: out[2 i] = P(qubit q = 0), out[2 i + 1] =
// total probability, both as compensated double sums.
template <typename T>
__global__ __launch_bounds__(256) void k_batch_probs(const BatchReg* __restrict__ regs, int nregs, int q,
                                                     double* __restrict__ out)
{
    using V = typename C2<T>::type;
    __shared__ double sh[4][4];
    for (int i = blockIdx.x; i < nregs; i += gridDim.x) {
        const BatchReg R = regs[i];
        const V* amp = (const V*)R.amp;
        const uint64_t len = 1ull << R.n;
        NSum s0 = {0.0, 0.0}, st = {0.0, 0.0};
        for (uint64_t e = threadIdx.x; e < len; e += 256) {
            const V a = amp[e];
            const double p = (double)a.x * (double)a.x + (double)a.y * (double)a.y;
            nadd(s0, ((e >> q) & 1) ? 0.0 : p);
            nadd(st, p);
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            s0 = nmerge(s0, NSum{__shfl_xor(s0.s, off, 64), __shfl_xor(s0.c, off, 64)});
            st = nmerge(st, NSum{__shfl_xor(st.s, off, 64), __shfl_xor(st.c, off, 64)});
        }
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
            sh[0][w] = s0.s;
            sh[1][w] = s0.c;
            sh[2][w] = st.s;
            sh[3][w] = st.c;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            NSum a = {sh[0][0], sh[1][0]}, b = {sh[2][0], sh[3][0]};
            for (int k = 1; k < 4; ++k) {
                a = nmerge(a, NSum{sh[0][k], sh[1][k]});
                b = nmerge(b, NSum{sh[2][k], sh[3][k]});
            }
            out[2 * i] = a.s + a.c;
            out[2 * i + 1] = b.s + b.c;
        }
        __syncthreads();
    }
}

void fill_phase(FPhase& F, const Layout& from, const Layout& to, int K)
{
    const std::vector<uint32_t> img = swizzle(from, to, K);
    memset(F.wthr, 0, sizeof(F.wthr));
    memset(F.wreg, 0, sizeof(F.wreg));
    memset(F.rthr, 0, sizeof(F.rthr));
    memset(F.rreg, 0, sizeof(F.rreg));
    for (size_t b = 0; b < from.thr.size(); ++b) F.wthr[b] = img[from.thr[b]];
    for (size_t b = 0; b < from.reg.size(); ++b) F.wreg[b] = img[from.reg[b]];
    for (size_t b = 0; b < to.thr.size(); ++b) F.rthr[b] = img[to.thr[b]];
    for (size_t b = 0; b < to.reg.size(); ++b) F.rreg[b] = img[to.reg[b]];
}

FOp encode_op(const OpRec& op, const PassPlan& P, const Layout& L)
{
    FOp f;
    memset(&f, 0, sizeof(f));
    std::vector<int> local(64, -1);
    for (size_t j = 0; j < P.S.size(); ++j) local[P.S[j]] = (int)j;
    auto classify = [&](int q) {
        const int j = local[q];
        if (j < 0) {
            f.gmask |= 1ull << q;
            return;
        }
        for (size_t b = 0; b < L.reg.size(); ++b)
            if (L.reg[b] == j) {
                f.rmask |= 1u << b;
                return;
            }
        for (size_t b = 0; b < L.thr.size(); ++b)
            if (L.thr[b] == j) {
                f.tmask |= 1u << b;
                return;
            }
    };
    for (int q : op.ctrls) classify(q);
    if (op.kind == 2) {
        f.kind = kPhase + (f.tmask ? 1 : 0);
        f.m[0] = cos(op.angle);
        f.m[1] = sin(op.angle);
        return f;
    }
    const int jt = local[op.target];
    for (size_t b = 0; b < L.reg.size(); ++b)
        if (L.reg[b] == jt) f.rb = (int)b;
    const int var = (f.rmask ? 1 : 0) | (f.tmask ? 2 : 0);
    const bool diag = op.kind == 0 && op.u[2] == 0.0 && op.u[3] == 0.0 && op.u[4] == 0.0 && op.u[5] == 0.0;
    f.kind = (op.kind == 0 ? (diag ? kDiag : kDense) : kNot) + 4 * f.rb + var;
    if (op.kind == 0)
        for (int k = 0; k < 8; ++k) f.m[k] = op.u[k];
    return f;
}

using Cx = std::complex<double>;

// Multiply the amplitudes whose register bits `rmask`, thread bits `tmask`
// and outside qubits `gmask` are all 1 by f.
FOp phase_fop(uint32_t rmask, uint32_t tmask, uint64_t gmask, Cx f)
{
    FOp o;
    memset(&o, 0, sizeof(o));
    o.kind = kPhase + (tmask ? 1 : 0);
    o.rmask = rmask;
    o.tmask = tmask;
    o.gmask = gmask;
    o.m[0] = f.real();
    o.m[1] = f.imag();
    return o;
}

// Diagonal factors deferred by the lowering (see lower_passes): the true
// state is gsc times prod_q exp(i phi[q] x_q) over the qubits with has[q],
// times the stored state.  Which qubits carry a factor, and whether gsc was
// touched, depends only on the op structure, not on matrix values, so a
// circuit with new parameters lowers to the same number of ops.
struct Defer {
    double phi[64] = {};
    bool has[64] = {};
    Cx gsc = 1.0;
    bool gsc_used = false;
    int shrink = 0;  // cores since gsc was last multiplied in
};

// Every core scales gsc by |d0| >= 1/sqrt 2, and the stored state grows by
// the inverse; after this many cores gsc is multiplied in (2^-30 keeps
// complex64 amplitudes far from overflow, 2^-500 complex128 ones).
inline int max_shrink(int prec) { return prec == QS_C128 ? 1000 : 60; }

// A dense 2x2 gate U written as diag(d0, d1) times a unit-diagonal core:
// form 2: U = diag(u00, u11) [[1, k], [-conj(k), 1]], k = u01 / u00;
// form 3: U = diag(u01, u10) [[k, 1], [1, -conj(k)]], k = u00 / u01;
// whichever has |k| <= 1.  Form 0: U diagonal; form 1: anti-diagonal.  Both
// identities need U unitary; form -1 when that fails by more than 1e-14.
struct CoreForm {
    int form;
    Cx k, d0, d1;
};

CoreForm core_form(const Cx (&u)[2][2])
{
    if (u[0][1] == 0.0 && u[1][0] == 0.0) return {0, 0.0, u[0][0], u[1][1]};
    if (u[0][0] == 0.0 && u[1][1] == 0.0) return {1, 0.0, u[0][1], u[1][0]};
    if (std::abs(u[0][0]) >= std::abs(u[0][1])) {
        const Cx k = u[0][1] / u[0][0];
        if (std::abs(u[1][0] + u[1][1] * std::conj(k)) > 1e-14) return {-1, 0.0, 0.0, 0.0};
        return {2, k, u[0][0], u[1][1]};
    }
    const Cx k = u[0][0] / u[0][1];
    if (std::abs(u[1][1] + u[1][0] * std::conj(k)) > 1e-14) return {-1, 0.0, 0.0, 0.0};
    return {3, k, u[0][1], u[1][0]};
}

// Device form of a planned pass list, appended to hp / hops / m4 (op
// indices in the phases are positions in hops; 4x4 ops index m4 in blocks
// of 32 values).  The ops are lowered on the way: an uncontrolled dense
// gate becomes its unit-diagonal core (half the multiply-adds) and its
// diagonal part, like every one-qubit phase, is deferred; the next dense or
// 4x4 op on that qubit takes the deferred phase into its matrix on the host
// (free), a NOT moves it, and the last pass multiplies in what is left.
void serialize(const std::vector<PassPlan>& plan, const std::vector<OpRec>& ops, int TB, int RB, int prec,
               std::vector<FPass>& hp, std::vector<FOp>& hops, std::vector<double>& m4)
{
    const int K = TB + RB;
    Defer d;
    for (size_t p = 0; p < plan.size(); ++p) {
        const PassPlan& P = plan[p];
        const bool last_pass = p + 1 == plan.size();
        std::vector<int> local(64, -1);
        for (int j = 0; j < K; ++j) local[P.S[j]] = j;
        FPass F;
        memset(&F, 0, sizeof(F));
        F.nphases = (int)P.phases.size();
        F.outside = make_insert(P.S.data(), (int)P.S.size(), 0);
        const Layout& L0 = P.phases.front().lay;
        for (int b = 0; b < TB; ++b) {
            F.ld_thr[b] = 1ull << P.S[L0.thr[b]];
            F.st_thr[b] = 1ull << P.S[P.store.thr[b]];
        }
        for (int b = 0; b < RB; ++b) {
            F.ld_reg[b] = 1ull << P.S[L0.reg[b]];
            F.st_reg[b] = 1ull << P.S[P.store.reg[b]];
        }
        for (size_t ph = 0; ph < P.phases.size(); ++ph) {
            FPhase& Fp = F.ph[ph];
            const Layout& L = P.phases[ph].lay;
            const Layout& prev = ph ? P.phases[ph - 1].lay : L;
            fill_phase(Fp, prev, L, K);
            Fp.op_begin = (int)hops.size();
            auto reg_bit = [&](int q) {
                for (int b = 0; b < RB; ++b)
                    if (L.reg[b] == local[q]) return b;
                return -1;
            };
            auto flush = [&](int q) {  // multiply in the deferred phase of register-bit qubit q
                if (!d.has[q]) return;
                hops.push_back(phase_fop(1u << reg_bit(q), 0, 0, std::polar(1.0, d.phi[q])));
                d.phi[q] = 0.0;
                d.has[q] = false;
            };
            for (int idx : P.phases[ph].ops) {
                const OpRec& op = ops[idx];
                if (op.kind == 2) {
                    if (op.ctrls.size() == 1 && local[op.ctrls[0]] >= 0) {
                        d.phi[op.ctrls[0]] += op.angle;
                        d.has[op.ctrls[0]] = true;
                    } else {
                        hops.push_back(encode_op(op, P, L));
                    }
                    continue;
                }
                if (op.kind == 4) {  // uncontrolled 4x4 on two register bits
                    const int q1 = op.target, q2 = op.target2;
                    int b1 = reg_bit(q1), b2 = reg_bit(q2);
                    Cx m[4][4];
                    for (int i = 0; i < 4; ++i)
                        for (int c = 0; c < 4; ++c) {
                            const double a = ((c & 1) && d.has[q1] ? d.phi[q1] : 0.0) +
                                             ((c & 2) && d.has[q2] ? d.phi[q2] : 0.0);
                            m[i][c] = Cx(op.m4[2 * (4 * i + c)], op.m4[2 * (4 * i + c) + 1]) * std::polar(1.0, a);
                        }
                    d.phi[q1] = d.phi[q2] = 0.0;
                    d.has[q1] = d.has[q2] = false;
                    if (b1 > b2) {  // index bit 0 belongs to b1: exchange the two index bits
                        Cx t[4][4];
                        const int sw[4] = {0, 2, 1, 3};
                        for (int i = 0; i < 4; ++i)
                            for (int c = 0; c < 4; ++c) t[sw[i]][sw[c]] = m[i][c];
                        for (int i = 0; i < 4; ++i)
                            for (int c = 0; c < 4; ++c) m[i][c] = t[i][c];
                        std::swap(b1, b2);
                    }
                    int pair = 0;
                    while (!(kPairB1[pair] == b1 && kPairB2[pair] == b2)) ++pair;
                    FOp f;
                    memset(&f, 0, sizeof(f));
                    f.kind = kDense4 + pair;
                    f.aux = (uint32_t)(m4.size() / 32);
                    for (int i = 0; i < 4; ++i)
                        for (int c = 0; c < 4; ++c) {
                            m4.push_back(m[i][c].real());
                            m4.push_back(m[i][c].imag());
                        }
                    hops.push_back(f);
                    continue;
                }
                FOp f = encode_op(op, P, L);
                const int t = op.target, b = f.rb;
                const bool uncond = f.rmask == 0 && f.tmask == 0 && f.gmask == 0;
                if (op.kind == 1) {
                    if (f.tmask || f.gmask) {  // lane- or tile-dependent exchange: no deferred phase across it
                        flush(t);
                        hops.push_back(f);
                        continue;
                    }
                    hops.push_back(f);
                    if (!d.has[t]) continue;
                    // X exp(i a x_t) = exp(i a) exp(-i a x_t) X where the controls hold
                    const double a = d.phi[t];
                    if (uncond) {
                        d.gsc *= std::polar(1.0, a);
                        d.gsc_used = true;
                        d.phi[t] = -a;
                    } else if (__builtin_popcount(f.rmask) == 1) {
                        // exp(i a (x_t xor x_c)) = exp(i a x_t) exp(i a x_c) exp(-2 i a x_t x_c)
                        const int c = P.S[L.reg[__builtin_ctz(f.rmask)]];
                        d.phi[c] += a;
                        d.has[c] = true;
                        hops.push_back(phase_fop(f.rmask | (1u << b), 0, 0, std::polar(1.0, -2.0 * a)));
                    } else {
                        hops.push_back(phase_fop(f.rmask, 0, 0, std::polar(1.0, a)));
                        hops.push_back(phase_fop(f.rmask | (1u << b), 0, 0, std::polar(1.0, -2.0 * a)));
                    }
                    continue;
                }
                // dense 2x2 (kind 0)
                Cx u[2][2];
                for (int i = 0; i < 2; ++i)
                    for (int c = 0; c < 2; ++c) u[i][c] = Cx(op.u[2 * (2 * i + c)], op.u[2 * (2 * i + c) + 1]);
                if (!uncond) {
                    flush(t);
                    hops.push_back(f);
                    continue;
                }
                if (d.has[t]) {
                    u[0][1] *= std::polar(1.0, d.phi[t]);
                    u[1][1] *= std::polar(1.0, d.phi[t]);
                }
                const CoreForm cf = core_form(u);
                if (cf.form < 0) {  // not unitary to 1e-14: the full matrix, phase folded in
                    for (int i = 0; i < 2; ++i)
                        for (int c = 0; c < 2; ++c) {
                            f.m[2 * (2 * i + c)] = u[i][c].real();
                            f.m[2 * (2 * i + c) + 1] = u[i][c].imag();
                        }
                    f.kind = kDense + 4 * b;
                    d.phi[t] = 0.0;
                    d.has[t] = false;
                    hops.push_back(f);
                    continue;
                }
                static const int kind_of[4] = {kNop, kNot, kCoreA, kCoreB};
                f.kind = kind_of[cf.form] + (cf.form == 0 ? 0 : 4 * b);
                for (int k = 0; k < 8; ++k) f.m[k] = 0.0;
                f.m[0] = cf.k.real();
                f.m[1] = cf.k.imag();
                hops.push_back(f);
                d.gsc *= cf.d0;
                d.gsc_used = true;
                d.phi[t] = std::arg(cf.d1 / cf.d0);
                d.has[t] = true;
                if (++d.shrink >= max_shrink(prec)) {  // a fixed point in the op structure
                    hops.push_back(phase_fop(0, 0, 0, d.gsc));
                    d.gsc = 1.0;
                    d.shrink = 0;
                }
            }
            if (last_pass && ph + 1 == P.phases.size()) {
                // multiply in every deferred factor, in the last layout
                for (int q = 0; q < 64; ++q) {
                    if (!d.has[q]) continue;
                    const Cx e = std::polar(1.0, d.phi[q]);
                    const int j = local[q];
                    if (j < 0) {
                        hops.push_back(phase_fop(0, 0, 1ull << q, e));
                    } else {
                        int rb = -1, tb = -1;
                        for (int b = 0; b < RB; ++b)
                            if (L.reg[b] == j) rb = b;
                        for (int b = 0; b < TB; ++b)
                            if (L.thr[b] == j) tb = b;
                        hops.push_back(rb >= 0 ? phase_fop(1u << rb, 0, 0, e) : phase_fop(0, 1u << tb, 0, e));
                    }
                    d.phi[q] = 0.0;
                    d.has[q] = false;
                }
                if (d.gsc_used) hops.push_back(phase_fop(0, 0, 0, d.gsc));
                d.gsc = 1.0;
                d.gsc_used = false;
            }
            Fp.op_end = (int)hops.size();
        }
        const Layout& last = P.phases.back().lay;
        F.final_transpose = (last.reg == P.store.reg && last.thr == P.store.thr) ? 0 : 1;
        fill_phase(F.fin, last, P.store, K);
        F.fin.op_begin = F.fin.op_end = 0;
        hp.push_back(F);
    }
}

// Tile shapes compiled in: (thread bits, register bits).  LDS holds the
// whole tile, so 2^K * element size <= 160 KiB.
struct Shape {
    int TB, RB;
};
// (8, 5) in complex128 would need 32 double2 registers per thread and spills
constexpr Shape kShapes128[] = {{6, 3}, {7, 3}, {8, 3}, {8, 4}, {9, 3}, {9, 4}, {10, 3}};
constexpr Shape kShapes64[] = {{6, 3}, {7, 3}, {8, 3}, {8, 4}, {9, 3}, {8, 5}, {9, 4}, {10, 3},
                               {9, 5}, {10, 4}};

template <typename T, int TB, int RB>
hipError_t launch_cfg(hipStream_t s, void* amp, const FPass* P, const FOp* ops, const void* m4, uint64_t ntiles)
{
    using V = typename C2<T>::type;
    uint64_t grid = ntiles;
    const uint64_t cap = 256ull * 16;
    if (grid > cap) grid = cap;
    hipLaunchKernelGGL((k_fused<T, TB, RB>), dim3((unsigned)grid), dim3(1 << TB), 0, s, (V*)amp, P, ops,
                       (const T*)m4, ntiles);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fused_pass(hipStream_t s, const FusedConfig& c, void* amp, const FPass* P, const FOp* ops,
                             const void* m4, uint64_t ntiles)
{
#define QS_SHAPE(tb, rb) \
    if (c.TB == tb && c.RB == rb) return launch_cfg<T, tb, rb>(s, amp, P, ops, m4, ntiles);
    QS_SHAPE(6, 3) QS_SHAPE(7, 3) QS_SHAPE(8, 3) QS_SHAPE(8, 4) QS_SHAPE(9, 3)
    QS_SHAPE(9, 4) QS_SHAPE(10, 3)
    if constexpr (sizeof(T) == 4) {
        QS_SHAPE(8, 5) QS_SHAPE(9, 5) QS_SHAPE(10, 4)
    }
#undef QS_SHAPE
    return hipErrorInvalidValue;
}

}  // namespace

bool fused_shape_supported(int prec, int TB, int RB)
{
    if (prec == QS_C128) {
        for (const Shape& sh : kShapes128)
            if (sh.TB == TB && sh.RB == RB) return true;
    } else {
        for (const Shape& sh : kShapes64)
            if (sh.TB == TB && sh.RB == RB) return true;
    }
    return false;
}

FusedConfig default_fused_config(int prec, int k, int n)
{
    int K = std::min(k, n);
    K = std::min(K, prec == QS_C128 ? 13 : 14);
    FusedConfig c{0, 0, kPhMax};
    if (K < 9) return c;
    static const int tb_of[15] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 6, 7, 8, 8, 8, 9};
    c.TB = tb_of[K];
    if (prec == QS_C128 && K == 13) c.TB = 9;  // 16 registers per thread, not 32
    c.RB = K - c.TB;
    return c;
}

// The 4x4 table in the register's precision.
std::vector<char> m4_bytes(const std::vector<double>& m4, int prec)
{
    std::vector<char> out;
    if (prec == QS_C128) {
        out.assign((const char*)m4.data(), (const char*)(m4.data() + m4.size()));
    } else {
        std::vector<float> f(m4.begin(), m4.end());
        out.assign((const char*)f.data(), (const char*)(f.data() + f.size()));
    }
    if (out.empty()) out.resize(sizeof(double));
    return out;
}

qs_status run_fused_sv(qs_reg r, const std::vector<OpRec>& circuit_ops, FusedConfig cfg, int* passes_out)
{
    if (cfg.max_phases <= 0 || cfg.max_phases > kPhMax) cfg.max_phases = kPhMax;
    const int nbits = r->nbits;
    if (cfg.TB == 0 || cfg.TB + cfg.RB > nbits) {  // too small to tile: one kernel per op
        for (const OpRec& op : circuit_ops) {
            qs_status s = apply_op(r, op);
            if (s) return s;
        }
        if (passes_out) *passes_out = (int)circuit_ops.size();
        return QS_OK;
    }
    // a density matrix runs as its 2N-qubit vector (Eq. 2): gates on q and
    // conj on q + N, channels as 4x4 superoperators on (q, q + N)
    std::vector<OpRec> dm_ops;
    if (r->kind == QS_DENSITY) dm_ops = dm_vector_ops(circuit_ops, r->n);
    const std::vector<OpRec>& ops = r->kind == QS_DENSITY ? dm_ops : circuit_ops;
    const int TB = cfg.TB, RB = cfg.RB, K = TB + RB;
    std::vector<PassPlan> plan = plan_passes(ops, nbits, TB, RB, cfg.max_phases, 1 << 12, std::min(4, TB));

    // serialise passes + ops
    std::vector<FPass> hp;
    std::vector<FOp> hops;
    std::vector<double> m4;
    serialize(plan, ops, TB, RB, r->prec, hp, hops, m4);
    if (hops.empty()) hops.push_back(FOp{});
    const std::vector<char> m4b = m4_bytes(m4, r->prec);

    const size_t pbytes = hp.size() * sizeof(FPass), obytes = hops.size() * sizeof(FOp);
    const size_t moff = (pbytes + obytes + 255) & ~(size_t)255;
    std::vector<char> host(moff + m4b.size());
    memcpy(host.data(), hp.data(), pbytes);
    memcpy(host.data() + pbytes, hops.data(), obytes);
    memcpy(host.data() + moff, m4b.data(), m4b.size());
    // stream-ordered plan buffer: no device-wide synchronisation, so
    // registers on other streams keep running
    void* dbuf = nullptr;
    hipError_t e = hipMallocAsync(&dbuf, host.size(), r->stream);
    if (e != hipSuccess) return hip_error(e, "plan buffer");
    // from pageable memory the copy has left `host` when the call returns
    e = hipMemcpyAsync(dbuf, host.data(), host.size(), hipMemcpyHostToDevice, r->stream);
    if (e != hipSuccess) {
        (void)hipFreeAsync(dbuf, r->stream);
        return hip_error(e, "plan upload");
    }
    const FPass* dP = (const FPass*)dbuf;
    const FOp* dO = (const FOp*)((char*)dbuf + pbytes);
    const void* dM = (const char*)dbuf + moff;
    const uint64_t ntiles = 1ull << (nbits - K);
    qs_status st = QS_OK;
    for (size_t p = 0; p < hp.size() && st == QS_OK; ++p) {
        st = profiled(r, QS_K_FUSED, [&](int*) {
            return r->prec == QS_C128 ? launch_fused_pass<double>(r->stream, cfg, r->amp, dP + p, dO, dM, ntiles)
                                      : launch_fused_pass<float>(r->stream, cfg, r->amp, dP + p, dO, dM, ntiles);
        });
    }
    // released once the passes that read it have run
    e = hipFreeAsync(dbuf, r->stream);
    if (st) return st;
    if (e != hipSuccess) return hip_error(e, "plan free");
    if (passes_out) *passes_out = (int)hp.size();
    return QS_OK;
}

// ===========================================================================
// Batched registers (one persistent launch)

namespace {

template <typename T, int TB, int RB>
hipError_t batch_launch_t(qs_batch_s* b, const qs_batch_s::Launch& L, int init)
{
    const char* base = (const char*)b->dbuf;
    const BatchItem* items = (const BatchItem*)(base + b->off_order);
    hipLaunchKernelGGL((k_batch<T, TB, RB>), dim3(std::min(L.count, L.grid)), dim3(1 << TB), 0, b->stream,
                       (const BatchReg*)(base + b->off_regs), items + L.off, L.count,
                       (const FPass*)(base + b->off_passes), (const FOp*)(base + b->off_ops),
                       (const T*)(base + b->off_m4), init);
    return hipGetLastError();
}

template <typename T>
hipError_t batch_launch_p(qs_batch_s* b, int init)
{
    for (const qs_batch_s::Launch& L : b->launches) {
        hipError_t e = hipErrorInvalidValue;
#define QS_B(tb, rb) \
    if (L.TB == tb && L.RB == rb) e = batch_launch_t<T, tb, rb>(b, L, init);
        QS_B(6, 3) QS_B(7, 3) QS_B(8, 3) QS_B(8, 4) QS_B(9, 3) QS_B(9, 4) QS_B(10, 3)
        if constexpr (sizeof(T) == 4) {
            QS_B(8, 5) QS_B(9, 5) QS_B(10, 4)
        }
#undef QS_B
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T, int TB, int RB>
int batch_occupancy()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch<T, TB, RB>, 1 << TB, 0) != hipSuccess) nb = 1;
    return nb < 1 ? 1 : nb;
}

template <typename T>
int batch_occupancy_p(int TB, int RB)
{
#define QS_O(tb, rb) \
    if (TB == tb && RB == rb) return batch_occupancy<T, tb, rb>();
    QS_O(6, 3) QS_O(7, 3) QS_O(8, 3) QS_O(8, 4) QS_O(9, 3) QS_O(9, 4) QS_O(10, 3)
    if constexpr (sizeof(T) == 4) {
        QS_O(8, 5) QS_O(9, 5) QS_O(10, 4)
    }
#undef QS_O
    return 1;
}

}  // namespace

struct BatchPlans {
    std::vector<std::vector<PassPlan>> plans;  // per register
    std::vector<bool> placeholder;             // an empty circuit's identity pass
};

void batch_plans_free(BatchPlans* p) { delete p; }

qs_status batch_build(qs_batch_s* b, const std::vector<qs_reg>& regs,
                      const std::vector<const std::vector<OpRec>*>& circs, int tile_qubits)
{
    int nmin = 64;
    for (qs_reg r : regs) nmin = std::min(nmin, r->n);
    const FusedConfig cfg = default_fused_config(b->prec, tile_qubits, 64);
    if (cfg.TB == 0 || nmin < 9)
        return set_error(QS_E_ARG, "batched registers need at least 9 qubits and a tile of 9 or more");
    b->TB = cfg.TB;
    b->RB = cfg.RB;
    std::vector<FPass> hp;
    std::vector<FOp> hops;
    std::vector<double> m4;
    std::vector<BatchReg> hr(regs.size());
    int maxpasses = 0;
    b->reg_TB.assign(regs.size(), 0);
    b->reg_RB.assign(regs.size(), 0);
    std::vector<uint64_t> per_item(regs.size());
    std::unique_ptr<BatchPlans> bp(new BatchPlans());
    b->reg_op_begin.assign(regs.size(), 0);
    b->reg_op_count.assign(regs.size(), 0);
    b->reg_m4_begin.assign(regs.size(), 0);
    b->reg_m4_count.assign(regs.size(), 0);
    for (size_t i = 0; i < regs.size(); ++i) {
        std::vector<OpRec> none;
        const std::vector<OpRec>* ops = circs[i];
        if (ops->empty()) {  // an empty circuit still gets one (identity) pass, which initialises
            OpRec id{};
            id.kind = 2;
            id.ctrls = {0};
            id.angle = 0.0;
            none.push_back(id);
            ops = &none;
        }
        // a register narrower than the batch tile is one tile of its own width
        const FusedConfig rc = regs[i]->n >= cfg.TB + cfg.RB ? cfg : default_fused_config(b->prec, regs[i]->n, regs[i]->n);
        b->reg_TB[i] = rc.TB;
        b->reg_RB[i] = rc.RB;
        std::vector<PassPlan> plan = plan_passes(*ops, regs[i]->n, rc.TB, rc.RB, kPhMax, 1 << 12, std::min(4, rc.TB));
        per_item[i] = 1ull << (regs[i]->n - (rc.TB + rc.RB));  // tile count, for now
        hr[i].amp = regs[i]->amp;
        hr[i].n = regs[i]->n;
        hr[i].pass0 = (uint32_t)hp.size();
        hr[i].npasses = (int)plan.size();
        hr[i].pad = 0;
        maxpasses = std::max(maxpasses, (int)plan.size());
        b->reg_op_begin[i] = hops.size();
        b->reg_m4_begin[i] = m4.size();
        serialize(plan, *ops, rc.TB, rc.RB, b->prec, hp, hops, m4);
        b->reg_op_count[i] = hops.size() - b->reg_op_begin[i];
        b->reg_m4_count[i] = m4.size() - b->reg_m4_begin[i];
        bp->plans.push_back(std::move(plan));
        bp->placeholder.push_back(ops == &none);
    }
    // tiles per work item: up to 16, fewer when the batch holds too few
    // tiles to give the 256 CUs about 8 items each
    uint64_t total_tiles = 0;
    for (uint64_t t : per_item) total_tiles += t;
    const uint64_t per = std::max<uint64_t>(1, std::min<uint64_t>(16, (total_tiles + 2047) / 2048));
    for (uint64_t& t : per_item) t = std::min(t, per);
    if (hp.empty()) hp.push_back(FPass{});
    if (hops.empty()) hops.push_back(FOp{});
    b->circ_ops.assign(circs.begin(), circs.end());
    b->host_ops.assign((const char*)hops.data(), (const char*)(hops.data() + hops.size()));
    b->host_m4 = m4;
    const std::vector<char> m4b = m4_bytes(m4, b->prec);
    // items level by level; within a level the largest registers first
    std::vector<uint32_t> byn(regs.size());
    for (size_t i = 0; i < byn.size(); ++i) byn[i] = (uint32_t)i;
    std::stable_sort(byn.begin(), byn.end(), [&](uint32_t a, uint32_t c) { return hr[a].n > hr[c].n; });
    std::vector<BatchItem> items;
    b->launches.clear();
    std::vector<std::pair<int, int>> shapes;  // distinct tile shapes, batch shape first
    shapes.push_back({cfg.TB, cfg.RB});
    for (size_t i = 0; i < regs.size(); ++i)
        if (std::find(shapes.begin(), shapes.end(), std::make_pair(b->reg_TB[i], b->reg_RB[i])) == shapes.end())
            shapes.push_back({b->reg_TB[i], b->reg_RB[i]});
    for (int p = 0; p < maxpasses; ++p) {
        for (const auto& sh : shapes) {
            const int off = (int)items.size();
            for (uint32_t i : byn) {
                if (p >= hr[i].npasses || b->reg_TB[i] != sh.first || b->reg_RB[i] != sh.second) continue;
                const uint64_t ntiles = 1ull << (hr[i].n - (sh.first + sh.second)), per = per_item[i];
                for (uint64_t t0 = 0; t0 < ntiles; t0 += per)
                    items.push_back(BatchItem{i, (uint32_t)p, (uint32_t)t0, (uint32_t)std::min(ntiles, t0 + per)});
            }
            const int count = (int)items.size() - off;
            if (count == 0) continue;
            const int per_cu = b->prec == QS_C128 ? batch_occupancy_p<double>(sh.first, sh.second)
                                                  : batch_occupancy_p<float>(sh.first, sh.second);
            b->launches.push_back({sh.first, sh.second, off, count, (int)(256L * per_cu)});
        }
    }
    b->nitems = (int)items.size();
    auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
    b->off_regs = 0;
    b->off_order = align(hr.size() * sizeof(BatchReg));
    b->off_passes = align(b->off_order + items.size() * sizeof(BatchItem));
    b->off_ops = align(b->off_passes + hp.size() * sizeof(FPass));
    b->off_m4 = align(b->off_ops + hops.size() * sizeof(FOp));
    const size_t total = align(b->off_m4 + m4b.size());
    std::vector<char> host(total, 0);
    memcpy(host.data() + b->off_regs, hr.data(), hr.size() * sizeof(BatchReg));
    memcpy(host.data() + b->off_order, items.data(), items.size() * sizeof(BatchItem));
    memcpy(host.data() + b->off_passes, hp.data(), hp.size() * sizeof(FPass));
    memcpy(host.data() + b->off_ops, hops.data(), hops.size() * sizeof(FOp));
    memcpy(host.data() + b->off_m4, m4b.data(), m4b.size());
    // stream-ordered allocation and upload: creating a batch does not wait
    // for work on other streams (a plain free or a synchronous copy would)
    b->host_plan = std::move(host);
    hipError_t e = hipMallocAsync(&b->dbuf, total, b->stream);
    if (e != hipSuccess) return hip_error(e, "batch plan buffer");
    e = hipMemcpyAsync(b->dbuf, b->host_plan.data(), total, hipMemcpyHostToDevice, b->stream);
    if (e != hipSuccess) return hip_error(e, "batch plan upload");
    b->grid = b->launches.empty() ? 1 : b->launches.front().grid;
    b->passes_total = (int)hp.size();
    b->plans = bp.release();
    return QS_OK;
}

qs_status batch_update(qs_batch_s* b)
{
    // lower every register's plan again with the circuits' current values:
    // the structure (and so the op count) is unchanged, only the kernel data
    // (matrices, core coefficients, deferred phases) follows the parameters
    FOp* ops = (FOp*)b->host_ops.data();
    for (size_t i = 0; i < b->regs.size(); ++i) {
        if (b->plans->placeholder[i]) continue;
        std::vector<FPass> hp;
        std::vector<FOp> hops;
        std::vector<double> m4;
        serialize(b->plans->plans[i], *b->circ_ops[i], b->reg_TB[i], b->reg_RB[i], b->prec, hp, hops, m4);
        if (hops.size() != b->reg_op_count[i] || m4.size() != b->reg_m4_count[i])
            return set_error(QS_E_ARG, "a batched circuit changed its structure");
        for (size_t k = 0; k < hops.size(); ++k) {
            FOp f = hops[k];
            if (f.kind >= kDense4 && f.kind < kDense4 + 10) f.aux += (uint32_t)(b->reg_m4_begin[i] / 32);
            ops[b->reg_op_begin[i] + k] = f;
        }
        std::copy(m4.begin(), m4.end(), b->host_m4.begin() + b->reg_m4_begin[i]);
    }
    // from pageable memory the copies have left the host tables when the
    // calls return; on the batch stream they follow earlier runs and precede
    // later ones
    hipError_t e = hipMemcpyAsync((char*)b->dbuf + b->off_ops, b->host_ops.data(), b->host_ops.size(),
                                  hipMemcpyHostToDevice, b->stream);
    if (e != hipSuccess) return hip_error(e, "batch parameter upload");
    if (!b->host_m4.empty()) {
        b->host_m4b = m4_bytes(b->host_m4, b->prec);
        e = hipMemcpyAsync((char*)b->dbuf + b->off_m4, b->host_m4b.data(), b->host_m4b.size(), hipMemcpyHostToDevice,
                           b->stream);
        if (e != hipSuccess) return hip_error(e, "batch parameter upload");
    }
    return QS_OK;
}

hipError_t batch_launch(qs_batch_s* b, int init)
{
    return b->prec == QS_C128 ? batch_launch_p<double>(b, init) : batch_launch_p<float>(b, init);
}

hipError_t batch_probs_launch(qs_batch_s* b, int q, double* dev_out)
{
    const BatchReg* regs = (const BatchReg*)((const char*)b->dbuf + b->off_regs);
    const int grid = std::min(b->count, 2048);
    if (b->prec == QS_C128)
        hipLaunchKernelGGL(k_batch_probs<double>, dim3(grid), dim3(256), 0, b->stream, regs, b->count, q, dev_out);
    else
        hipLaunchKernelGGL(k_batch_probs<float>, dim3(grid), dim3(256), 0, b->stream, regs, b->count, q, dev_out);
    return hipGetLastError();
}

}  // namespace qs
