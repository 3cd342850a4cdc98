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
    int rb;          // target register bit (dense / not)
    uint32_t rmask;  // register bits that must be 1
    uint32_t tmask;  // thread-index bits that must be 1
    uint64_t gmask;  // global qubits outside the tile that must be 1
    double m[8];     // dense matrix, or phase factor in m[0], m[1]
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
enum : int { kDense = 0, kNot = 32, kPhase = 64, kDiag = 96 };

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
__device__ __forceinline__ void apply_op(typename C2<T>::type (&v)[1 << RB], const FOp& op, uint32_t tid)
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
                                             const FOp* __restrict__ ops, uint64_t tile,
                                             typename C2<T>::type* lds, uint32_t tid, bool zero_init = false)
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
            apply_op<T, RB>(v, op, tid);
        }
    }
    if (P->final_transpose) relayout<T, TB, RB>(v, lds, P->fin, tid);
#pragma unroll
    for (int r = 0; r < E; ++r) amp[base + st_t + span_sum<RB, uint64_t>((uint32_t)r, P->st_reg)] = v[r];
}

template <typename T, int TB, int RB>
__global__ __launch_bounds__(1 << TB) void k_fused(typename C2<T>::type* __restrict__ amp,
                                                   const FPass* __restrict__ P,
                                                   const FOp* __restrict__ ops, uint64_t ntiles)
{
    using V = typename C2<T>::type;
    __shared__ V lds[1 << (TB + RB)];
    for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x)
        process_tile<T, TB, RB>(amp, P, ops, tile, lds, threadIdx.x);
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
                                                   const FOp* __restrict__ ops, int init)
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
            process_tile<T, TB, RB>((V*)R.amp, P, ops, tile, lds, tid, zi);
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

// Device form of a planned pass list, appended to hp / hops (op indices in
// the phases are positions in hops).
void serialize(const std::vector<PassPlan>& plan, const std::vector<OpRec>& ops, int TB, int RB,
               std::vector<FPass>& hp, std::vector<FOp>& hops, std::vector<int>* src = nullptr)
{
    const int K = TB + RB;
    for (size_t p = 0; p < plan.size(); ++p) {
        const PassPlan& P = plan[p];
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
            const Layout& prev = ph ? P.phases[ph - 1].lay : P.phases[ph].lay;
            fill_phase(Fp, prev, P.phases[ph].lay, K);
            Fp.op_begin = (int)hops.size();
            for (int idx : P.phases[ph].ops) {
                hops.push_back(encode_op(ops[idx], P, P.phases[ph].lay));
                if (src) src->push_back(idx);
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
hipError_t launch_cfg(hipStream_t s, void* amp, const FPass* P, const FOp* ops, uint64_t ntiles)
{
    using V = typename C2<T>::type;
    uint64_t grid = ntiles;
    const uint64_t cap = 256ull * 16;
    if (grid > cap) grid = cap;
    hipLaunchKernelGGL((k_fused<T, TB, RB>), dim3((unsigned)grid), dim3(1 << TB), 0, s, (V*)amp, P, ops, ntiles);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fused_pass(hipStream_t s, const FusedConfig& c, void* amp, const FPass* P, const FOp* ops,
                             uint64_t ntiles)
{
#define QS_SHAPE(tb, rb) \
    if (c.TB == tb && c.RB == rb) return launch_cfg<T, tb, rb>(s, amp, P, ops, ntiles);
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

qs_status run_fused_sv(qs_reg r, const std::vector<OpRec>& ops, FusedConfig cfg, int* passes_out)
{
    if (cfg.max_phases <= 0 || cfg.max_phases > kPhMax) cfg.max_phases = kPhMax;
    if (cfg.TB == 0 || cfg.TB + cfg.RB > r->n) {  // too small to tile: one kernel per op
        for (const OpRec& op : ops) {
            qs_status s = apply_op(r, op);
            if (s) return s;
        }
        if (passes_out) *passes_out = (int)ops.size();
        return QS_OK;
    }
    const int TB = cfg.TB, RB = cfg.RB, K = TB + RB;
    std::vector<PassPlan> plan = plan_passes(ops, r->n, TB, RB, cfg.max_phases, 1 << 12, std::min(4, TB));

    // serialise passes + ops
    std::vector<FPass> hp;
    std::vector<FOp> hops;
    serialize(plan, ops, TB, RB, hp, hops);
    if (hops.empty()) hops.push_back(FOp{});

    const size_t pbytes = hp.size() * sizeof(FPass), obytes = hops.size() * sizeof(FOp);
    std::vector<char> host(pbytes + obytes);
    memcpy(host.data(), hp.data(), pbytes);
    memcpy(host.data() + pbytes, hops.data(), obytes);
    // stream-ordered plan buffer: no device-wide synchronisation, so
    // registers on other streams keep running
    void* dbuf = nullptr;
    hipError_t e = hipMallocAsync(&dbuf, pbytes + obytes, r->stream);
    if (e != hipSuccess) return hip_error(e, "plan buffer");
    // from pageable memory the copy has left `host` when the call returns
    e = hipMemcpyAsync(dbuf, host.data(), pbytes + obytes, hipMemcpyHostToDevice, r->stream);
    if (e != hipSuccess) {
        (void)hipFreeAsync(dbuf, r->stream);
        return hip_error(e, "plan upload");
    }
    const FPass* dP = (const FPass*)dbuf;
    const FOp* dO = (const FOp*)((char*)dbuf + pbytes);
    const uint64_t ntiles = 1ull << (r->n - K);
    qs_status st = QS_OK;
    for (size_t p = 0; p < hp.size() && st == QS_OK; ++p) {
        st = profiled(r, QS_K_FUSED, [&](int*) {
            return r->prec == QS_C128 ? launch_fused_pass<double>(r->stream, cfg, r->amp, dP + p, dO, ntiles)
                                      : launch_fused_pass<float>(r->stream, cfg, r->amp, dP + p, dO, ntiles);
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
hipError_t batch_launch_t(qs_batch_s* b, int init)
{
    const char* base = (const char*)b->dbuf;
    const BatchItem* items = (const BatchItem*)(base + b->off_order);
    for (size_t p = 0; p < b->level_off.size(); ++p) {
        const int count = b->level_count[p];
        if (count == 0) continue;
        const int grid = std::min(count, b->grid);
        hipLaunchKernelGGL((k_batch<T, TB, RB>), dim3(grid), dim3(1 << TB), 0, b->stream,
                           (const BatchReg*)(base + b->off_regs), items + b->level_off[p], count,
                           (const FPass*)(base + b->off_passes), (const FOp*)(base + b->off_ops), init);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T>
hipError_t batch_launch_p(qs_batch_s* b, int init)
{
#define QS_B(tb, rb) \
    if (b->TB == tb && b->RB == rb) return batch_launch_t<T, tb, rb>(b, init);
    QS_B(6, 3) QS_B(7, 3) QS_B(8, 3) QS_B(8, 4) QS_B(9, 3) QS_B(9, 4) QS_B(10, 3)
    if constexpr (sizeof(T) == 4) {
        QS_B(8, 5) QS_B(9, 5) QS_B(10, 4)
    }
#undef QS_B
    return hipErrorInvalidValue;
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

qs_status batch_build(qs_batch_s* b, const std::vector<qs_reg>& regs,
                      const std::vector<const std::vector<OpRec>*>& circs, int tile_qubits)
{
    b->op_src.clear();
    int nmin = 64;
    for (qs_reg r : regs) nmin = std::min(nmin, r->n);
    const FusedConfig cfg = default_fused_config(b->prec, tile_qubits, nmin);
    if (cfg.TB == 0 || cfg.TB + cfg.RB > nmin)
        return set_error(QS_E_ARG, "batched registers need at least 9 qubits and a tile no wider than the smallest");
    b->TB = cfg.TB;
    b->RB = cfg.RB;
    std::vector<FPass> hp;
    std::vector<FOp> hops;
    std::vector<BatchReg> hr(regs.size());
    const int contig = std::min(4, cfg.TB);
    const int K = cfg.TB + cfg.RB;
    int maxpasses = 0;
    std::vector<uint64_t> per_item(regs.size());
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
        std::vector<PassPlan> plan = plan_passes(*ops, regs[i]->n, cfg.TB, cfg.RB, kPhMax, 1 << 12, contig);
        const uint64_t ntiles = 1ull << (regs[i]->n - K);
        per_item[i] = std::max<uint64_t>(1, std::min<uint64_t>(16, ntiles));  // tiles per item
        hr[i].amp = regs[i]->amp;
        hr[i].n = regs[i]->n;
        hr[i].pass0 = (uint32_t)hp.size();
        hr[i].npasses = (int)plan.size();
        hr[i].pad = 0;
        maxpasses = std::max(maxpasses, (int)plan.size());
        std::vector<int> src;
        serialize(plan, *ops, cfg.TB, cfg.RB, hp, hops, &src);
        // the placeholder of an empty circuit has no source op: updates skip it
        for (int idx : src) b->op_src.push_back(ops == &none ? std::make_pair(-1, -1) : std::make_pair((int)i, idx));
    }
    if (hp.empty()) hp.push_back(FPass{});
    if (hops.empty()) {
        hops.push_back(FOp{});
        b->op_src.push_back({-1, -1});
    }
    b->circ_ops.assign(circs.begin(), circs.end());
    b->host_ops.assign((const char*)hops.data(), (const char*)(hops.data() + hops.size()));
    // items level by level; within a level the largest registers first
    std::vector<uint32_t> byn(regs.size());
    for (size_t i = 0; i < byn.size(); ++i) byn[i] = (uint32_t)i;
    std::stable_sort(byn.begin(), byn.end(), [&](uint32_t a, uint32_t c) { return hr[a].n > hr[c].n; });
    std::vector<BatchItem> items;
    b->level_off.clear();
    b->level_count.clear();
    for (int p = 0; p < maxpasses; ++p) {
        b->level_off.push_back((int)items.size());
        for (uint32_t i : byn) {
            if (p >= hr[i].npasses) continue;
            const uint64_t ntiles = 1ull << (hr[i].n - K), per = per_item[i];
            for (uint64_t t0 = 0; t0 < ntiles; t0 += per)
                items.push_back(BatchItem{i, (uint32_t)p, (uint32_t)t0, (uint32_t)std::min(ntiles, t0 + per)});
        }
        b->level_count.push_back((int)items.size() - b->level_off.back());
    }
    b->nitems = (int)items.size();
    auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
    b->off_regs = 0;
    b->off_order = align(hr.size() * sizeof(BatchReg));
    b->off_passes = align(b->off_order + items.size() * sizeof(BatchItem));
    b->off_ops = align(b->off_passes + hp.size() * sizeof(FPass));
    const size_t total = align(b->off_ops + hops.size() * sizeof(FOp));
    std::vector<char> host(total, 0);
    memcpy(host.data() + b->off_regs, hr.data(), hr.size() * sizeof(BatchReg));
    memcpy(host.data() + b->off_order, items.data(), items.size() * sizeof(BatchItem));
    memcpy(host.data() + b->off_passes, hp.data(), hp.size() * sizeof(FPass));
    memcpy(host.data() + b->off_ops, hops.data(), hops.size() * sizeof(FOp));
    hipError_t e = hipMalloc(&b->dbuf, total);
    if (e != hipSuccess) return hip_error(e, "batch plan buffer");
    e = hipMemcpy(b->dbuf, host.data(), total, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_error(e, "batch plan upload");
    const int per_cu = b->prec == QS_C128 ? batch_occupancy_p<double>(cfg.TB, cfg.RB)
                                          : batch_occupancy_p<float>(cfg.TB, cfg.RB);
    b->grid = (int)(256L * per_cu);
    b->passes_total = (int)hp.size();
    return QS_OK;
}

qs_status batch_update(qs_batch_s* b)
{
    FOp* ops = (FOp*)b->host_ops.data();
    const size_t n = b->host_ops.size() / sizeof(FOp);
    for (size_t k = 0; k < n; ++k) {
        const int ci = b->op_src[k].first, oi = b->op_src[k].second;
        if (ci < 0) continue;
        const std::vector<OpRec>& cops = *b->circ_ops[ci];
        if (oi >= (int)cops.size()) return set_error(QS_E_ARG, "a batched circuit lost operations");
        const OpRec& op = cops[oi];
        FOp& f = ops[k];
        if (op.kind == 2) {
            f.m[0] = cos(op.angle);
            f.m[1] = sin(op.angle);
        } else if (op.kind == 0) {
            // the dense / diagonal choice follows the new matrix; register
            // bit and condition variant (the low 5 bits) stay
            const bool diag = op.u[2] == 0.0 && op.u[3] == 0.0 && op.u[4] == 0.0 && op.u[5] == 0.0;
            f.kind = (diag ? kDiag : kDense) + (f.kind & 31);
            for (int q = 0; q < 8; ++q) f.m[q] = op.u[q];
        }
    }
    // from pageable memory the copy has left host_ops when the call returns;
    // on the batch stream it follows earlier runs and precedes later ones
    const hipError_t e = hipMemcpyAsync((char*)b->dbuf + b->off_ops, b->host_ops.data(), b->host_ops.size(),
                                        hipMemcpyHostToDevice, b->stream);
    if (e != hipSuccess) return hip_error(e, "batch parameter upload");
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
