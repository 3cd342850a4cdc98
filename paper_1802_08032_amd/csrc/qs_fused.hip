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
            const bool pc = ((uint32_t)r0 & rmask) == rmask;
            T mm[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) mm[k] = pc ? m[k] : ident<T>(k);
            apply2<T, V>(mm, v[r0], v[r0 | (1 << RBIT)]);
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
        bool c = true;
        if constexpr (MASKED) c = ((uint32_t)r0 & rmask) == rmask;
        if constexpr (LANE) c = c && sel;
        if constexpr (!MASKED && !LANE) {
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
    for (int r = 0; r < (1 << RB); ++r) {
        const bool pc = ((uint32_t)r & rmask) == rmask;
        const T ar = pc ? fr : T(1), ai = pc ? fi : T(0);
        v[r] = cmul<T, V>(ar, ai, v[r]);
    }
}

// Op codes: the host specialises every op so that the device dispatches with
// one switch and each case is straight-line code.
//   code = 4 * rb + variant        dense gate (variant: bit 0 register controls,
//                                  bit 1 thread-bit controls)
//   code = 32 + 4 * rb + variant   NOT
//   code = 64 + lane               phase (lane: thread-bit controls present)
enum : int { kDense = 0, kNot = 32, kPhase = 64 };

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
    case kNot + 4 * RBIT + 3: if constexpr (RB > RBIT) not_case<T, RB, RBIT, 3>(v, op, tid); break;
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

template <typename T, int TB, int RB>
__global__ __launch_bounds__(1 << TB) void k_fused(typename C2<T>::type* __restrict__ amp,
                                                   const FPass* __restrict__ P,
                                                   const FOp* __restrict__ ops, uint64_t ntiles)
{
    using V = typename C2<T>::type;
    constexpr int E = 1 << RB;
    __shared__ V lds[1 << (TB + RB)];
    const uint32_t tid = threadIdx.x;
    const uint64_t ld_t = span_sum<TB, uint64_t>(tid, P->ld_thr);
    const uint64_t st_t = span_sum<TB, uint64_t>(tid, P->st_thr);
    const int nph = P->nphases;
    for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint64_t base = expand(tile, P->outside);
        V v[E];
#pragma unroll
        for (int r = 0; r < E; ++r) v[r] = amp[base + ld_t + span_sum<RB, uint64_t>((uint32_t)r, P->ld_reg)];
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
    f.kind = (op.kind == 0 ? kDense : kNot) + 4 * f.rb + var;
    if (op.kind == 0)
        for (int k = 0; k < 8; ++k) f.m[k] = op.u[k];
    return f;
}

// Tile shapes compiled in: (thread bits, register bits).  LDS holds the
// whole tile, so 2^K * element size <= 160 KiB.
struct Shape {
    int TB, RB;
};
constexpr Shape kShapes128[] = {{6, 3}, {7, 3}, {8, 3}, {8, 4}, {9, 3}, {8, 5}, {9, 4}, {10, 3}};
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
    QS_SHAPE(8, 5) QS_SHAPE(9, 4) QS_SHAPE(10, 3)
    if constexpr (sizeof(T) == 4) {
        QS_SHAPE(9, 5) QS_SHAPE(10, 4)
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
    std::vector<PassPlan> plan = plan_passes(ops, r->n, TB, RB, cfg.max_phases, 1 << 12, 6);

    // serialise passes + ops
    std::vector<FPass> hp(plan.size());
    std::vector<FOp> hops;
    for (size_t p = 0; p < plan.size(); ++p) {
        const PassPlan& P = plan[p];
        FPass& F = hp[p];
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
            for (int idx : P.phases[ph].ops) hops.push_back(encode_op(ops[idx], P, P.phases[ph].lay));
            Fp.op_end = (int)hops.size();
        }
        const Layout& last = P.phases.back().lay;
        F.final_transpose = (last.reg == P.store.reg && last.thr == P.store.thr) ? 0 : 1;
        fill_phase(F.fin, last, P.store, K);
        F.fin.op_begin = F.fin.op_end = 0;
    }
    if (hops.empty()) hops.push_back(FOp{});

    const size_t pbytes = hp.size() * sizeof(FPass), obytes = hops.size() * sizeof(FOp);
    std::vector<char> host(pbytes + obytes);
    memcpy(host.data(), hp.data(), pbytes);
    memcpy(host.data() + pbytes, hops.data(), obytes);
    void* dbuf = nullptr;
    hipError_t e = hipMalloc(&dbuf, pbytes + obytes);
    if (e != hipSuccess) return hip_error(e, "plan buffer");
    e = hipMemcpy(dbuf, host.data(), pbytes + obytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        hipFree(dbuf);
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
    // the plan buffer is released once the passes that read it have finished
    e = hipStreamSynchronize(r->stream);
    hipFree(dbuf);
    if (st) return st;
    if (e != hipSuccess) return hip_error(e, "fused passes");
    if (passes_out) *passes_out = (int)hp.size();
    return QS_OK;
}

}  // namespace qs
