// Run-time specialised fused passes.  For a planned pass (tile qubits,
// register layouts, ops) this file writes the HIP source of one kernel in
// which every op is unrolled with compile-time register indices and literal
// HBM / LDS offsets, compiles it for gfx950 with hipRTC, and caches the
// code object per source text.  Compared with the generic fused kernel
// (qs_fused.hip) there is no op interpreter: NOTs whose controls are all
// register bits become register renames, register-bit controls select
// pairs at compile time, and the compiler schedules across consecutive
// gates.  Gate matrices stay kernel data, so circuits that differ only in
// angles or unitaries reuse the same code.
#include <hip/hiprtc.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/stat.h>

#include <algorithm>
#include <atomic>
#include <complex>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "qs_plan.h"

namespace qs {
namespace {

// Diagonal factors deferred from pass to pass: the true state is gsc times
// prod_q mul[q]^(x_q) (over global qubits q with has[q]) times the stored
// state.
struct Deferred {
    std::complex<double> mul[64];
    bool has[64] = {};
    std::complex<double> gsc = 1.0;
    Deferred()
    {
        for (std::complex<double>& m : mul) m = 1.0;
    }
};

struct GenOut {
    std::string src;
    std::vector<double> mats;  // kernel data: matrices, core coefficients, phases
    bool bad = false;          // a relayout's swizzle broke the address split
    Deferred out;              // deferred factors after the pass
};

std::string hex64(uint64_t v)
{
    char b[32];
    snprintf(b, sizeof b, "0x%llxull", (unsigned long long)v);
    return b;
}

std::string hex32(uint32_t v)
{
    char b[24];
    snprintf(b, sizeof b, "0x%xu", v);
    return b;
}

// Sum (or XOR) over the thread-index bits b of img[b], as a C expression.
std::string tid_expr(const std::vector<uint64_t>& img, bool use_xor, bool wide)
{
    std::ostringstream o;
    o << "(";
    for (size_t b = 0; b < img.size(); ++b) {
        if (b) o << (use_xor ? " ^ " : " + ");
        o << "((tid & " << (1u << b) << "u) ? " << (wide ? hex64(img[b]) : hex32((uint32_t)img[b])) << " : "
          << (wide ? "0ull" : "0u") << ")";
    }
    o << ")";
    return o.str();
}

const char* kPrelude = R"(
__device__ __forceinline__ void qs_ap(const R (&m)[8], V& a, V& b)
{
    V na, nb;
    na.x = m[0] * a.x - m[1] * a.y + m[2] * b.x - m[3] * b.y;
    na.y = m[0] * a.y + m[1] * a.x + m[2] * b.y + m[3] * b.x;
    nb.x = m[4] * a.x - m[5] * a.y + m[6] * b.x - m[7] * b.y;
    nb.y = m[4] * a.y + m[5] * a.x + m[6] * b.y + m[7] * b.x;
    a = na;
    b = nb;
}
// LDS-only workgroup barrier: waits for this wave's LDS traffic, not for
// its outstanding global loads (the prefetch of the next tile).
#define QS_BAR() asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory")
// Wave-level ordering for a re-layout whose data stays within each wave:
// the LDS operations of one wave complete in order, so waiting for them is
// enough.
#define QS_WBAR() asm volatile("s_waitcnt lgkmcnt(0)\n" ::: "memory")
// 4x4 complex matrix on (a, b, c, d) = index bit(t1) + 2 bit(t2).
__device__ __forceinline__ void qs_ap4(const R (&m)[32], V& a, V& b, V& c, V& d)
{
    const V x[4] = {a, b, c, d};
    V y[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        // one product or multiply-add per statement, so that every term is
        // a fused multiply-add (1 multiply + 7 FMAs per component; an
        // accumulation of two-product terms costs 4 multiplies, 4 FMAs and
        // 4 adds)
        R re = m[8 * i] * x[0].x;
        R im = m[8 * i] * x[0].y;
        re = -m[8 * i + 1] * x[0].y + re;
        im = m[8 * i + 1] * x[0].x + im;
#pragma unroll
        for (int j = 1; j < 4; ++j) {
            const R mr = m[2 * (4 * i + j)], mi = m[2 * (4 * i + j) + 1];
            re = mr * x[j].x + re;
            re = -mi * x[j].y + re;
            im = mr * x[j].y + im;
            im = mi * x[j].x + im;
        }
        y[i].x = re;
        y[i].y = im;
    }
    a = y[0];
    b = y[1];
    c = y[2];
    d = y[3];
}
typedef R VE __attribute__((ext_vector_type(2)));
__device__ __forceinline__ V qs_ldnt(const V* p)
{
    const VE e = __builtin_nontemporal_load((const VE*)p);
    V v;
    v.x = e.x;
    v.y = e.y;
    return v;
}
__device__ __forceinline__ void qs_stnt(V v, V* p)
{
    VE e;
    e.x = v.x;
    e.y = v.y;
    __builtin_nontemporal_store(e, (VE*)p);
}
__device__ __forceinline__ void qs_cm(R fr, R fi, V& a)
{
    V r;
    r.x = fr * a.x - fi * a.y;
    r.y = fr * a.y + fi * a.x;
    a = r;
}
// Unit-diagonal core of a unitary gate: (a, b) <- (a + k b, b - conj(k) a),
// k = kr + i ki; two multiply-adds per output component.
__device__ __forceinline__ void qs_core(R kr, R ki, V& a, V& b)
{
    V na, nb;
    na.x = kr * b.x + a.x;
    na.x = -ki * b.y + na.x;
    na.y = kr * b.y + a.y;
    na.y = ki * b.x + na.y;
    nb.x = -kr * a.x + b.x;
    nb.x = -ki * a.y + nb.x;
    nb.y = -kr * a.y + b.y;
    nb.y = ki * a.x + nb.y;
    a = na;
    b = nb;
}
// Unit-diagonal core of any 2x2 matrix: (a, b) <- (a + k0 b, b + k1 a),
// k0 = k0r + i k0i, k1 = k1r + i k1i.
__device__ __forceinline__ void qs_core_g(R k0r, R k0i, R k1r, R k1i, V& a, V& b)
{
    V na, nb;
    na.x = k0r * b.x + a.x;
    na.x = -k0i * b.y + na.x;
    na.y = k0r * b.y + a.y;
    na.y = k0i * b.x + na.y;
    nb.x = k1r * a.x + b.x;
    nb.x = -k1i * a.y + nb.x;
    nb.y = k1r * a.y + b.y;
    nb.y = k1i * a.x + nb.y;
    a = na;
    b = nb;
}
// Unit-diagonal core of a 4x4 gate: x_i <- x_i + sum_{j != i} c_ij x_j for
// the four members at once; c holds the twelve c_ij row by row (j != i),
// real and imaginary parts interleaved.
__device__ __forceinline__ void qs_core4(const R (&c)[24], V& a, V& b, V& d, V& e)
{
    const V x[4] = {a, b, d, e};
    V y[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        R re = x[i].x, im = x[i].y;
        int k = 6 * i;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (j == i) continue;
            re = c[k] * x[j].x + re;
            re = -c[k + 1] * x[j].y + re;
            im = c[k] * x[j].y + im;
            im = c[k + 1] * x[j].x + im;
            k += 2;
        }
        y[i].x = re;
        y[i].y = im;
    }
    a = y[0];
    b = y[1];
    d = y[2];
    e = y[3];
}
// A kernel-data value kept in scalar registers: selecting between two such
// values per lane then costs a select, not a per-lane load.
__device__ __forceinline__ R qs_s(R x)
{
    asm("" : "+s"(x));
    return x;
}
// Amplitude i of the basis state |idx>.
__device__ __forceinline__ V qs_basis(unsigned long long i, unsigned long long idx)
{
    V v;
    v.x = i == idx ? (R)1 : (R)0;
    v.y = (R)0;
    return v;
}
)";

using Cx = std::complex<double>;

// `in`: factors deferred by earlier passes.  `last_pass`: multiply every
// deferred factor in before storing (otherwise the per-qubit factors are
// handed on in GenOut::out).  `readout_n` > 0 (last pass of an n-qubit state
// vector): the pass also sums, as it stores the final state, the total
// probability and P(qubit q = 0) for every q, per workgroup into
// part[blockIdx.x * (n + 1) + 0 .. n] (the total first).
GenOut generate(const PassPlan& P, const std::vector<OpRec>& all, int TB, int RB, bool dbl, bool init,
                const Deferred& in, bool last_pass, int readout_n)
{
    const int K = TB + RB, E = 1 << RB;
    GenOut g;
    std::ostringstream s;     // loop body: the ops
    std::ostringstream head;  // kernel header and prologue
    head << (dbl ? "typedef double R;\ntypedef double2 V;\n" : "typedef float R;\ntypedef float2 V;\n");
    head << kPrelude;
    head << "extern \"C\" __global__ void __launch_bounds__(" << (1 << TB)
         << ") qs_pass(V* __restrict__ amp, const R* __restrict__ mats, unsigned long long ntiles"
         << (init ? ", unsigned long long init_index" : "") << (readout_n > 0 ? ", double* __restrict__ part" : "")
         << ")\n{\n";
    head << "    __shared__ V lds[" << (1 << K) << "];\n";
    head << "    const unsigned tid = threadIdx.x;\n";

    std::vector<int> local(64, -1);
    for (int j = 0; j < K; ++j) local[P.S[j]] = j;
    auto global_imgs = [&](const Layout& L, std::vector<uint64_t>& thr, std::vector<uint64_t>& reg) {
        thr.clear();
        reg.clear();
        for (int b = 0; b < TB; ++b) thr.push_back(1ull << P.S[L.thr[b]]);
        for (int b = 0; b < RB; ++b) reg.push_back(1ull << P.S[L.reg[b]]);
    };
    std::vector<uint64_t> ldthr, ldreg, stthr, streg;
    global_imgs(P.phases.front().lay, ldthr, ldreg);
    global_imgs(P.store, stthr, streg);
    head << "    const unsigned long long ldt = " << tid_expr(ldthr, false, true) << ";\n";
    head << "    const unsigned long long stt = " << tid_expr(stthr, false, true) << ";\n";

    // re-layout transitions: (from, to) pairs, including the final one
    struct Trans {
        std::vector<uint32_t> img;
        const Layout* from;
        const Layout* to;
    };
    std::vector<Trans> trans;
    for (size_t ph = 1; ph < P.phases.size(); ++ph)
        trans.push_back({swizzle(P.phases[ph - 1].lay, P.phases[ph].lay, K), &P.phases[ph - 1].lay,
                         &P.phases[ph].lay});
    const Layout& last = P.phases.back().lay;
    const bool final_t = !(last.reg == P.store.reg && last.thr == P.store.thr);
    if (final_t) trans.push_back({swizzle(last, P.store, K), &last, &P.store});
    // A re-layout is wave-local when every wave reads back exactly the LDS
    // addresses it wrote (the qubits of the wave-index bits stay in place):
    // it then needs no workgroup barrier.  Checked here address by address.
    std::vector<char> wave_local(trans.size(), 0);
    std::vector<std::vector<std::vector<uint32_t>>> read_set(trans.size());
    for (size_t t = 0; t < trans.size(); ++t) {
        std::vector<uint64_t> wi, ri;
        for (int b = 0; b < TB; ++b) wi.push_back(trans[t].img[trans[t].from->thr[b]]);
        for (int b = 0; b < TB; ++b) ri.push_back(trans[t].img[trans[t].to->thr[b]]);
        head << "    const unsigned tw" << t << " = " << tid_expr(wi, true, false) << ";\n";
        head << "    const unsigned tr" << t << " = " << tid_expr(ri, true, false) << ";\n";
        std::vector<uint32_t> wr, rr;
        for (int b = 0; b < RB; ++b) wr.push_back(trans[t].img[trans[t].from->reg[b]]);
        for (int b = 0; b < RB; ++b) rr.push_back(trans[t].img[trans[t].to->reg[b]]);
        auto addrs = [&](uint32_t tid0, uint32_t count, const std::vector<uint64_t>& timg, const std::vector<uint32_t>& rimg) {
            std::vector<uint32_t> a;
            for (uint32_t tid = tid0; tid < tid0 + count; ++tid) {
                uint32_t tw = 0;
                for (int b = 0; b < TB; ++b)
                    if ((tid >> b) & 1) tw ^= (uint32_t)timg[b];
                for (uint32_t r = 0; r < (1u << RB); ++r) {
                    uint32_t x = tw;
                    for (int b = 0; b < RB; ++b)
                        if ((r >> b) & 1) x ^= rimg[b];
                    a.push_back(x);
                }
            }
            std::sort(a.begin(), a.end());
            return a;
        };
        const uint32_t wave = std::min(64u, 1u << TB);
        bool local_ok = true;
        for (uint32_t w0 = 0; w0 < (1u << TB); w0 += wave) {
            read_set[t].push_back(addrs(w0, wave, ri, rr));
            local_ok = local_ok && addrs(w0, wave, wi, wr) == read_set[t].back();
        }
        wave_local[t] = local_ok;
    }
    // The next re-layout may follow without a workgroup barrier when both are
    // wave-local and every wave then writes the addresses it has just read.
    std::vector<char> local_next(trans.size(), 0);
    for (size_t t = 0; t + 1 < trans.size(); ++t)
        local_next[t] = wave_local[t] && wave_local[t + 1] && read_set[t] == read_set[t + 1];

    auto reg_off = [&](const std::vector<uint64_t>& img, int r, bool use_xor) {
        uint64_t o = 0;
        for (int b = 0; b < RB; ++b)
            if ((r >> b) & 1) o = use_xor ? (o ^ img[b]) : (o + img[b]);
        return o;
    };
    // Amplitudes stream through once per pass, so loads and stores are
    // marked non-temporal.  The first pass of a run that starts from a basis
    // state forms its tiles instead of reading them.
    auto ld = [&](const std::string& bvar, int r) {
        const std::string at = bvar + " + ldt + " + hex64(reg_off(ldreg, r, false));
        return init ? "qs_basis(" + at + ", init_index)" : "qs_ldnt(&amp[" + at + "])";
    };

    std::vector<int> name(E);
    for (int r = 0; r < E; ++r) name[r] = r;
    auto vn = [&](int r) { return "v" + std::to_string(name[r]); };

    // Conditional NOTs (condition on thread or tile bits only) are not applied
    // to the registers right away.  pend[b] names a per-lane bool: where it is
    // true, the registers of every pair on register bit b hold the two
    // amplitudes the other way round.  The flip is folded into the next LDS or
    // HBM write address, into a later gate on bit b, or applied with selects
    // when an op needs bit b as a control or as a 4x4 target.
    std::vector<std::string> pend(RB);
    // pend_uni[b]: the flip's condition is the same on every lane of a wave
    // (tile-index bits and wave-index thread bits only)
    std::vector<char> pend_uni(RB, 1);
    int nflip = 0;

    // Deferred diagonal factors.  The true state is
    //   gsc * prod_j mul[j]^(x_j) * prod_{j<k} qmul[j][k]^(x_j x_k)
    // times what the registers hold (x_j: the bit of tile qubit j; only
    // entries with has / hasq set).  A dense gate's diagonal part, a
    // one-qubit phase and the factors a NOT moves around land here; the next
    // dense or 4x4 op on the qubit takes them into its matrix on the host,
    // and whatever is left is multiplied in before the tile is stored (the
    // per-qubit factors only by the last pass).  The factors refer to the
    // true state, so they are unaffected by pending flips, except where they
    // are multiplied into registers (a flipped lane holds true bit value 1
    // in the register of stored bit 0).  Pair factors only ever join two
    // register-bit qubits with no pending flip.
    std::vector<Cx> mul(K, 1.0);
    std::vector<bool> has(K, false);
    std::vector<std::vector<Cx>> qmul(K, std::vector<Cx>(K, 1.0));
    std::vector<std::vector<bool>> hasq(K, std::vector<bool>(K, false));
    Cx gsc = in.gsc;
    bool any_deferred = gsc != Cx(1.0, 0.0);
    for (int j = 0; j < K; ++j) {
        mul[j] = in.mul[P.S[j]];
        has[j] = in.has[P.S[j]];
        any_deferred = any_deferred || has[j];
    }
    // factors of qubits outside the tile (multiplied in by the last pass,
    // from the tile index: its bit i is the i-th qubit outside S)
    std::vector<int> outside;
    for (int q = 0; q < 64; ++q)
        if (local[q] < 0 && in.has[q]) outside.push_back(q);
    any_deferred = any_deferred || (last_pass && !outside.empty());
    // Cores scale gsc by |d0| and the stored state by the inverse; per-qubit
    // factors of other magnitude than 1 come from 4x4 cores.  Factors are
    // multiplied in before the stored state leaves a range the precision
    // keeps comfortably.
    const double lo = dbl ? 0x1p-300 : 0x1p-30, hi = 1.0 / lo;
    const double qlo = dbl ? 0x1p-100 : 0x1p-12, qhi = 1.0 / qlo;

    auto materialize = [&](uint32_t bits) {
        for (int b = 0; b < RB; ++b) {
            if (!((bits >> b) & 1) || pend[b].empty()) continue;
            if (pend_uni[b]) {
                // the same on the whole wave: a branch around plain swaps
                s << "        if (__builtin_amdgcn_readfirstlane((int)(" << pend[b] << "))) {\n";
                for (int r0 = 0; r0 < E; ++r0) {
                    if ((r0 >> b) & 1) continue;
                    const std::string A = vn(r0), B = vn(r0 | (1 << b));
                    s << "            { const V t = " << A << "; " << A << " = " << B << "; " << B << " = t; }\n";
                }
                s << "        }\n";
                pend[b].clear();
                continue;
            }
            s << "        {\n            const bool c = " << pend[b] << ";\n";
            for (int r0 = 0; r0 < E; ++r0) {
                if ((r0 >> b) & 1) continue;
                const std::string A = vn(r0), B = vn(r0 | (1 << b));
                // component-wise selects keep both values in registers
                s << "            { const V ta = " << A << ", tb = " << B << "; " << A << ".x = c ? tb.x : ta.x; " << A
                  << ".y = c ? tb.y : ta.y; " << B << ".x = c ? ta.x : tb.x; " << B << ".y = c ? ta.y : tb.y; }\n";
            }
            s << "        }\n";
            pend[b].clear();
        }
    };
    // multiply the registers at positions `regs` by the constant f
    auto mul_regs = [&](const std::vector<int>& regs, Cx f) {
        if (regs.empty()) return;
        const size_t off = g.mats.size();
        g.mats.push_back(f.real());
        g.mats.push_back(f.imag());
        s << "        { const R fr = mt[" << off << "], fi = mt[" << off + 1 << "];";
        for (int r : regs) s << " qs_cm(fr, fi, " << vn(r) << ");";
        s << " }\n";
    };
    // Phases whose controls are all thread or tile-index bits multiply a
    // per-lane factor lfd instead of every register: lfd scales all of a
    // lane's amplitudes alike, so it commutes with every op inside the
    // lane's registers and is multiplied in before data leaves the lane (an
    // LDS re-layout or the store).
    bool lfd_active = false, lfd_declared = false;
    auto flush_lfd = [&]() {
        if (!lfd_active) return;
        s << "        {";
        for (int r = 0; r < E; ++r) s << " qs_cm(lfd.x, lfd.y, " << vn(r) << ");";
        s << " }\n";
        lfd_active = false;
    };
    auto all_regs_with = [&](uint32_t bits) {
        std::vector<int> regs;
        for (int r = 0; r < E; ++r)
            if (((uint32_t)r & bits) == bits) regs.push_back(r);
        return regs;
    };
    // current register bit of tile qubit j in layout L (-1: a thread bit)
    auto reg_bit_in = [&](const Layout& L, int j) {
        for (int b = 0; b < RB; ++b)
            if (L.reg[b] == j) return b;
        return -1;
    };
    const Layout* cur = &P.phases.front().lay;
    auto partners = [&](int j) {
        std::vector<int> ks;
        for (int k = 0; k < K; ++k)
            if (k != j && hasq[j][k]) ks.push_back(k);
        return ks;
    };
    // multiply in the pair factor of (j, k), both register bits
    auto flush_pair = [&](int j, int k) {
        if (!hasq[j][k]) return;
        mul_regs(all_regs_with((1u << reg_bit_in(*cur, j)) | (1u << reg_bit_in(*cur, k))), qmul[j][k]);
        hasq[j][k] = hasq[k][j] = false;
        qmul[j][k] = qmul[k][j] = 1.0;
    };
    auto flush_pairs_of = [&](int j, int except) {
        for (int k : partners(j))
            if (k != except) flush_pair(j, k);
    };
    // multiply in every factor of tile qubit j, held at register bit b
    auto flush_qubit = [&](int j, int b) {
        flush_pairs_of(j, -1);
        if (!has[j]) return;
        materialize(1u << b);
        mul_regs(all_regs_with(1u << b), mul[j]);
        mul[j] = 1.0;
        has[j] = false;
    };
    auto keep_in_range = [&]() {
        for (int j = 0; j < K; ++j)
            for (int k : partners(j))
                if (std::abs(qmul[j][k]) < qlo || std::abs(qmul[j][k]) > qhi) flush_pair(j, k);
        for (int j = 0; j < K; ++j) {
            const int b = reg_bit_in(*cur, j);
            if (has[j] && b >= 0 && (std::abs(mul[j]) < qlo || std::abs(mul[j]) > qhi)) flush_qubit(j, b);
        }
        if (std::abs(gsc) < lo || std::abs(gsc) > hi) {
            mul_regs(all_regs_with(0), gsc);
            gsc = 1.0;
        }
    };
    auto flip_expr = [&](const std::vector<uint64_t>& img, bool wide) {
        std::string e;
        for (int b = 0; b < RB; ++b) {
            if (pend[b].empty()) continue;
            const std::string v = wide ? hex64(img[b]) : hex32((uint32_t)img[b]);
            e += (e.empty() ? "" : " ^ ") + std::string("(") + pend[b] + " ? " + v + " : " + (wide ? "0ull" : "0u") + ")";
        }
        return e;
    };

    size_t tcount = 0;
    auto emit_relayout = [&](size_t t) {
        const Trans& T = trans[t];
        flush_lfd();
        // pair factors join register bits only: multiply in those whose
        // qubits leave the register bits
        for (int j = 0; j < K; ++j)
            for (int k : partners(j))
                if (k > j && (reg_bit_in(*T.to, j) < 0 || reg_bit_in(*T.to, k) < 0)) flush_pair(j, k);
        std::vector<uint64_t> wreg, rreg;
        for (int b = 0; b < RB; ++b) wreg.push_back(T.img[T.from->reg[b]]);
        for (int b = 0; b < RB; ++b) rreg.push_back(T.img[T.to->reg[b]]);
        // The swizzle mixes only into address bits 0..2 and the thread and
        // register parts have disjoint bits above them, so tw ^ x equals
        // (tw ^ (x & 7)) + (x & ~7): at most eight distinct address registers
        // per side, the rest goes into the instructions' immediate offsets.
        for (int j = 0; j < K; ++j)
            if ((T.img[j] ^ (1u << j)) & ~7u) g.bad = true;
        auto addr = [&](const char* side, uint32_t x) {
            std::ostringstream a;
            a << "((" << side << t << "z ^ " << (x & 7u) << "u) + " << hex32(x & ~7u) << ")";
            return a.str();
        };
        s << "        const unsigned tw" << t << "z = tw" << t << " ^ z, tr" << t << "z = tr" << t << " ^ z;\n";
        const std::string fx = flip_expr(wreg, false);
        if (fx.empty()) {
            for (int r = 0; r < E; ++r)
                s << "        lds[" << addr("tw", (uint32_t)reg_off(wreg, r, true)) << "] = " << vn(r) << ";\n";
        } else {
            // a flipped lane writes register r where register r ^ flips goes
            s << "        const unsigned twf" << t << " = tw" << t << "z ^ " << fx << ";\n";
            for (int r = 0; r < E; ++r)
                s << "        lds[twf" << t << " ^ " << hex32((uint32_t)reg_off(wreg, r, true)) << "] = " << vn(r) << ";\n";
            for (int b = 0; b < RB; ++b) pend[b].clear();
        }
        s << (wave_local[t] ? "        QS_WBAR();\n" : "        QS_BAR();\n");
        // read into fresh names so that no value is overwritten before it is stored
        for (int r = 0; r < E; ++r)
            s << "        const V w" << t << "_" << r << " = lds[" << addr("tr", (uint32_t)reg_off(rreg, r, true)) << "];\n";
        // the next re-layout may write where other waves still read unless
        // both are wave-local over the same per-wave address sets; the last
        // one of a tile is followed by the next tile's first, so it always
        // waits for the whole workgroup
        const bool next_local = t + 1 < trans.size() && local_next[t];
        s << (next_local ? "        QS_WBAR();\n" : "        QS_BAR();\n");
        for (int r = 0; r < E; ++r) s << "        v" << r << " = w" << t << "_" << r << ";\n";
        for (int r = 0; r < E; ++r) name[r] = r;
        cur = T.to;
    };

    for (size_t ph = 0; ph < P.phases.size(); ++ph) {
        const Layout& L = P.phases[ph].lay;
        if (ph > 0) emit_relayout(tcount++);
        auto reg_bit = [&](int j) { return reg_bit_in(L, j); };
        for (int idx : P.phases[ph].ops) {
            const OpRec& op = all[idx];
            uint32_t rmask = 0, tmask = 0;
            uint64_t gmask = 0;
            auto classify = [&](int q) {
                const int j = local[q];
                if (j < 0) {
                    gmask |= 1ull << q;
                    return;
                }
                for (int b = 0; b < RB; ++b)
                    if (L.reg[b] == j) {
                        rmask |= 1u << b;
                        return;
                    }
                for (int b = 0; b < TB; ++b)
                    if (L.thr[b] == j) {
                        tmask |= 1u << b;
                        return;
                    }
            };
            for (int q : op.ctrls) classify(q);
            // a one-qubit phase on a tile qubit is deferred (no code)
            if (op.kind == 2 && op.ctrls.size() == 1 && local[op.ctrls[0]] >= 0) {
                const int j = local[op.ctrls[0]];
                mul[j] *= std::polar(1.0, op.angle);
                has[j] = true;
                any_deferred = true;
                continue;
            }
            std::string cond;
            if (gmask) cond = "((base & " + hex64(gmask) + ") == " + hex64(gmask) + ")";
            if (tmask) {
                const std::string t = "((tid & " + hex32(tmask) + ") == " + hex32(tmask) + ")";
                cond = cond.empty() ? t : cond + " && " + t;
            }
            materialize(rmask);  // register controls are read as they stand
            // (kernel data offsets are taken right before an op's data is
            // appended: flushes of deferred factors append their own first)
            if (op.kind == 2 && cond.empty() && __builtin_popcount(rmask) == 2) {
                // a phase on two register qubits (both without a pending
                // flip now): one more pair factor
                const int j1 = L.reg[__builtin_ctz(rmask)], j2 = L.reg[31 - __builtin_clz(rmask)];
                const Cx f = std::polar(1.0, op.angle) * (hasq[j1][j2] ? qmul[j1][j2] : Cx(1.0));
                qmul[j1][j2] = qmul[j2][j1] = f;
                hasq[j1][j2] = hasq[j2][j1] = true;
                any_deferred = true;
                continue;
            }
            if (op.kind == 2 && rmask == 0 && !cond.empty()) {
                // a phase conditioned on thread or tile-index bits only: lfd
                const size_t off = g.mats.size();
                g.mats.insert(g.mats.end(), {cos(op.angle), sin(op.angle)});
                if (!lfd_declared) s << "        V lfd;\n";
                if (!lfd_active) s << "        lfd.x = (R)1;\n        lfd.y = (R)0;\n";
                lfd_declared = lfd_active = true;
                s << "        { const bool c = " << cond << "; R fr = mt[" << off << "], fi = mt[" << off + 1
                  << "]; fr = c ? fr : (R)1; fi = c ? fi : (R)0; qs_cm(fr, fi, lfd); }\n";
                continue;
            }
            if (op.kind == 2) {  // phase on the registers whose masked bits are 1
                const size_t off = g.mats.size();
                g.mats.insert(g.mats.end(), {cos(op.angle), sin(op.angle), 0, 0, 0, 0, 0, 0});
                s << "        {\n            R fr = mt[" << off << "], fi = mt[" << off + 1 << "];\n";
                if (!cond.empty())
                    s << "            const bool c = " << cond << ";\n            fr = c ? fr : (R)1; fi = c ? fi : (R)0;\n";
                for (int r = 0; r < E; ++r)
                    if (((uint32_t)r & rmask) == rmask) s << "            qs_cm(fr, fi, " << vn(r) << ");\n";
                s << "        }\n";
                continue;
            }
            if (op.kind == 4) {  // 4x4 on two register bits
                const int j1 = local[op.target], j2 = local[op.target2];
                const int b1 = reg_bit(j1), b2 = reg_bit(j2);
                materialize((1u << b1) | (1u << b2));
                flush_pairs_of(j1, j2);
                flush_pairs_of(j2, j1);
                // the deferred factors of both qubits and of the pair go into the columns
                Cx dcol[4];
                for (int c = 0; c < 4; ++c) {
                    dcol[c] = 1.0;
                    if ((c & 1) && has[j1]) dcol[c] *= mul[j1];
                    if ((c & 2) && has[j2]) dcol[c] *= mul[j2];
                    if (c == 3 && hasq[j1][j2]) dcol[c] *= qmul[j1][j2];
                }
                const bool deferred = has[j1] || has[j2] || hasq[j1][j2];
                Cx m[4][4];
                for (int i = 0; i < 4; ++i)
                    for (int c = 0; c < 4; ++c) m[i][c] = Cx(op.m4[2 * (4 * i + c)], op.m4[2 * (4 * i + c) + 1]) * dcol[c];
                mul[j1] = mul[j2] = 1.0;
                has[j1] = has[j2] = false;
                qmul[j1][j2] = qmul[j2][j1] = 1.0;
                hasq[j1][j2] = hasq[j2][j1] = false;
                if (cond.empty() && rmask == 0) {
                    // unit-diagonal core: M = D C P, P a permutation of the
                    // four members (register renames), D = diag deferred
                    static const int perms[24][4] = {
                        {0, 1, 2, 3}, {0, 1, 3, 2}, {0, 2, 1, 3}, {0, 2, 3, 1}, {0, 3, 1, 2}, {0, 3, 2, 1},
                        {1, 0, 2, 3}, {1, 0, 3, 2}, {1, 2, 0, 3}, {1, 2, 3, 0}, {1, 3, 0, 2}, {1, 3, 2, 0},
                        {2, 0, 1, 3}, {2, 0, 3, 1}, {2, 1, 0, 3}, {2, 1, 3, 0}, {2, 3, 0, 1}, {2, 3, 1, 0},
                        {3, 0, 1, 2}, {3, 0, 2, 1}, {3, 1, 0, 2}, {3, 1, 2, 0}, {3, 2, 0, 1}, {3, 2, 1, 0}};
                    int best = -1;
                    double bestv = 0.0;
                    for (int p = 0; p < 24; ++p) {
                        double v = 1.0;
                        for (int i = 0; i < 4; ++i) v *= std::abs(m[i][perms[p][i]]);
                        if (v > bestv) {
                            bestv = v;
                            best = p;
                        }
                    }
                    if (best >= 0) {
                        const int* pi = perms[best];
                        Cx D[4];
                        for (int i = 0; i < 4; ++i) D[i] = m[i][pi[i]];
                        const Cx n1 = D[1] / D[0], n2 = D[2] / D[0], nq = D[3] * D[0] / (D[1] * D[2]);
                        bool ok = true;
                        for (const Cx& x : {n1, n2, nq})
                            ok = ok && std::abs(x) >= qlo && std::abs(x) <= qhi;
                        double cmax = 0.0;
                        for (int i = 0; i < 4; ++i)
                            for (int c = 0; c < 4; ++c)
                                if (c != i) cmax = std::max(cmax, std::abs(m[i][pi[c]] / D[i]));
                        ok = ok && cmax <= (dbl ? 1e100 : 1e6);
                        if (ok) {
                            // y_i = x_{pi(i)} + sum_{c != i} C[i][c] x_{pi(c)}: the
                            // member registers in the order pi, outputs in
                            // place, then renamed to their positions
                            const size_t off = g.mats.size();
                            for (int i = 0; i < 4; ++i)
                                for (int c = 0; c < 4; ++c) {
                                    if (c == i) continue;
                                    const Cx cc = m[i][pi[c]] / D[i];
                                    g.mats.push_back(cc.real());
                                    g.mats.push_back(cc.imag());
                                }
                            s << "        {\n            R c[24];\n";
                            for (int k = 0; k < 24; ++k) s << "            c[" << k << "] = mt[" << off + k << "];\n";
                            for (int r0 = 0; r0 < E; ++r0) {
                                if (((r0 >> b1) & 1) || ((r0 >> b2) & 1)) continue;
                                const int rr[4] = {r0, r0 | (1 << b1), r0 | (1 << b2), r0 | (1 << b1) | (1 << b2)};
                                s << "            qs_core4(c, " << vn(rr[pi[0]]) << ", " << vn(rr[pi[1]]) << ", "
                                  << vn(rr[pi[2]]) << ", " << vn(rr[pi[3]]) << ");\n";
                                int nn[4];
                                for (int i = 0; i < 4; ++i) nn[i] = name[rr[pi[i]]];
                                for (int i = 0; i < 4; ++i) name[rr[i]] = nn[i];
                            }
                            s << "        }\n";
                            gsc *= D[0];
                            mul[j1] = n1;
                            mul[j2] = n2;
                            qmul[j1][j2] = qmul[j2][j1] = nq;
                            has[j1] = has[j2] = true;
                            hasq[j1][j2] = hasq[j2][j1] = true;
                            any_deferred = true;
                            keep_in_range();
                            continue;
                        }
                    }
                }
                const size_t off = g.mats.size();
                for (int i = 0; i < 4; ++i)
                    for (int c = 0; c < 4; ++c) {
                        g.mats.push_back(m[i][c].real());
                        g.mats.push_back(m[i][c].imag());
                    }
                const size_t doff = g.mats.size();
                if (deferred)
                    for (int c = 0; c < 4; ++c) {
                        g.mats.push_back(dcol[c].real());
                        g.mats.push_back(dcol[c].imag());
                    }
                s << "        {\n            R m[32];\n";
                for (int k = 0; k < 32; ++k) s << "            m[" << k << "] = mt[" << off + k << "];\n";
                if (!cond.empty()) {
                    // lanes the condition excludes keep only the deferred diagonal
                    s << "            const bool c = " << cond << ";\n";
                    for (int k = 0; k < 32; ++k) {
                        const int e = k / 2, rr = e / 4, cc = e % 4;
                        if (rr == cc && deferred)
                            s << "            m[" << k << "] = c ? m[" << k << "] : mt[" << doff + 2 * cc + (k & 1)
                              << "];\n";
                        else
                            s << "            m[" << k << "] = c ? m[" << k << "] : (R)"
                              << ((rr == cc && k % 2 == 0) ? 1 : 0) << ";\n";
                    }
                }
                for (int r0 = 0; r0 < E; ++r0) {
                    if (((r0 >> b1) & 1) || ((r0 >> b2) & 1)) continue;
                    if (((uint32_t)r0 & rmask) != rmask) {
                        // registers the controls exclude keep only the deferred diagonal
                        if (deferred)
                            for (int c = 1; c < 4; ++c) {
                                const int r = r0 | ((c & 1) << b1) | ((c >> 1) << b2);
                                s << "            qs_cm(mt[" << doff + 2 * c << "], mt[" << doff + 2 * c + 1 << "], "
                                  << vn(r) << ");\n";
                            }
                        continue;
                    }
                    s << "            qs_ap4(m, " << vn(r0) << ", " << vn(r0 | (1 << b1)) << ", " << vn(r0 | (1 << b2))
                      << ", " << vn(r0 | (1 << b1) | (1 << b2)) << ");\n";
                }
                s << "        }\n";
                continue;
            }
            const int j = local[op.target];
            const int b = reg_bit(j);
            if (op.kind == 1) {  // NOT
                if (!cond.empty()) {
                    flush_qubit(j, b);  // a conditional exchange cannot keep a deferred factor
                    if (rmask == 0) {
                        const std::string f = "f" + std::to_string(nflip++);
                        s << "        const bool " << f << " = " << (pend[b].empty() ? "" : "(" + pend[b] + ") != ")
                          << "(" << cond << ");\n";
                        const bool uni = (tmask & ((1u << std::min(TB, 6)) - 1)) == 0;
                        pend_uni[b] = (pend[b].empty() ? 1 : pend_uni[b]) && uni;
                        pend[b] = f;
                    } else {
                        s << "        {\n            const bool c = " << cond << ";\n";
                        for (int r0 = 0; r0 < E; ++r0) {
                            if ((r0 >> b) & 1) continue;
                            if (((uint32_t)r0 & rmask) != rmask) continue;
                            const std::string A = vn(r0), B = vn(r0 | (1 << b));
                            s << "            { const V ta = " << A << ", tb = " << B << "; " << A
                              << ".x = c ? tb.x : ta.x; " << A << ".y = c ? tb.y : ta.y; " << B << ".x = c ? ta.x : tb.x; "
                              << B << ".y = c ? ta.y : tb.y; }\n";
                        }
                        s << "        }\n";
                    }
                    continue;
                }
                // the stored state goes through X where the controls are set,
                // a permutation of register names (a pending flip on b
                // commutes with it); the deferred factors follow the
                // substitution x_t -> x_t xor (controls)
                const int nc = __builtin_popcount(rmask);
                const int jc = nc == 1 ? L.reg[__builtin_ctz(rmask)] : -1;
                if (nc > 1) flush_qubit(j, b);
                if (nc == 1 && (has[j] || !partners(j).empty())) {
                    materialize(1u << b);  // pair factors join flip-free bits
                    flush_pairs_of(j, jc);
                }
                for (int r0 = 0; r0 < E; ++r0) {
                    if ((r0 >> b) & 1) continue;
                    if (((uint32_t)r0 & rmask) != rmask) continue;
                    std::swap(name[r0], name[r0 | (1 << b)]);
                }
                if (nc == 0) {
                    // x_t -> 1 - x_t: mul^x_t -> mul (1/mul)^x_t; q^(x_t x_k) -> q^x_k (1/q)^(x_t x_k)
                    if (has[j]) {
                        gsc *= mul[j];
                        mul[j] = 1.0 / mul[j];
                    }
                    for (int k : partners(j)) {
                        mul[k] = (has[k] ? mul[k] : Cx(1.0)) * qmul[j][k];
                        has[k] = true;
                        qmul[j][k] = qmul[k][j] = 1.0 / qmul[j][k];
                    }
                } else if (nc == 1 && (has[j] || hasq[j][jc])) {
                    // x_t -> x_t xor x_c = x_t + x_c - 2 x_t x_c; (x_t xor x_c) x_c = x_c - x_t x_c
                    const Cx mt_ = has[j] ? mul[j] : Cx(1.0), q_ = hasq[j][jc] ? qmul[j][jc] : Cx(1.0);
                    mul[jc] = (has[jc] ? mul[jc] : Cx(1.0)) * mt_ * q_;
                    has[jc] = true;
                    qmul[j][jc] = qmul[jc][j] = 1.0 / (mt_ * mt_ * q_);
                    hasq[j][jc] = hasq[jc][j] = true;
                }
                keep_in_range();
                continue;
            }
            // dense 2x2 on register bit b
            Cx u[2][2];
            for (int i = 0; i < 2; ++i)
                for (int c = 0; c < 2; ++c) u[i][c] = Cx(op.u[2 * (2 * i + c)], op.u[2 * (2 * i + c) + 1]);
            if (cond.empty() && rmask == 0) {
                if (!pend[b].empty()) flush_pairs_of(j, -1);  // classes and flips do not mix
                const std::vector<int> ps = partners(j);
                const int ncls = 1 << ps.size();
                const Cx mj = has[j] ? mul[j] : Cx(1.0);
                // class v: the partners' bits; column 1 of U takes mul[j] and
                // the pair factors of the partners that are set
                std::vector<Cx> mv(ncls);
                for (int v = 0; v < ncls; ++v) {
                    mv[v] = mj;
                    for (size_t i = 0; i < ps.size(); ++i)
                        if ((v >> i) & 1) mv[v] *= qmul[j][ps[i]];
                }
                // one form for every class (|u00| against |u01 mv|)
                int form = -1;
                bool uniform = true;
                for (int v = 0; v < ncls; ++v) {
                    int f;
                    const Cx a01 = u[0][1] * mv[v], a11 = u[1][1] * mv[v];
                    if (a01 == 0.0 && u[1][0] == 0.0) f = 0;
                    else if (u[0][0] == 0.0 && a11 == 0.0) f = 1;
                    else if (std::abs(u[0][0] * a11) >= std::abs(a01 * u[1][0]) && u[0][0] != 0.0 && a11 != 0.0) f = 2;
                    else if (a01 != 0.0 && u[1][0] != 0.0) f = 3;
                    else f = -1;
                    if (v == 0) form = f;
                    else if (f != form) uniform = false;
                }
                if (form >= 0 && uniform) {
                    // per register pair: a' = a + k0 b, b' = b + k1 a (form 2);
                    // form 3 is form 2 on the exchanged pair (a rename).  For a
                    // unitary gate and unit-modulus deferred factors k1 = -conj(k0)
                    // (one coefficient per class).  A lane whose pair is stored
                    // exchanged applies X C X: k0 and k1 trade places.
                    std::vector<Cx> k0s(ncls), k1s(ncls);
                    bool skew = true;
                    if (form >= 2)
                        for (int v = 0; v < ncls; ++v) {
                            const Cx a01 = u[0][1] * mv[v], a11 = u[1][1] * mv[v];
                            k0s[v] = form == 2 ? a01 / u[0][0] : u[0][0] / a01;
                            k1s[v] = form == 2 ? u[1][0] / a11 : a11 / u[1][0];
                            skew = skew && std::abs(k1s[v] + std::conj(k0s[v])) <= 1e-14 * std::max(1.0, std::abs(k0s[v]));
                        }
                    if (form >= 2) {
                        s << "        {";
                        if (!pend[b].empty()) s << " const bool f_ = " << pend[b] << ";";
                        for (int v = 0; v < ncls; ++v) {
                            const size_t o = g.mats.size();
                            if (skew) {
                                // X C X has coefficient -conj(k): the sign of Re k flips
                                g.mats.insert(g.mats.end(), {k0s[v].real(), k0s[v].imag()});
                                s << " const R a" << v << " = " << (pend[b].empty() ? "" : "f_ ? -mt[" + std::to_string(o) + "] : ")
                                  << "mt[" << o << "], b" << v << " = mt[" << o + 1 << "];";
                                continue;
                            }
                            g.mats.insert(g.mats.end(), {k0s[v].real(), k0s[v].imag(), k1s[v].real(), k1s[v].imag()});
                            if (pend[b].empty()) {
                                s << " const R a" << v << " = mt[" << o << "], b" << v << " = mt[" << o + 1 << "], c" << v
                                  << " = mt[" << o + 2 << "], d" << v << " = mt[" << o + 3 << "];";
                            } else {
                                s << " const R p" << v << " = qs_s(mt[" << o << "]), q" << v << " = qs_s(mt[" << o + 1
                                  << "]), r" << v << " = qs_s(mt[" << o + 2 << "]), t" << v << " = qs_s(mt[" << o + 3
                                  << "]); const R a" << v << " = f_ ? r" << v << " : p" << v << ", b" << v << " = f_ ? t" << v
                                  << " : q" << v << ", c" << v << " = f_ ? p" << v << " : r" << v << ", d" << v << " = f_ ? q"
                                  << v << " : t" << v << ";";
                            }
                        }
                    }
                    for (int r0 = 0; r0 < E; ++r0) {
                        if ((r0 >> b) & 1) continue;
                        const int r1 = r0 | (1 << b);
                        int v = 0;
                        for (size_t i = 0; i < ps.size(); ++i) v |= ((r0 >> reg_bit(ps[i])) & 1) << i;
                        if (form >= 2) {
                            const std::string x = form == 2 ? vn(r0) : vn(r1), y = form == 2 ? vn(r1) : vn(r0);
                            if (skew)
                                s << " qs_core(a" << v << ", b" << v << ", " << x << ", " << y << ");";
                            else
                                s << " qs_core_g(a" << v << ", b" << v << ", c" << v << ", d" << v << ", " << x << ", " << y
                                  << ");";
                        }
                        if (form == 1 || form == 3) std::swap(name[r0], name[r1]);
                    }
                    if (form >= 2) s << " }\n";
                    // deferred diagonal: diag(d0, d1) with d0 = u00 (forms 0,
                    // 2: column 0 is not scaled) or u01 mv (forms 1, 3)
                    if (form == 0 || form == 2) {
                        gsc *= u[0][0];
                        mul[j] = u[1][1] * mj / u[0][0];
                    } else {
                        gsc *= u[0][1] * mj;
                        for (int k : ps) {
                            mul[k] = (has[k] ? mul[k] : Cx(1.0)) * qmul[j][k];
                            has[k] = true;
                            qmul[j][k] = qmul[k][j] = 1.0 / qmul[j][k];
                        }
                        mul[j] = u[1][0] / (u[0][1] * mj);
                    }
                    has[j] = true;
                    any_deferred = true;
                    keep_in_range();
                    continue;
                }
                flush_pairs_of(j, -1);
            }
            // full matrix: the deferred factor of the target goes into column
            // 1; lanes or registers the controls exclude keep only that factor
            flush_pairs_of(j, -1);
            const Cx ep = has[j] ? mul[j] : Cx(1.0);
            const bool deferred = has[j];
            if (deferred) {
                u[0][1] *= ep;
                u[1][1] *= ep;
            }
            mul[j] = 1.0;
            has[j] = false;
            const size_t off = g.mats.size();
            for (int i = 0; i < 2; ++i)
                for (int c = 0; c < 2; ++c) {
                    g.mats.push_back(u[i][c].real());
                    g.mats.push_back(u[i][c].imag());
                }
            if (deferred) {
                g.mats.push_back(ep.real());
                g.mats.push_back(ep.imag());
            }
            s << "        {\n            R m[8];\n";
            for (int k = 0; k < 8; ++k) s << "            m[" << k << "] = mt[" << off + k << "];\n";
            if (!cond.empty()) {
                s << "            const bool c = " << cond << ";\n";
                for (int k = 0; k < 8; ++k) {
                    if (deferred && (k == 6 || k == 7))
                        s << "            m[" << k << "] = c ? m[" << k << "] : mt[" << off + 8 + (k - 6) << "];\n";
                    else
                        s << "            m[" << k << "] = c ? m[" << k << "] : (R)" << ((k == 0 || k == 6) ? 1 : 0)
                          << ";\n";
                }
            }
            if (!pend[b].empty()) {
                // flipped lanes apply X U X: rows and columns exchanged
                s << "            { const bool f = " << pend[b] << "; const R t0 = m[0], t1 = m[1], t2 = m[2], t3 = m[3];\n"
                  << "              m[0] = f ? m[6] : t0; m[1] = f ? m[7] : t1; m[6] = f ? t0 : m[6]; m[7] = f ? t1 : m[7];\n"
                  << "              m[2] = f ? m[4] : t2; m[3] = f ? m[5] : t3; m[4] = f ? t2 : m[4]; m[5] = f ? t3 : m[5]; }\n";
            }
            // a diagonal matrix (u01 = u10 = 0, e.g. a Z rotation) multiplies
            // each amplitude of the pair by its own entry: half the work
            const bool diag = u[0][1] == 0.0 && u[1][0] == 0.0;
            for (int r0 = 0; r0 < E; ++r0) {
                if ((r0 >> b) & 1) continue;
                if (((uint32_t)r0 & rmask) != rmask) {
                    if (deferred)
                        s << "            qs_cm(mt[" << off + 8 << "], mt[" << off + 9 << "], " << vn(r0 | (1 << b))
                          << ");\n";
                    continue;
                }
                if (diag)
                    s << "            qs_cm(m[0], m[1], " << vn(r0) << "); qs_cm(m[6], m[7], " << vn(r0 | (1 << b)) << ");\n";
                else
                    s << "            qs_ap(m, " << vn(r0) << ", " << vn(r0 | (1 << b)) << ");\n";
            }
            s << "        }\n";
        }
    }
    // Deferred factors are multiplied in where they cost least: before the
    // final re-layout if the qubits carrying them all sit in register bits
    // there and not after it.
    auto lane_factors = [&](const Layout& L) {
        int c = 0;
        for (int b = 0; b < TB; ++b) c += has[L.thr[b]] ? 1 : 0;
        return c;
    };
    auto emit_deferred = [&](const Layout& L, std::ostringstream& pro) {
        if (!any_deferred) return;
        // register factor: gsc, the factors of the register-bit qubits and
        // the pair factors (which join register bits only)
        const size_t roff = g.mats.size();
        for (int r = 0; r < E; ++r) {
            Cx f = gsc;
            for (int b = 0; b < RB; ++b)
                if (((r >> b) & 1) && has[L.reg[b]]) f *= mul[L.reg[b]];
            for (int b = 0; b < RB; ++b)
                for (int c = b + 1; c < RB; ++c)
                    if (((r >> b) & 1) && ((r >> c) & 1) && hasq[L.reg[b]][L.reg[c]]) f *= qmul[L.reg[b]][L.reg[c]];
            g.mats.push_back(f.real());
            g.mats.push_back(f.imag());
        }
        // register bits holding a factor under a pending flip: a flipped
        // lane keeps true bit value v of such a bit in the register of stored
        // value 1 - v, so its factor differs by mul^(+-1)
        std::vector<int> fb;
        for (int b = 0; b < RB; ++b)
            if (!pend[b].empty() && has[L.reg[b]]) fb.push_back(b);
        while (fb.size() > 2) {
            materialize(1u << fb.back());
            fb.pop_back();
        }
        const int nl = lane_factors(L);
        const bool tilefac = last_pass && !outside.empty();
        if (nl == 0 && fb.empty() && !tilefac) {
            for (int r = 0; r < E; ++r)
                s << "        qs_cm(mt[" << roff + 2 * r << "], mt[" << roff + 2 * r + 1 << "], " << vn(r) << ");\n";
            return;
        }
        // lane factor: the factors of the thread-bit qubits, fixed per lane
        // (the layout does not change from tile to tile), formed once
        pro << "    V lf;\n    lf.x = (R)1;\n    lf.y = (R)0;\n";
        for (int b = 0; b < TB; ++b) {
            if (!has[L.thr[b]]) continue;
            const size_t o = g.mats.size();
            g.mats.push_back(mul[L.thr[b]].real());
            g.mats.push_back(mul[L.thr[b]].imag());
            pro << "    if (tid & " << (1u << b) << "u) qs_cm(mats[" << o << "], mats[" << o + 1 << "], lf);\n";
        }
        // per tile: the factors of qubits outside the tile, from tables over
        // 8-bit slices of the tile index
        if (tilefac) {
            std::vector<int> rank(64, -1);  // tile-index bit of each qubit outside S
            for (int q = 0, i = 0; q < 64; ++q)
                if (local[q] < 0) rank[q] = i++;
            s << "        V tf;\n        tf.x = (R)1;\n        tf.y = (R)0;\n";
            for (int c = 0; c < 8; ++c) {
                std::vector<int> qs_;
                for (int q : outside)
                    if (rank[q] >= 8 * c && rank[q] < 8 * c + 8) qs_.push_back(q);
                if (qs_.empty()) continue;
                const size_t o = g.mats.size();
                for (int v = 0; v < 256; ++v) {
                    Cx a = 1.0;
                    for (int q : qs_)
                        if ((v >> (rank[q] - 8 * c)) & 1) a *= in.mul[q];
                    g.mats.push_back(a.real());
                    g.mats.push_back(a.imag());
                }
                s << "        { const unsigned ix = (unsigned)((tile >> " << 8 * c << ") & 255ull); qs_cm(mt[" << o
                  << " + 2 * ix], mt[" << o + 1 << " + 2 * ix], tf); }\n";
            }
        }
        // per tile: one lane factor per combination of stored values of the
        // flipped bits
        const int nv = 1 << fb.size();
        for (int v = 0; v < nv; ++v) {
            s << "        V lf" << v << " = lf;\n";
            if (tilefac) s << "        qs_cm(tf.x, tf.y, lf" << v << ");\n";
            for (size_t i = 0; i < fb.size(); ++i) {
                const Cx mq = mul[L.reg[fb[i]]];
                const Cx a = ((v >> i) & 1) ? 1.0 / mq : mq;
                const size_t o = g.mats.size();
                g.mats.push_back(a.real());
                g.mats.push_back(a.imag());
                s << "        if (" << pend[fb[i]] << ") qs_cm(mt[" << o << "], mt[" << o + 1 << "], lf" << v << ");\n";
            }
        }
        for (int r = 0; r < E; ++r) {
            int v = 0;
            for (size_t i = 0; i < fb.size(); ++i) v |= ((r >> fb[i]) & 1) << i;
            s << "        { V f = lf" << v << "; qs_cm(mt[" << roff + 2 * r << "], mt[" << roff + 2 * r + 1
              << "], f); qs_cm(f.x, f.y, " << vn(r) << "); }\n";
        }
    };
    std::ostringstream pro;  // per-lane constants formed before the tile loop
    g.out = in;
    if (!last_pass) {
        // hand the per-qubit factors and gsc on; pair factors are multiplied in
        if (final_t) emit_relayout(tcount++);
        for (int j = 0; j < K; ++j)
            for (int k : partners(j))
                if (k > j) flush_pair(j, k);
        for (int j = 0; j < K; ++j) {
            g.out.mul[P.S[j]] = mul[j];
            g.out.has[P.S[j]] = has[j];
        }
        g.out.gsc = gsc;
    } else {
        if (final_t && lane_factors(last) == 0 && lane_factors(P.store) > 0) {
            emit_deferred(last, pro);
            any_deferred = false;
            for (int j = 0; j < K; ++j)
                for (int k = 0; k < K; ++k) hasq[j][k] = false;
            emit_relayout(tcount++);
        } else {
            if (final_t) emit_relayout(tcount++);
            emit_deferred(P.store, pro);
        }
        for (int j = 0; j < K; ++j) {
            g.out.mul[P.S[j]] = 1.0;
            g.out.has[P.S[j]] = false;
        }
        for (int q : outside) {
            g.out.mul[q] = 1.0;
            g.out.has[q] = false;
        }
        g.out.gsc = 1.0;
    }
    flush_lfd();
    s << "        const unsigned long long bs = base + stt;\n";
    const std::string fx = flip_expr(streg, true);
    if (fx.empty()) {
        for (int r = 0; r < E; ++r)
            s << "        qs_stnt(" << vn(r) << ", &amp[bs + " << hex64(reg_off(streg, r, false)) << "]);\n";
    } else {
        // register offsets are sums of distinct powers of two, so a flipped
        // lane's offset for register r is the XOR of r's and the flips' offsets
        s << "        const unsigned long long sf = " << fx << ";\n";
        for (int r = 0; r < E; ++r)
            s << "        qs_stnt(" << vn(r) << ", &amp[bs + (" << hex64(reg_off(streg, r, false)) << " ^ sf)]);\n";
    }
    // Readouts of the stored state (Sec. II.B.1 probabilities): the lane's
    // |amplitude|^2 in double precision, their sum t, and for each register
    // bit b the sum s0 over registers with bit b clear; a lane whose flip on
    // bit b is pending stored those at bit b set, so it counts t - s0.
    // Thread-bit qubits are fixed per lane (taken from ro_t at the end);
    // qubits outside the tile by the tile's bit in the store address.
    const int nv = readout_n + 1;
    std::vector<int> ro_global;
    if (readout_n > 0) {
        for (int q = 0; q < readout_n; ++q)
            if (local[q] < 0) ro_global.push_back(q);
        s << "        {\n";
        for (int r = 0; r < E; ++r) {
            const std::string a = vn(r);
            s << "            const double p" << r << " = (double)" << a << ".x * (double)" << a << ".x + (double)" << a
              << ".y * (double)" << a << ".y;\n";
        }
        auto sum_of = [&](const std::vector<int>& rs) {
            // pairwise, so that the rounding does not grow with the count
            std::vector<std::string> t;
            for (int r : rs) t.push_back("p" + std::to_string(r));
            while (t.size() > 1) {
                std::vector<std::string> u;
                for (size_t i = 0; i + 1 < t.size(); i += 2) u.push_back("(" + t[i] + " + " + t[i + 1] + ")");
                if (t.size() & 1) u.push_back(t.back());
                t.swap(u);
            }
            return t[0];
        };
        std::vector<int> all_r;
        for (int r = 0; r < E; ++r) all_r.push_back(r);
        s << "            const double t = " << sum_of(all_r) << ";\n";
        s << "            ro_t += t;\n";
        for (int b = 0; b < RB; ++b) {
            std::vector<int> rs;
            for (int r = 0; r < E; ++r)
                if (!((r >> b) & 1)) rs.push_back(r);
            if (pend[b].empty())
                s << "            ro_r" << b << " += " << sum_of(rs) << ";\n";
            else
                s << "            { const double s0 = " << sum_of(rs) << "; ro_r" << b << " += (" << pend[b]
                  << ") ? t - s0 : s0; }\n";
        }
        for (int q : ro_global) s << "            ro_g" << q << " += ((bs >> " << q << ") & 1ull) ? 0.0 : t;\n";
        s << "        }\n";
    }
    s << "        if (!more) break;\n";
    for (int r = 0; r < E; ++r) s << "        v" << r << " = n" << r << ";\n";
    s << "        tile = ntile;\n        base = ins(tile);\n    }\n";
    if (readout_n > 0) {
        // Workgroup sums through the LDS (free after the last re-layout), a
        // chunk of values at a time: thread tid writes its value j to row j,
        // then thread j adds row j in thread order (rows padded by one
        // double, so the readers hit distinct banks).
        const int nt = 1 << TB;
        const int lds_doubles = (1 << K) * (dbl ? 2 : 1);
        const int rows = lds_doubles / (nt + 1);
        auto value = [&](int j) -> std::string {
            if (j == 0) return "ro_t";
            const int q = j - 1, l = local[q];
            if (l < 0) return "ro_g" + std::to_string(q);
            for (int b = 0; b < RB; ++b)
                if (P.store.reg[b] == l) return "ro_r" + std::to_string(b);
            for (int b = 0; b < TB; ++b)
                if (P.store.thr[b] == l) return "(((tid >> " + std::to_string(b) + ") & 1u) ? 0.0 : ro_t)";
            g.bad = true;
            return "0.0";
        };
        s << "    {\n        double* ld = (double*)lds;\n        QS_BAR();\n";
        for (int c0 = 0; c0 < nv; c0 += rows) {
            const int cnt = std::min(rows, nv - c0);
            for (int j = c0; j < c0 + cnt; ++j)
                s << "        ld[" << (j - c0) * (nt + 1) << " + tid] = " << value(j) << ";\n";
            s << "        QS_BAR();\n";
            s << "        if (tid < " << cnt << "u) {\n            double a = 0.0;\n";
            s << "            for (unsigned i = 0; i < " << nt << "u; ++i) a += ld[tid * " << nt + 1 << "u + i];\n";
            s << "            part[(unsigned long long)blockIdx.x * " << nv << "ull + " << c0 << "ull + tid] = a;\n";
            s << "        }\n        QS_BAR();\n";
        }
        s << "    }\n";
    }
    s << "}\n";

    // Tile loop with a one-tile prefetch: tile t + gridDim.x is loaded while
    // tile t is computed.  The matrix pointer is made to depend
    // on the tile (the added term is always 0) so that the scalar matrix loads
    // stay in the loop instead of being hoisted out of it.
    std::ostringstream loop;
    loop << pro.str();
    loop << "    unsigned long long tile = blockIdx.x;\n";
    if (readout_n > 0) {
        loop << "    if (tile >= ntiles) {\n";
        loop << "        for (unsigned j = tid; j < " << nv << "u; j += " << (1 << TB) << "u) part[(unsigned long long)blockIdx.x * "
             << nv << "ull + j] = 0.0;\n";
        loop << "        return;\n    }\n";
        loop << "    double ro_t = 0.0";
        for (int b = 0; b < RB; ++b) loop << ", ro_r" << b << " = 0.0";
        for (int q : ro_global) loop << ", ro_g" << q << " = 0.0";
        loop << ";\n";
    } else {
        loop << "    if (tile >= ntiles) return;\n";
    }
    loop << "    auto ins = [](unsigned long long t) -> unsigned long long {\n";
    loop << "        unsigned long long b = t;\n";
    for (int j = 0; j < K; ++j) {
        const int p = P.S[j];
        loop << "        b = ((b >> " << p << ") << " << (p + 1) << ") | (b & " << hex64((1ull << p) - 1) << ");\n";
    }
    loop << "        return b;\n    };\n";
    loop << "    unsigned long long base = ins(tile);\n";
    for (int r = 0; r < E; ++r) loop << "    V v" << r << " = " << ld("base", r) << ";\n";
    // Drain the first tile's loads before the loop.  The compiler's wait
    // analysis merges the loop entry with the back edge; with these loads
    // still pending at the entry it makes every iteration wait for the loads
    // of the next tile before computing the current one.
    loop << "    __builtin_amdgcn_s_waitcnt(0x0F70);\n";
    loop << "    for (;;) {\n";
    // z is always 0; LDS addresses derived from it are computed in the loop
    // next to their use instead of being hoisted and held in registers.
    loop << "        const unsigned z = (unsigned)(tile >> 62);\n";
    loop << "        const R* mt = mats + z;\n";
    loop << "        const unsigned long long ntile = tile + gridDim.x;\n";
    loop << "        const bool more = ntile < ntiles;\n";
    for (int r = 0; r < E; ++r) loop << "        V n" << r << ";\n";
    loop << "        if (more) {\n";
    loop << "            const unsigned long long nb = ins(ntile);\n";
    for (int r = 0; r < E; ++r) loop << "            n" << r << " = " << ld("nb", r) << ";\n";
    loop << "        }\n";
    g.src = head.str() + loop.str() + s.str();
    return g;
}


// ---------------------------------------------------------------------------
// Code-object cache: in memory per (device, source), and on disk under
// $QS_JIT_CACHE (default $HOME/.cache/qstate) keyed by a 128-bit FNV hash.

struct Loaded {
    hipModule_t mod;
    hipFunction_t fn;
};

std::mutex g_mu;
std::unordered_map<std::string, Loaded> g_loaded;  // key: device + '\n' + source

const char* kOpts[] = {"--offload-arch=gfx950", "-O3", "-Xclang", "-target-feature", "-Xclang",
                       "-packed-fp32-ops"};

std::string cache_path(const std::string& src)
{
    uint64_t h1 = 1469598103934665603ull, h2 = 0x9e3779b97f4a7c15ull;
    for (unsigned char ch : src) {
        h1 = (h1 ^ ch) * 1099511628211ull;
        h2 = (h2 ^ ch) * 0x100000001b3ull + 0x7f4a7c15ull;
    }
    for (const char* o : kOpts)
        for (const char* p = o; *p; ++p) h1 = (h1 ^ (unsigned char)*p) * 1099511628211ull;
    const char* dir = getenv("QS_JIT_CACHE");
    std::string d;
    if (dir && *dir) {
        d = dir;
    } else {
        const char* home = getenv("HOME");
        d = std::string(home ? home : "/tmp") + "/.cache/qstate";
    }
    char name[64];
    snprintf(name, sizeof name, "/%016llx%016llx.co", (unsigned long long)h1, (unsigned long long)h2);
    return d + name;
}

void mkdirs(const std::string& path)
{
    for (size_t i = 1; i < path.size(); ++i)
        if (path[i] == '/') mkdir(path.substr(0, i).c_str(), 0755);
}

bool read_file(const std::string& p, std::vector<char>& out)
{
    FILE* f = fopen(p.c_str(), "rb");
    if (!f) return false;
    fseek(f, 0, SEEK_END);
    const long n = ftell(f);
    fseek(f, 0, SEEK_SET);
    out.resize(n > 0 ? (size_t)n : 0);
    const bool ok = n > 0 && fread(out.data(), 1, (size_t)n, f) == (size_t)n;
    fclose(f);
    return ok;
}

// Compile one source to a code object (empty + message on failure).
std::vector<char> compile(const std::string& src, std::string& err)
{
    std::vector<char> code;
    const std::string path = cache_path(src);
    if (read_file(path, code)) return code;
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "qs_pass.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS) {
        err = "hiprtcCreateProgram failed";
        return {};
    }
    const hiprtcResult rc = hiprtcCompileProgram(prog, (int)(sizeof kOpts / sizeof kOpts[0]), kOpts);
    if (rc != HIPRTC_SUCCESS) {
        size_t ls = 0;
        hiprtcGetProgramLogSize(prog, &ls);
        std::string log(ls + 1, '\0');
        hiprtcGetProgramLog(prog, &log[0]);
        err = std::string("hipRTC: ") + hiprtcGetErrorString(rc) + "\n" + log.substr(0, 2000);
        hiprtcDestroyProgram(&prog);
        return {};
    }
    size_t cs = 0;
    hiprtcGetCodeSize(prog, &cs);
    code.resize(cs);
    hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    mkdirs(path);
    const std::string tmp = path + ".tmp" + std::to_string((unsigned long long)std::hash<std::thread::id>()(std::this_thread::get_id()));
    FILE* f = fopen(tmp.c_str(), "wb");
    if (f) {
        const bool ok = fwrite(code.data(), 1, code.size(), f) == code.size();
        fclose(f);
        if (ok) rename(tmp.c_str(), path.c_str());
        else remove(tmp.c_str());
    }
    return code;
}

// Load (compiling where needed, several sources in parallel) one kernel per source.
qs_status load_all(int device, const std::vector<std::string>& srcs, std::vector<hipFunction_t>& fns)
{
    fns.assign(srcs.size(), nullptr);
    std::vector<size_t> todo;
    {
        std::lock_guard<std::mutex> g(g_mu);
        for (size_t i = 0; i < srcs.size(); ++i) {
            auto it = g_loaded.find(std::to_string(device) + "\n" + srcs[i]);
            if (it != g_loaded.end()) fns[i] = it->second.fn;
            else todo.push_back(i);
        }
    }
    if (todo.empty()) return QS_OK;
    std::vector<std::vector<char>> codes(srcs.size());
    std::vector<std::string> errs(srcs.size());
    std::atomic<size_t> next{0};
    const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    const size_t nthreads = std::min<size_t>(hw, todo.size());
    std::vector<std::thread> pool;
    for (size_t t = 0; t < nthreads; ++t)
        pool.emplace_back([&] {
            for (size_t k; (k = next.fetch_add(1)) < todo.size();) {
                const size_t i = todo[k];
                codes[i] = compile(srcs[i], errs[i]);
            }
        });
    for (auto& th : pool) th.join();
    std::lock_guard<std::mutex> g(g_mu);
    for (size_t i : todo) {
        if (codes[i].empty()) return set_error(QS_E_DEVICE, "pass compilation failed: " + errs[i]);
        const std::string key = std::to_string(device) + "\n" + srcs[i];
        auto it = g_loaded.find(key);
        if (it != g_loaded.end()) {
            fns[i] = it->second.fn;
            continue;
        }
        Loaded L;
        hipError_t e = hipModuleLoadData(&L.mod, codes[i].data());
        if (e != hipSuccess) return hip_error(e, "hipModuleLoadData");
        e = hipModuleGetFunction(&L.fn, L.mod, "qs_pass");
        if (e != hipSuccess) return hip_error(e, "hipModuleGetFunction");
        g_loaded.emplace(key, L);
        fns[i] = L.fn;
    }
    return QS_OK;
}

}  // namespace

size_t esz_of(int prec) { return prec == QS_C128 ? sizeof(double) : sizeof(float); }

// Estimated multiply-adds per amplitude (the planner's op costs) at which a
// compiled pass stops streaming at the HBM rate and its arithmetic sets the
// time.  complex128 tiles move 16 bytes per amplitude each way; complex64
// tiles half of that at about the same instruction rate.
double balance_point(bool dbl) { return dbl ? 120.0 : 60.0; }

// Per-circuit cache of the compiled form for one (register shape, tile).
struct JitPlan {
    int n = -1, kind = -1, prec = 0, TB = 0, RB = 0, max_phases = 0, contig = 0, device = -1;
    size_t nops = 0;
    uint64_t version = 0;  // circuit parameter version the plan was built from
    std::vector<hipFunction_t> fns;
    std::vector<size_t> mat_off;  // element offset of each pass's matrices
    std::vector<int> blocks_per_cu;  // resident workgroups per CU for each pass kernel
    void* dmats = nullptr;        // device copy of all matrices
    // pass 0 forming its tiles from a basis state instead of reading them
    // (same matrices as pass 0), compiled on first use
    std::string init_src;
    hipFunction_t init_fn = nullptr;
    int init_blocks_per_cu = 1;
    // the last pass also summing the readouts (state vectors), compiled on
    // first use: [0] reads its tiles, [1] forms them (a one-pass plan run
    // from a basis state)
    std::string ro_src[2];
    hipFunction_t ro_fn[2] = {nullptr, nullptr};
    int ro_blocks_per_cu[2] = {1, 1};
};

void jit_plan_free(JitPlan* p)
{
    if (!p) return;
    if (p->dmats) {
        (void)hipSetDevice(p->device);
        (void)hipFree(p->dmats);
    }
    delete p;
}

qs_status run_compiled_sv(qs_reg r, qs_circuit_s* c, FusedConfig cfg, int* passes_out, const uint64_t* init_index,
                          double* readout)
{
    if (readout && r->kind != QS_STATEVEC) return set_error(QS_E_KIND, "readouts of compiled passes need a state vector");
    // a density matrix runs as its 2N-qubit vector (Eq. 2)
    std::vector<OpRec> dm_ops;
    if (r->kind == QS_DENSITY) dm_ops = dm_vector_ops(c->ops, r->n);
    const std::vector<OpRec>& ops = r->kind == QS_DENSITY ? dm_ops : c->ops;
    const int nbits = r->nbits;
    if (cfg.max_phases <= 0 || cfg.max_phases > kPhMax) cfg.max_phases = kPhMax;
    JitPlan* J = c->jit;
    // a 2N-qubit state vector and an N-qubit density matrix share nbits but
    // not their op lists (Eq. 2 adds the conjugate gates): the kind is part
    // of the key
    const bool fresh = !J || J->n != nbits || J->kind != r->kind || J->prec != r->prec || J->TB != cfg.TB ||
                       J->RB != cfg.RB ||
                       J->max_phases != cfg.max_phases || J->contig != cfg.contig || J->device != r->env->device ||
                       J->nops != c->ops.size() || J->version != c->version;
    if (fresh) {
        if (J) {
            (void)hipStreamSynchronize(r->stream);  // kernels of the old plan may still read its matrices
            jit_plan_free(J);
            c->jit = nullptr;
        }
        const bool dbl = r->prec == QS_C128;
        // compiled plans are reused: worth the slower lookahead partition
        std::vector<PassPlan> plan =
            plan_passes(ops, nbits, cfg.TB, cfg.RB, cfg.max_phases, 1 << 12, cfg.contig, true, balance_point(dbl));
        std::vector<OpRec> ext(ops);
        for (PassPlan& P : plan) {
            replan_phases_beam(P, ops, cfg.TB, cfg.RB, cfg.max_phases, cfg.contig, 8);
            assign_thread_positions(P, cfg.TB, cfg.contig);
            merge_phase_ops(P, ext);
        }
        std::vector<std::string> srcs;
        std::vector<double> mats;
        std::unique_ptr<JitPlan> nj(new JitPlan());
        Deferred carry;
        for (size_t p = 0; p < plan.size(); ++p) {
            const bool lastp = p + 1 == plan.size();
            GenOut go = generate(plan[p], ext, cfg.TB, cfg.RB, dbl, false, carry, lastp, 0);
            if (go.bad) return set_error(QS_E_ARG, "internal: relayout swizzle outside address bits 0..2");
            if (p == 0) nj->init_src = generate(plan[p], ext, cfg.TB, cfg.RB, dbl, true, carry, lastp, 0).src;
            // the last pass with the readouts (state vectors; compiled on first use)
            if (lastp && r->kind == QS_STATEVEC) {
                nj->ro_src[0] = generate(plan[p], ext, cfg.TB, cfg.RB, dbl, false, carry, true, nbits).src;
                if (p == 0) nj->ro_src[1] = generate(plan[p], ext, cfg.TB, cfg.RB, dbl, true, carry, true, nbits).src;
            }
            carry = go.out;
            nj->mat_off.push_back(mats.size());
            mats.insert(mats.end(), go.mats.begin(), go.mats.end());
            srcs.push_back(std::move(go.src));
        }
        if (mats.empty()) mats.push_back(0.0);
        qs_status s = load_all(r->env->device, srcs, nj->fns);
        if (s) return s;
        for (hipFunction_t fn : nj->fns) {
            int nb = 0;
            hipError_t e = hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 1 << cfg.TB, 0);
            if (e != hipSuccess) return hip_error(e, "occupancy query");
            nj->blocks_per_cu.push_back(std::max(1, nb));
        }
        const size_t bytes = mats.size() * (dbl ? sizeof(double) : sizeof(float));
        hipError_t e = hipMalloc(&nj->dmats, bytes);
        if (e != hipSuccess) return hip_error(e, "matrix buffer");
        if (dbl) {
            e = hipMemcpy(nj->dmats, mats.data(), bytes, hipMemcpyHostToDevice);
        } else {
            std::vector<float> mf(mats.begin(), mats.end());
            e = hipMemcpy(nj->dmats, mf.data(), bytes, hipMemcpyHostToDevice);
        }
        if (e != hipSuccess) {
            (void)hipFree(nj->dmats);
            nj->dmats = nullptr;
            return hip_error(e, "matrix upload");
        }
        nj->n = nbits;
        nj->kind = r->kind;
        nj->prec = r->prec;
        nj->TB = cfg.TB;
        nj->RB = cfg.RB;
        nj->max_phases = cfg.max_phases;
        nj->contig = cfg.contig;
        nj->device = r->env->device;
        nj->nops = c->ops.size();
        nj->version = c->version;
        J = c->jit = nj.release();
    }
    unsigned long long ntiles = 1ull << (nbits - (cfg.TB + cfg.RB));
    unsigned long long init_at = 0;
    if (init_index) {
        // basis index j of a density matrix is the vector entry j + 2^N j
        init_at = r->kind == QS_DENSITY ? *init_index + (*init_index << r->n) : *init_index;
        if (J->fns.empty()) {
            // no pass to fold the initialisation into
            const Launch L{r->stream, r->env->device};
            const uint64_t len = 1ull << nbits;
            qs_status s = profiled(r, QS_K_INIT, [&](int*) {
                return r->prec == QS_C128 ? launch_init_basis<double>(L, r->amp, len, init_at, 1.0, 0.0)
                                          : launch_init_basis<float>(L, r->amp, len, init_at, 1.0, 0.0);
            });
            if (s) return s;
        } else if (!J->init_fn) {
            std::vector<hipFunction_t> f;
            qs_status s = load_all(r->env->device, {J->init_src}, f);
            if (s) return s;
            int nb = 0;
            hipError_t e = hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f[0], 1 << cfg.TB, 0);
            if (e != hipSuccess) return hip_error(e, "occupancy query");
            J->init_blocks_per_cu = std::max(1, nb);
            J->init_fn = f[0];
        }
    }
    // the last pass with the readout sums
    const size_t np = J->fns.size();
    const int ro_var = init_index && np == 1 ? 1 : 0;
    const int nv = nbits + 1;
    unsigned ro_grid = 0;
    double* ro_buf = nullptr;
    // releases the readout buffer once the work queued before it is done
    struct RoFree {
        double*& p;
        hipStream_t s;
        ~RoFree()
        {
            if (p) (void)hipFreeAsync(p, s);
        }
    } ro_free{ro_buf, r->stream};
    if (readout && np > 0) {
        if (!J->ro_fn[ro_var]) {
            std::vector<hipFunction_t> f;
            qs_status s = load_all(r->env->device, {J->ro_src[ro_var]}, f);
            if (s) return s;
            int nb = 0;
            hipError_t e = hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f[0], 1 << cfg.TB, 0);
            if (e != hipSuccess) return hip_error(e, "occupancy query");
            J->ro_blocks_per_cu[ro_var] = std::max(1, nb);
            J->ro_fn[ro_var] = f[0];
        }
        ro_grid = (unsigned)std::min<unsigned long long>(ntiles, 256ull * J->ro_blocks_per_cu[ro_var]);
        // per call and stream-ordered: the workgroups' rows, then the sums
        hipError_t e = hipMallocAsync((void**)&ro_buf, ((size_t)ro_grid + 1) * nv * sizeof(double), r->stream);
        if (e != hipSuccess) return hip_error(e, "readout sums");
    }
    for (size_t p = 0; p < np; ++p) {
        void* amp = r->amp;
        const void* mp = (const char*)J->dmats + J->mat_off[p] * esz_of(r->prec);
        const bool first_init = init_index && p == 0;
        const bool ro = readout && p + 1 == np;
        double* part = ro_buf;
        void* args[] = {&amp, &mp, &ntiles, &init_at, &part};
        void* args_ro[] = {&amp, &mp, &ntiles, &part};
        hipFunction_t fn = first_init ? J->init_fn : J->fns[p];
        int bpc = first_init ? J->init_blocks_per_cu : J->blocks_per_cu[p];
        if (ro) {
            fn = J->ro_fn[ro_var];
            bpc = J->ro_blocks_per_cu[ro_var];
        }
        // a persistent grid: the workgroups that fit on the 256 CUs at once
        const unsigned grid = (unsigned)std::min<unsigned long long>(ntiles, 256ull * bpc);
        void** kargs = ro && !first_init ? args_ro : args;
        qs_status s = profiled(r, QS_K_FUSED, [&](int*) {
            return hipModuleLaunchKernel(fn, grid, 1, 1, 1u << cfg.TB, 1, 1, 0, r->stream, kargs, nullptr);
        });
        if (s) return s;
    }
    if (readout) {
        if (np == 0) {
            // no pass to fold the sums into: the reduction kernels
            qs_status s = qs_calc_total_prob(r, &readout[0]);
            for (int q = 0; q < nbits && s == QS_OK; ++q) s = qs_calc_prob_of_outcome(r, q, 0, &readout[1 + q]);
            if (s) return s;
        } else {
            const Launch L{r->stream, r->env->device};
            double* sums = ro_buf + (size_t)ro_grid * nv;
            qs_status s = profiled(r, QS_K_REDUCE, [&](int*) {
                return launch_sum_columns(L, ro_buf, (int)ro_grid, nv, sums);
            });
            if (s) return s;
            hipError_t e = hipMemcpyAsync(readout, sums, nv * sizeof(double), hipMemcpyDeviceToHost, r->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(r->stream);
            if (e != hipSuccess) return hip_error(e, "readout copy");
        }
    }
    if (passes_out) *passes_out = (int)J->fns.size();
    return QS_OK;
}

// Source of the specialised kernels for one circuit (inspection / tests).
qs_status generate_sources(const std::vector<OpRec>& circuit_ops, int n, int kind, int prec, FusedConfig cfg,
                           std::vector<std::string>& out, std::vector<std::vector<double>>* mats, bool readout)
{
    if (readout && kind != QS_STATEVEC) return set_error(QS_E_KIND, "readouts of compiled passes need a state vector");
    if (cfg.max_phases <= 0 || cfg.max_phases > kPhMax) cfg.max_phases = kPhMax;
    std::vector<OpRec> dm_ops;
    if (kind == QS_DENSITY) dm_ops = dm_vector_ops(circuit_ops, n);
    const std::vector<OpRec>& ops = kind == QS_DENSITY ? dm_ops : circuit_ops;
    if (kind == QS_DENSITY) n *= 2;
    std::vector<PassPlan> plan =
        plan_passes(ops, n, cfg.TB, cfg.RB, cfg.max_phases, 1 << 12, cfg.contig, true, balance_point(prec == QS_C128));
    std::vector<OpRec> ext(ops);
    for (PassPlan& P : plan) {
        replan_phases_beam(P, ops, cfg.TB, cfg.RB, cfg.max_phases, cfg.contig, 8);
        assign_thread_positions(P, cfg.TB, cfg.contig);
        merge_phase_ops(P, ext);
    }
    out.clear();
    if (mats) mats->clear();
    Deferred carry;
    for (size_t p = 0; p < plan.size(); ++p) {
        GenOut go = generate(plan[p], ext, cfg.TB, cfg.RB, prec == QS_C128, false, carry, p + 1 == plan.size(),
                             readout && p + 1 == plan.size() ? n : 0);
        if (go.bad) return set_error(QS_E_ARG, "internal: relayout swizzle outside address bits 0..2");
        carry = go.out;
        out.push_back(go.src);
        if (mats) mats->push_back(go.mats);
    }
    return QS_OK;
}

}  // namespace qs
