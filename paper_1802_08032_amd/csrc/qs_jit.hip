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

struct GenOut {
    std::string src;
    std::vector<double> mats;  // 8 values per op that reads a matrix or phase
    bool bad = false;          // a relayout's swizzle broke the address split
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
)";

GenOut generate(const PassPlan& P, const std::vector<OpRec>& all, int TB, int RB, bool dbl)
{
    const int K = TB + RB, E = 1 << RB;
    GenOut g;
    std::ostringstream s;
    s << (dbl ? "typedef double R;\ntypedef double2 V;\n" : "typedef float R;\ntypedef float2 V;\n");
    s << kPrelude;
    s << "extern \"C\" __global__ void __launch_bounds__(" << (1 << TB)
      << ") qs_pass(V* __restrict__ amp, const R* __restrict__ mats, unsigned long long ntiles)\n{\n";
    s << "    __shared__ V lds[" << (1 << K) << "];\n";
    s << "    const unsigned tid = threadIdx.x;\n";

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
    (void)K;
    global_imgs(P.store, stthr, streg);
    s << "    const unsigned long long ldt = " << tid_expr(ldthr, false, true) << ";\n";
    s << "    const unsigned long long stt = " << tid_expr(stthr, false, true) << ";\n";

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
    for (size_t t = 0; t < trans.size(); ++t) {
        std::vector<uint64_t> wi, ri;
        for (int b = 0; b < TB; ++b) wi.push_back(trans[t].img[trans[t].from->thr[b]]);
        for (int b = 0; b < TB; ++b) ri.push_back(trans[t].img[trans[t].to->thr[b]]);
        s << "    const unsigned tw" << t << " = " << tid_expr(wi, true, false) << ";\n";
        s << "    const unsigned tr" << t << " = " << tid_expr(ri, true, false) << ";\n";
    }

    // Tile loop with a one-tile prefetch: tile t + gridDim.x is loaded while
    // tile t is computed.  The matrix pointer is made to depend
    // on the tile (the added term is always 0) so that the scalar matrix loads
    // stay in the loop instead of being hoisted out of it.
    s << "    unsigned long long tile = blockIdx.x;\n";
    s << "    if (tile >= ntiles) return;\n";
    s << "    auto ins = [](unsigned long long t) -> unsigned long long {\n";
    s << "        unsigned long long b = t;\n";
    for (int j = 0; j < K; ++j) {
        const int p = P.S[j];
        s << "        b = ((b >> " << p << ") << " << (p + 1) << ") | (b & " << hex64((1ull << p) - 1) << ");\n";
    }
    s << "        return b;\n    };\n";
    s << "    unsigned long long base = ins(tile);\n";
    auto reg_off = [&](const std::vector<uint64_t>& img, int r, bool use_xor) {
        uint64_t o = 0;
        for (int b = 0; b < RB; ++b)
            if ((r >> b) & 1) o = use_xor ? (o ^ img[b]) : (o + img[b]);
        return o;
    };
    // Amplitudes stream through once per pass, so loads and stores are
    // marked non-temporal.
    auto ld = [&](const std::string& bvar, int r) {
        return "qs_ldnt(&amp[" + bvar + " + ldt + " + hex64(reg_off(ldreg, r, false)) + "])";
    };
    for (int r = 0; r < E; ++r) s << "    V v" << r << " = " << ld("base", r) << ";\n";
    // Drain the first tile's loads before the loop.  The compiler's wait
    // analysis merges the loop entry with the back edge; with these loads
    // still pending at the entry it makes every iteration wait for the loads
    // of the next tile before computing the current one.
    s << "    __builtin_amdgcn_s_waitcnt(0x0F70);\n";
    s << "    for (;;) {\n";
    // z is always 0; LDS addresses derived from it are computed in the loop
    // next to their use instead of being hoisted and held in registers.
    s << "        const unsigned z = (unsigned)(tile >> 62);\n";
    s << "        const R* mt = mats + z;\n";
    s << "        const unsigned long long ntile = tile + gridDim.x;\n";
    s << "        const bool more = ntile < ntiles;\n";
    for (int r = 0; r < E; ++r) s << "        V n" << r << ";\n";
    s << "        if (more) {\n";
    s << "            const unsigned long long nb = ins(ntile);\n";
    for (int r = 0; r < E; ++r) s << "            n" << r << " = " << ld("nb", r) << ";\n";
    s << "        }\n";

    std::vector<int> name(E);
    for (int r = 0; r < E; ++r) name[r] = r;
    auto vn = [&](int r) { return "v" + std::to_string(name[r]); };

    // Conditional NOTs (condition on thread or tile bits only) are not applied
    // to the registers right away.  pend[b] names a per-lane bool: where it is
    // true, the registers of every pair on register bit b hold the two
    // amplitudes the other way round.  The flip is folded into the next LDS or
    // HBM write address, into the matrix of a later gate on bit b (rows and
    // columns exchanged), or applied with selects when an op needs bit b as a
    // control or as a target of a 4x4 or phase.
    std::vector<std::string> pend(RB);
    int nflip = 0;
    auto materialize = [&](uint32_t bits) {
        for (int b = 0; b < RB; ++b) {
            if (!((bits >> b) & 1) || pend[b].empty()) continue;
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
        s << "        QS_BAR();\n";
        // read into fresh names so that no value is overwritten before it is stored
        for (int r = 0; r < E; ++r)
            s << "        const V w" << t << "_" << r << " = lds[" << addr("tr", (uint32_t)reg_off(rreg, r, true)) << "];\n";
        s << "        QS_BAR();\n";
        for (int r = 0; r < E; ++r) s << "        v" << r << " = w" << t << "_" << r << ";\n";
        for (int r = 0; r < E; ++r) name[r] = r;
    };

    for (size_t ph = 0; ph < P.phases.size(); ++ph) {
        const Layout& L = P.phases[ph].lay;
        if (ph > 0) emit_relayout(tcount++);
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
            std::string cond;
            if (gmask) cond = "((base & " + hex64(gmask) + ") == " + hex64(gmask) + ")";
            if (tmask) {
                const std::string t = "((tid & " + hex32(tmask) + ") == " + hex32(tmask) + ")";
                cond = cond.empty() ? t : cond + " && " + t;
            }
            materialize(rmask);  // register controls are read as they stand
            const size_t off = g.mats.size();
            if (op.kind == 2) {  // phase on the registers whose masked bits are 1
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
                int b1 = -1, b2 = -1;
                for (int k = 0; k < RB; ++k) {
                    if (L.reg[k] == local[op.target]) b1 = k;
                    if (L.reg[k] == local[op.target2]) b2 = k;
                }
                materialize((1u << b1) | (1u << b2));
                for (int k = 0; k < 32; ++k) g.mats.push_back(op.m4[k]);
                s << "        {\n            R m[32];\n";
                for (int k = 0; k < 32; ++k) s << "            m[" << k << "] = mt[" << off + k << "];\n";
                if (!cond.empty()) {
                    s << "            const bool c = " << cond << ";\n";
                    for (int k = 0; k < 32; ++k) {
                        const bool diag = (k % 2 == 0) && ((k / 2) % 5 == 0);
                        s << "            m[" << k << "] = c ? m[" << k << "] : (R)" << (diag ? 1 : 0) << ";\n";
                    }
                }
                for (int r0 = 0; r0 < E; ++r0) {
                    if (((r0 >> b1) & 1) || ((r0 >> b2) & 1)) continue;
                    if (((uint32_t)r0 & rmask) != rmask) continue;
                    s << "            qs_ap4(m, " << vn(r0) << ", " << vn(r0 | (1 << b1)) << ", " << vn(r0 | (1 << b2))
                      << ", " << vn(r0 | (1 << b1) | (1 << b2)) << ");\n";
                }
                s << "        }\n";
                continue;
            }
            int b = -1;
            for (int k = 0; k < RB; ++k)
                if (L.reg[k] == local[op.target]) b = k;
            if (op.kind == 1) {  // NOT
                if (cond.empty()) {
                    // a permutation of register names (a pending flip on b commutes with it)
                    for (int r0 = 0; r0 < E; ++r0) {
                        if ((r0 >> b) & 1) continue;
                        if (((uint32_t)r0 & rmask) != rmask) continue;
                        std::swap(name[r0], name[r0 | (1 << b)]);
                    }
                } else if (rmask == 0) {
                    const std::string f = "f" + std::to_string(nflip++);
                    s << "        const bool " << f << " = " << (pend[b].empty() ? "" : "(" + pend[b] + ") != ") << "("
                      << cond << ");\n";
                    pend[b] = f;
                } else {
                    s << "        {\n            const bool c = " << cond << ";\n";
                    for (int r0 = 0; r0 < E; ++r0) {
                        if ((r0 >> b) & 1) continue;
                        if (((uint32_t)r0 & rmask) != rmask) continue;
                        const std::string A = vn(r0), B = vn(r0 | (1 << b));
                        s << "            { const V ta = " << A << ", tb = " << B << "; " << A << ".x = c ? tb.x : ta.x; "
                          << A << ".y = c ? tb.y : ta.y; " << B << ".x = c ? ta.x : tb.x; " << B
                          << ".y = c ? ta.y : tb.y; }\n";
                    }
                    s << "        }\n";
                }
                continue;
            }
            for (int k = 0; k < 8; ++k) g.mats.push_back(op.u[k]);
            s << "        {\n            R m[8];\n";
            for (int k = 0; k < 8; ++k) s << "            m[" << k << "] = mt[" << off + k << "];\n";
            if (!cond.empty()) {
                s << "            const bool c = " << cond << ";\n";
                for (int k = 0; k < 8; ++k)
                    s << "            m[" << k << "] = c ? m[" << k << "] : (R)" << ((k == 0 || k == 6) ? 1 : 0) << ";\n";
            }
            if (!pend[b].empty()) {
                // flipped lanes apply X U X: rows and columns exchanged
                s << "            { const bool f = " << pend[b] << "; const R t0 = m[0], t1 = m[1], t2 = m[2], t3 = m[3];\n"
                  << "              m[0] = f ? m[6] : t0; m[1] = f ? m[7] : t1; m[6] = f ? t0 : m[6]; m[7] = f ? t1 : m[7];\n"
                  << "              m[2] = f ? m[4] : t2; m[3] = f ? m[5] : t3; m[4] = f ? t2 : m[4]; m[5] = f ? t3 : m[5]; }\n";
            }
            // a diagonal matrix (u01 = u10 = 0, e.g. a Z rotation) multiplies
            // each amplitude of the pair by its own entry: half the work
            const bool diag = op.u[2] == 0.0 && op.u[3] == 0.0 && op.u[4] == 0.0 && op.u[5] == 0.0;
            for (int r0 = 0; r0 < E; ++r0) {
                if ((r0 >> b) & 1) continue;
                if (((uint32_t)r0 & rmask) != rmask) continue;
                if (diag)
                    s << "            qs_cm(m[0], m[1], " << vn(r0) << "); qs_cm(m[6], m[7], " << vn(r0 | (1 << b)) << ");\n";
                else
                    s << "            qs_ap(m, " << vn(r0) << ", " << vn(r0 | (1 << b)) << ");\n";
            }
            s << "        }\n";
        }
    }
    if (final_t) emit_relayout(tcount++);
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
    s << "        if (!more) break;\n";
    for (int r = 0; r < E; ++r) s << "        v" << r << " = n" << r << ";\n";
    s << "        tile = ntile;\n        base = ins(tile);\n    }\n}\n";
    g.src = s.str();
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

// Per-circuit cache of the compiled form for one (register shape, tile).
struct JitPlan {
    int n = -1, kind = -1, prec = 0, TB = 0, RB = 0, max_phases = 0, contig = 0, device = -1;
    size_t nops = 0;
    uint64_t version = 0;  // circuit parameter version the plan was built from
    std::vector<hipFunction_t> fns;
    std::vector<size_t> mat_off;  // element offset of each pass's matrices
    std::vector<int> blocks_per_cu;  // resident workgroups per CU for each pass kernel
    void* dmats = nullptr;        // device copy of all matrices
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

qs_status run_compiled_sv(qs_reg r, qs_circuit_s* c, FusedConfig cfg, int* passes_out)
{
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
            plan_passes(ops, nbits, cfg.TB, cfg.RB, cfg.max_phases, 1 << 12, cfg.contig, true);
        std::vector<OpRec> ext(ops);
        for (PassPlan& P : plan) merge_phase_ops(P, ext);
        std::vector<std::string> srcs;
        std::vector<double> mats;
        std::unique_ptr<JitPlan> nj(new JitPlan());
        for (const PassPlan& P : plan) {
            GenOut go = generate(P, ext, cfg.TB, cfg.RB, dbl);
            if (go.bad) return set_error(QS_E_ARG, "internal: relayout swizzle outside address bits 0..2");
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
    for (size_t p = 0; p < J->fns.size(); ++p) {
        void* amp = r->amp;
        const void* mp = (const char*)J->dmats + J->mat_off[p] * esz_of(r->prec);
        void* args[] = {&amp, &mp, &ntiles};
        // a persistent grid: the workgroups that fit on the 256 CUs at once
        const unsigned grid = (unsigned)std::min<unsigned long long>(ntiles, 256ull * J->blocks_per_cu[p]);
        qs_status s = profiled(r, QS_K_FUSED, [&](int*) {
            return hipModuleLaunchKernel(J->fns[p], grid, 1, 1, 1u << cfg.TB, 1, 1, 0, r->stream, args, nullptr);
        });
        if (s) return s;
    }
    if (passes_out) *passes_out = (int)J->fns.size();
    return QS_OK;
}

// Source of the specialised kernels for one circuit (inspection / tests).
qs_status generate_sources(const std::vector<OpRec>& circuit_ops, int n, int kind, int prec, FusedConfig cfg,
                           std::vector<std::string>& out)
{
    if (cfg.max_phases <= 0 || cfg.max_phases > kPhMax) cfg.max_phases = kPhMax;
    std::vector<OpRec> dm_ops;
    if (kind == QS_DENSITY) dm_ops = dm_vector_ops(circuit_ops, n);
    const std::vector<OpRec>& ops = kind == QS_DENSITY ? dm_ops : circuit_ops;
    if (kind == QS_DENSITY) n *= 2;
    std::vector<PassPlan> plan = plan_passes(ops, n, cfg.TB, cfg.RB, cfg.max_phases, 1 << 12, cfg.contig, true);
    std::vector<OpRec> ext(ops);
    for (PassPlan& P : plan) merge_phase_ops(P, ext);
    out.clear();
    for (const PassPlan& P : plan) {
        GenOut go = generate(P, ext, cfg.TB, cfg.RB, prec == QS_C128);
        if (go.bad) return set_error(QS_E_ARG, "internal: relayout swizzle outside address bits 0..2");
        out.push_back(go.src);
    }
    return QS_OK;
}

}  // namespace qs
