// Host-side planner for fused passes: partitions a gate list into passes
// whose targets fit a tile of K qubits, and each pass into register layouts
// (phases).  Used by the generic fused kernel and by the run-time compiled
// pass kernels.
#include <algorithm>
#include <vector>

#include "qs_plan.h"

namespace qs {

uint64_t qubit_mask(const OpRec& op)
{
    uint64_t m = 0;
    for (int q : op.ctrls) m |= 1ull << q;
    if (op.kind != 2) m |= 1ull << op.target;
    return m;
}

// A layout is coalesced when its first `contig` thread bits carry local
// qubits 0..contig-1 (= global qubits 0..contig-1): consecutive lanes then
// touch consecutive amplitudes in HBM.
bool coalesced(const Layout& L, int contig)
{
    for (int b = 0; b < contig; ++b)
        if (L.thr[b] != b) return false;
    return true;
}

namespace {

Layout make_layout(int TB, int RB, const std::vector<int>& regs)
{
    const int K = TB + RB;
    Layout L;
    L.reg = regs;
    for (int j = 0; j < K; ++j)
        if (std::find(regs.begin(), regs.end(), j) == regs.end()) L.thr.push_back(j);
    (void)RB;
    return L;
}

// Choose `RB` register qubits: first the given preferred targets (in order),
// then fill from `fill` order; never local 0..5 when `coalesce` is set.
std::vector<int> pick_regs(int TB, int RB, const std::vector<int>& pref, bool coalesce, int contig)
{
    const int K = TB + RB;
    std::vector<int> regs;
    auto ok = [&](int j) {
        if (coalesce && j < contig) return false;
        return std::find(regs.begin(), regs.end(), j) == regs.end();
    };
    for (int j : pref) {
        if ((int)regs.size() == RB) break;
        if (ok(j)) regs.push_back(j);
    }
    for (int j = K - 1; j >= 0 && (int)regs.size() < RB; --j)
        if (ok(j)) regs.push_back(j);
    return regs;
}

// Assign the pass's ops to register layouts in dependency order.  Returns
// false if more than kPhMax phases would be needed; then `keep` receives how
// many of the pass ops (a dependency-closed prefix set) fit.
void plan_phases(PassPlan& P, const std::vector<OpRec>& all, int TB, int RB, int max_phases, int contig)
{
    const int K = TB + RB;
    std::vector<int> local(64, -1);
    for (int j = 0; j < K; ++j) local[P.S[j]] = j;
    auto lmask = [&](const OpRec& op) {
        uint32_t m = 0;
        for (int q : op.ctrls)
            if (local[q] >= 0) m |= 1u << local[q];
        if (op.kind != 2) m |= 1u << local[op.target];
        return m;
    };
    std::vector<int> rem = P.ops;
    std::vector<int> kept;
    // next preferred register targets from the remaining ops
    auto preferred = [&](const std::vector<int>& ops_left) {
        std::vector<int> pref;
        uint32_t blocked = 0;
        for (int idx : ops_left) {
            const OpRec& op = all[idx];
            const uint32_t m = lmask(op);
            if (op.kind != 2 && !(m & blocked)) pref.push_back(local[op.target]);
            blocked |= m;
        }
        for (int idx : ops_left)
            if (all[idx].kind != 2) pref.push_back(local[all[idx].target]);
        return pref;
    };
    bool first = true;
    while (!rem.empty()) {
        if ((int)P.phases.size() == max_phases) break;
        PhasePlan ph;
        ph.lay = make_layout(TB, RB, pick_regs(TB, RB, preferred(rem), first, contig));
        first = false;
        uint32_t regm = 0;
        for (int j : ph.lay.reg) regm |= 1u << j;
        uint32_t blocked = 0;
        std::vector<int> next;
        for (int idx : rem) {
            const OpRec& op = all[idx];
            const uint32_t m = lmask(op);
            const bool ready = !(m & blocked);
            const bool fits = op.kind == 2 || ((regm >> local[op.target]) & 1);
            if (ready && fits) {
                ph.ops.push_back(idx);
            } else {
                blocked |= m;
                next.push_back(idx);
            }
        }
        for (int idx : ph.ops) kept.push_back(idx);
        P.phases.push_back(ph);
        rem.swap(next);
    }
    P.ops = kept;  // anything left goes back to the pool
    // store layout: the last phase if it is coalesced, else the first one
    P.store = coalesced(P.phases.back().lay, contig) ? P.phases.back().lay : P.phases.front().lay;
}

}  // namespace

// Greedy pass partition: walk the remaining ops in order; take an op when
// no earlier untaken op shares a qubit with it and its target fits in S.
std::vector<PassPlan> plan_passes(const std::vector<OpRec>& all, int n, int TB, int RB, int max_phases,
                                  int max_ops, int contig)
{
    const int K = TB + RB;
    std::vector<PassPlan> passes;
    std::vector<char> done(all.size(), 0);
    size_t ndone = 0, first = 0;
    while (ndone < all.size()) {
        while (done[first]) ++first;
        uint64_t S = (1ull << contig) - 1;  // first lanes: global qubits 0..contig-1
        int ssize = contig;
        uint64_t blocked = 0;
        std::vector<int> take;
        for (size_t i = first; i < all.size() && (int)take.size() < max_ops; ++i) {
            if (done[i]) continue;
            const OpRec& op = all[i];
            const uint64_t m = qubit_mask(op);
            if (m & blocked) {
                blocked |= m;
                continue;
            }
            if (op.kind == 2) {
                take.push_back((int)i);
                continue;
            }
            const uint64_t tb = 1ull << op.target;
            if (S & tb) {
                take.push_back((int)i);
            } else if (ssize < K) {
                S |= tb;
                ++ssize;
                take.push_back((int)i);
            } else {
                blocked |= m;
            }
        }
        // fill S up to K qubits with the lowest unused ones
        for (int q = 0; q < n && ssize < K; ++q)
            if (!((S >> q) & 1)) {
                S |= 1ull << q;
                ++ssize;
            }
        PassPlan P;
        for (int q = 0; q < n; ++q)
            if ((S >> q) & 1) P.S.push_back(q);
        P.ops = take;
        plan_phases(P, all, TB, RB, max_phases, contig);
        for (int idx : P.ops) {
            done[idx] = 1;
            ++ndone;
        }
        passes.push_back(std::move(P));
    }
    return passes;
}

// GF(2)-linear LDS address map for a re-layout from A to B.  Local bit j
// maps to 1 << j, XORed in its low 3 bits with c_j (j >= 3), so the map is
// invertible.  c_j is chosen so that thread bits 0..2 of both layouts span
// the 8 low values (the 8 lanes sharing one 128-byte LDS cycle).
std::vector<uint32_t> swizzle(const Layout& A, const Layout& B, int K)
{
    std::vector<uint32_t> c(K, 0);
    auto low = [&](int j) -> uint32_t { return j < 3 ? (1u << j) : c[j]; };
    auto independent = [&](const Layout& L) {
        const uint32_t a = low(L.thr[0]), b = low(L.thr[1]), d = low(L.thr[2]);
        const uint32_t vals[7] = {a, b, d, a ^ b, a ^ d, b ^ d, a ^ b ^ d};
        for (uint32_t v : vals)
            if (v == 0) return false;
        return true;
    };
    // assign free bits greedily; try all 8 values for each unset bit used by A or B
    std::vector<int> cand;
    for (int b = 0; b < 3; ++b) {
        if (A.thr[b] >= 3) cand.push_back(A.thr[b]);
        if (B.thr[b] >= 3) cand.push_back(B.thr[b]);
    }
    std::sort(cand.begin(), cand.end());
    cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
    // exhaustive search over at most 6 bits x 8 values is cheap
    const int nc = (int)cand.size();
    uint64_t total = 1;
    for (int k = 0; k < nc; ++k) total *= 8;
    for (uint64_t code = 0; code < total; ++code) {
        uint64_t x = code;
        for (int k = 0; k < nc; ++k) {
            c[cand[k]] = (uint32_t)(x & 7);
            x >>= 3;
        }
        if (independent(A) && independent(B)) break;
    }
    std::vector<uint32_t> img(K);
    for (int j = 0; j < K; ++j) img[j] = (1u << j) ^ (j >= 3 ? c[j] : 0u);
    return img;
}


}  // namespace qs
