// Host-side planner for fused passes: partitions a gate list into passes
// whose targets fit a tile of K qubits, and each pass into register layouts
// (phases).  Used by the generic fused kernel and by the run-time compiled
// pass kernels.
#include <math.h>

#include <algorithm>
#include <complex>
#include <unordered_set>
#include <vector>

#include "qs_plan.h"

namespace qs {

uint64_t target_mask(const OpRec& op)
{
    if (op.kind == 2) return 0;
    uint64_t m = 1ull << op.target;
    if (op.kind == 4) m |= 1ull << op.target2;
    return m;
}

uint64_t qubit_mask(const OpRec& op)
{
    uint64_t m = target_mask(op);
    for (int q : op.ctrls) m |= 1ull << q;
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
    auto ltargets = [&](const OpRec& op) -> uint32_t {
        if (op.kind == 2) return 0;
        uint32_t m = 1u << local[op.target];
        if (op.kind == 4) m |= 1u << local[op.target2];
        return m;
    };
    auto lmask = [&](const OpRec& op) {
        uint32_t m = 0;
        for (int q : op.ctrls)
            if (local[q] >= 0) m |= 1u << local[q];
        return m | ltargets(op);
    };
    std::vector<int> rem = P.ops;
    std::vector<int> kept;
    // next preferred register targets from the remaining ops
    auto preferred = [&](const std::vector<int>& ops_left) {
        std::vector<int> pref;
        uint32_t blocked = 0;
        auto push_targets = [&](const OpRec& op) {
            if (op.kind == 2) return;
            pref.push_back(local[op.target]);
            if (op.kind == 4) pref.push_back(local[op.target2]);
        };
        for (int idx : ops_left) {
            const OpRec& op = all[idx];
            const uint32_t m = lmask(op);
            if (!(m & blocked)) push_targets(op);
            blocked |= m;
        }
        for (int idx : ops_left) push_targets(all[idx]);
        return pref;
    };
    // number of remaining ops a phase with register qubits `regm` admits
    auto admitted = [&](uint32_t regm) {
        uint32_t blocked = 0;
        int count = 0;
        for (int idx : rem) {
            const OpRec& op = all[idx];
            const uint32_t m = lmask(op);
            if (!(m & blocked) && (ltargets(op) & ~regm) == 0) {
                ++count;
            } else {
                blocked |= m;
            }
        }
        return count;
    };
    bool first = true;
    while (!rem.empty()) {
        if ((int)P.phases.size() == max_phases) break;
        PhasePlan ph;
        // the preferred register set, unless another RB-subset of the tile
        // qubits admits more ops (fewer phases, fewer re-layouts)
        std::vector<int> regs = pick_regs(TB, RB, preferred(rem), first, contig);
        uint32_t best = 0;
        for (int j : regs) best |= 1u << j;
        int best_n = admitted(best);
        const uint32_t allowed = ((1u << K) - 1) & ~(first ? (1u << contig) - 1 : 0u);
        for (uint32_t s = allowed; s; s = (s - 1) & allowed) {
            if (__builtin_popcount(s) != RB) continue;
            const int c = admitted(s);
            if (c > best_n) {
                best_n = c;
                best = s;
            }
        }
        // a phase that takes every remaining op is the last one: keep qubits
        // 0..contig-1 on the lanes if that costs nothing, so it can be stored
        // without a final re-layout
        const uint32_t low = (1u << contig) - 1;
        if (best_n == (int)rem.size() && (best & low)) {
            const uint32_t hi = allowed & ~low;
            for (uint32_t s = hi; s; s = (s - 1) & hi)
                if (__builtin_popcount(s) == RB && admitted(s) == best_n) {
                    best = s;
                    break;
                }
        }
        regs.clear();
        for (int j = 0; j < K; ++j)
            if ((best >> j) & 1) regs.push_back(j);
        ph.lay = make_layout(TB, RB, regs);
        first = false;
        uint32_t regm = best;
        uint32_t blocked = 0;
        std::vector<int> next;
        for (int idx : rem) {
            const OpRec& op = all[idx];
            const uint32_t m = lmask(op);
            const bool ready = !(m & blocked);
            const bool fits = (ltargets(op) & ~regm) == 0;
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

// One pass's ops: walk the remaining ops in order and take an op when no
// earlier untaken op shares a qubit with it and its targets lie in S.  With
// `grow`, S may take in new target qubits up to K of them.
std::vector<int> scan_pass(const std::vector<OpRec>& all, const std::vector<char>& done, size_t first,
                           uint64_t& S, int& ssize, int K, int max_ops, bool grow)
{
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
        const uint64_t need = target_mask(op) & ~S;
        const int extra = __builtin_popcountll(need);
        if (extra == 0 || (grow && ssize + extra <= K)) {
            S |= need;
            ssize += extra;
            take.push_back((int)i);
        } else {
            blocked |= m;
        }
    }
    return take;
}

// Pass partition with candidate tile sets.  Each pass's tile qubits S
// hold global qubits 0..contig-1 plus K - contig more.  Candidates: S grown
// greedily from the targets in op order; with windows >= 1 every run of
// K - contig consecutive qubits; with windows == 2 also every pair of runs
// n/2 apart (the row and column qubits of a density matrix's vector); the
// candidate that
// admits the most ops wins (the greedy one on ties).  Runs suit circuits
// with nearest-neighbour two-qubit gates, whose light cones are intervals.
std::vector<PassPlan> partition(const std::vector<OpRec>& all, int n, int TB, int RB, int max_phases,
                                int max_ops, int contig, int windows, bool lookahead)
{
    const int K = TB + RB;
    std::vector<PassPlan> passes;
    std::vector<char> done(all.size(), 0);
    size_t ndone = 0, first = 0;
    const uint64_t low = (1ull << contig) - 1;  // first lanes: global qubits 0..contig-1
    const int w = K - contig;
    std::vector<uint64_t> cands;
    auto run = [](int s, int len) { return len > 0 ? ((1ull << len) - 1) << s : 0ull; };
    if (windows >= 1)
        for (int s = contig; s + w <= n; ++s) cands.push_back(low | run(s, w));
    if (windows >= 2) {
        const int h = n / 2, a = w / 2;
        for (int s = contig; s + a <= h && s + h + (w - a) <= n; ++s)
            cands.push_back(low | run(s, a) | run(s + h, w - a));
    }
    // ops the best candidate admits on top of `done` (lookahead)
    auto best_next = [&](std::vector<char>& d) {
        size_t f = 0;
        while (f < all.size() && d[f]) ++f;
        if (f == all.size()) return (size_t)0;
        uint64_t S = low;
        int ssize = contig;
        size_t best = scan_pass(all, d, f, S, ssize, K, max_ops, true).size();
        for (uint64_t c : cands) {
            uint64_t Sw = c;
            int sz = __builtin_popcountll(c);
            best = std::max(best, scan_pass(all, d, f, Sw, sz, K, max_ops, false).size());
        }
        return best;
    };
    while (ndone < all.size()) {
        while (done[first]) ++first;
        uint64_t S = low;
        int ssize = contig;
        std::vector<int> take = scan_pass(all, done, first, S, ssize, K, max_ops, true);
        size_t score = 0;
        if (lookahead) {
            for (int idx : take) done[idx] = 1;
            score = take.size() + best_next(done);
            for (int idx : take) done[idx] = 0;
        }
        for (uint64_t c : cands) {
            uint64_t Sw = c;
            int sz = __builtin_popcountll(c);
            std::vector<int> tw = scan_pass(all, done, first, Sw, sz, K, max_ops, false);
            bool better = tw.size() > take.size();
            if (lookahead) {
                for (int idx : tw) done[idx] = 1;
                const size_t sc = tw.size() + best_next(done);
                for (int idx : tw) done[idx] = 0;
                better = sc > score || (sc == score && tw.size() > take.size());
                if (better) score = sc;
            }
            if (better) {
                take.swap(tw);
                S = Sw;
                ssize = sz;
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

double op_cost(const OpRec& op, int nregctrl);

// Pass partition by beam search: keep the `width` partial partitions that
// have applied the most ops after each pass, extending each by every
// candidate tile set: S grown greedily, every run of K - contig qubits, and
// every pair of runs of about half that length (a window split around a
// region the pass does not need).  Partial partitions that applied the same
// ops are merged (Zobrist hash of the set).  Returns an empty plan if a
// pass's ops need more register layouts than allowed.
std::vector<PassPlan> partition_beam(const std::vector<OpRec>& all, int n, int TB, int RB, int max_phases,
                                     int max_ops, int contig, int width)
{
    const int K = TB + RB;
    const uint64_t low = (1ull << contig) - 1;
    const int w = K - contig;
    auto run = [](int s0, int len) { return len > 0 ? ((1ull << len) - 1) << s0 : 0ull; };
    std::vector<uint64_t> cands;
    for (int s0 = contig; s0 + w <= n; ++s0) cands.push_back(low | run(s0, w));
    for (int a = std::max(1, w / 2 - 1); a <= std::min(w - 1, w / 2 + 1); ++a)
        for (int s1 = contig; s1 + a <= n; ++s1)
            for (int s2 = s1 + a + 1; s2 + (w - a) <= n; ++s2) cands.push_back(low | run(s1, a) | run(s2, w - a));
    std::vector<uint64_t> key(all.size());
    uint64_t x = 0x9e3779b97f4a7c15ull;
    for (uint64_t& k : key) {  // splitmix64
        x += 0x9e3779b97f4a7c15ull;
        uint64_t z = x;
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        k = z ^ (z >> 31);
    }
    struct Node {
        std::vector<char> done;
        size_t ndone = 0;
        uint64_t hash = 0;
        std::vector<uint64_t> S;
        std::vector<std::vector<int>> takes;
    };
    struct Child {
        size_t score;
        size_t parent;
        uint64_t S, hash;
        std::vector<int> take;
    };
    std::vector<Node> beam(1);
    beam[0].done.assign(all.size(), 0);
    for (int step = 0; step < 4096; ++step) {
        for (const Node& nd : beam) {
            if (nd.ndone != all.size()) continue;
            std::vector<PassPlan> out;
            for (size_t p = 0; p < nd.S.size(); ++p) {
                uint64_t S = nd.S[p];
                int ssize = __builtin_popcountll(S);
                for (int q = 0; q < n && ssize < K; ++q)
                    if (!((S >> q) & 1)) {
                        S |= 1ull << q;
                        ++ssize;
                    }
                PassPlan P;
                for (int q = 0; q < n; ++q)
                    if ((S >> q) & 1) P.S.push_back(q);
                P.ops = nd.takes[p];
                plan_phases(P, all, TB, RB, max_phases, contig);
                if (P.ops.size() != nd.takes[p].size()) return {};
                out.push_back(std::move(P));
            }
            return out;
        }
        std::vector<Child> kids;
        for (size_t b = 0; b < beam.size(); ++b) {
            const Node& nd = beam[b];
            size_t first = 0;
            while (nd.done[first]) ++first;
            auto expand = [&](uint64_t S0, bool grow) {
                uint64_t S = S0;
                int ssize = __builtin_popcountll(S0);
                std::vector<int> take = scan_pass(all, nd.done, first, S, ssize, K, max_ops, grow);
                if (take.empty()) return;
                uint64_t h = nd.hash;
                for (int i : take) h ^= key[i];
                kids.push_back(Child{nd.ndone + take.size(), b, S, h, std::move(take)});
            };
            expand(low, true);
            for (uint64_t c : cands) expand(c, false);
        }
        if (kids.empty()) return {};
        std::stable_sort(kids.begin(), kids.end(), [](const Child& a, const Child& c) { return a.score > c.score; });
        std::vector<Node> next;
        std::unordered_set<uint64_t> seen;
        for (Child& c : kids) {
            if ((int)next.size() == width) break;
            if (!seen.insert(c.hash).second) continue;
            Node nd = beam[c.parent];
            for (int i : c.take) nd.done[i] = 1;
            nd.ndone = c.score;
            nd.hash = c.hash;
            nd.S.push_back(c.S);
            nd.takes.push_back(std::move(c.take));
            next.push_back(std::move(nd));
        }
        beam.swap(next);
    }
    return {};
}

// Estimated multiply-adds per amplitude of a pass's ops (controls inside
// the tile counted as register controls), plus a charge per LDS re-layout
// between register layouts (about two dense gates' worth of time where the
// pass is bound by its arithmetic).
constexpr double kRelayoutCost = 8.0;
double pass_cost(const PassPlan& P, const std::vector<OpRec>& all)
{
    uint64_t inS = 0;
    for (int q : P.S) inS |= 1ull << q;
    double c = 0.0;
    for (int idx : P.ops) {
        const OpRec& op = all[idx];
        int nc = 0;
        if (op.kind != 2)
            for (int q : op.ctrls) nc += (inS >> q) & 1;
        c += op_cost(op, nc);
    }
    return c + kRelayoutCost * (P.phases.empty() ? 0 : P.phases.size() - 1);
}

bool replan(PassPlan& P, const std::vector<OpRec>& all, int TB, int RB, int max_phases, int contig)
{
    const size_t want = P.ops.size();
    std::sort(P.ops.begin(), P.ops.end());
    P.phases.clear();
    plan_phases(P, all, TB, RB, max_phases, contig);
    return P.ops.size() == want;
}

// Even out the arithmetic of neighbouring passes.  A pass costs about
// max(hbm, its arithmetic): below `hbm` multiply-adds per amplitude it
// streams the state at the HBM rate, above it the FP units set its time.
// Ops move from the end of a pass to the start of the next one (or from the
// start of a pass to the end of the previous one) while that lowers the sum
// of the two passes' costs, or keeps it and lowers the larger of the two.  An op can move when its targets lie in the
// other pass's tile and no op that stays in its pass and shares a qubit
// with it lies between (so for any two ops sharing a qubit the earlier one
// still runs in the same or an earlier pass, and within a pass ops run in
// circuit order).
void rebalance(std::vector<PassPlan>& passes, const std::vector<OpRec>& all, int TB, int RB, int max_phases,
               int contig, double hbm)
{
    if (hbm <= 0.0 || passes.size() < 2) return;
    std::vector<double> cost;
    for (const PassPlan& P : passes) cost.push_back(pass_cost(P, all));
    auto inside = [&](const PassPlan& P, const OpRec& op) {
        uint64_t inS = 0;
        for (int q : P.S) inS |= 1ull << q;
        return (target_mask(op) & ~inS) == 0;
    };
    auto total = [&](double a, double b) { return std::max(hbm, a) + std::max(hbm, b); };
    // move one op from passes[from] to passes[to] (to = from +- 1); false if none helps
    auto move_one = [&](size_t from, size_t to, std::vector<char>& stuck) {
        PassPlan& A = passes[from];
        PassPlan& B = passes[to];
        std::vector<int> ops = A.ops;
        std::sort(ops.begin(), ops.end());
        const bool fwd = to > from;
        // the best single move: lower total, or the same total with the
        // heavier pass lighter (that lets work travel on towards a lighter pass)
        const double t_old = total(cost[from], cost[to]), m_old = std::max(cost[from], cost[to]);
        double bt = t_old, bm = m_old, bc0 = 0.0, bc1 = 0.0;
        PassPlan b0, b1;
        bool found = false;
        uint64_t stay = 0;
        int tried = 0;
        for (size_t k = 0; k < ops.size() && ops.size() > 1 && tried < 24; ++k) {
            const int idx = fwd ? ops[ops.size() - 1 - k] : ops[k];
            const OpRec& op = all[idx];
            const uint64_t m = qubit_mask(op);
            if (!stuck[idx] && !(m & stay) && inside(B, op)) {
                ++tried;
                PassPlan P0 = A;
                PassPlan P1 = B;
                P0.ops.erase(std::find(P0.ops.begin(), P0.ops.end(), idx));
                P1.ops.push_back(idx);
                if (replan(P0, all, TB, RB, max_phases, contig) && replan(P1, all, TB, RB, max_phases, contig)) {
                    const double c0 = pass_cost(P0, all), c1 = pass_cost(P1, all);
                    const double t = total(c0, c1), mx = std::max(c0, c1);
                    if (t < bt - 1e-9 || (t < bt + 1e-9 && mx < bm - 1e-9)) {
                        bt = t;
                        bm = mx;
                        bc0 = c0;
                        bc1 = c1;
                        b0 = std::move(P0);
                        b1 = std::move(P1);
                        found = true;
                    }
                } else {
                    stuck[idx] = 1;  // would need more register layouts than allowed
                }
            }
            stay |= m;
        }
        if (!found) return false;
        A = std::move(b0);
        B = std::move(b1);
        cost[from] = bc0;
        cost[to] = bc1;
        return true;
    };
    std::vector<char> stuck(all.size(), 0);
    for (int sweep = 0; sweep < 8; ++sweep) {
        bool moved = false;
        for (size_t p = 0; p + 1 < passes.size(); ++p) {
            for (int guard = 0; guard < 256 && cost[p] > hbm && cost[p] > cost[p + 1]; ++guard) {
                if (!move_one(p, p + 1, stuck)) break;
                moved = true;
            }
            for (int guard = 0; guard < 256 && cost[p + 1] > hbm && cost[p + 1] > cost[p]; ++guard) {
                if (!move_one(p + 1, p, stuck)) break;
                moved = true;
            }
        }
        if (!moved) break;
    }
}

}  // namespace

// Three partitions (greedy only, with runs, with runs and pairs of runs);
// the one with the fewest passes is kept (a pass costs one HBM round trip
// of the state), the later one on ties.  With `lookahead`, a fourth
// partition picks each pass's tile set by the ops it admits plus the most
// the next pass could then admit; it is kept only if it needs fewer passes.
// That costs about as many scans as the candidates squared per pass (tens
// of milliseconds for a few hundred ops), worth it where a plan is reused.
std::vector<PassPlan> plan_passes(const std::vector<OpRec>& all, int n, int TB, int RB, int max_phases,
                                  int max_ops, int contig, bool lookahead, double balance)
{
    std::vector<std::vector<PassPlan>> cands;
    for (int mode = 0; mode <= 2; ++mode) cands.push_back(partition(all, n, TB, RB, max_phases, max_ops, contig, mode, false));
    if (lookahead) cands.push_back(partition(all, n, TB, RB, max_phases, max_ops, contig, 2, true));
    if (lookahead && balance > 0.0 && all.size() <= 1500) {
        // a wider search for fewer passes (compiled plans are reused; the
        // search costs about a millisecond per op)
        std::vector<PassPlan> bm = partition_beam(all, n, TB, RB, max_phases, max_ops, contig, 16);
        if (!bm.empty()) cands.push_back(std::move(bm));
    }
    if (lookahead && balance > 0.0) {
        // where a pass is well above the balance point: partitions whose
        // passes take at most 1.5, 1.75 or 2 times the average op count
        // (lighter passes, possibly more of them)
        const std::vector<PassPlan>& la = cands.back();
        double heaviest = 0.0;
        for (const PassPlan& P : la) heaviest = std::max(heaviest, pass_cost(P, all));
        const double avg = (double)all.size() / std::max<size_t>(1, la.size());
        if (heaviest > 1.25 * balance)
            for (double f : {1.25, 1.4, 1.5, 1.6, 1.75, 2.0}) {
                const int cap = (int)ceil(f * avg);
                if (cap < max_ops) cands.push_back(partition(all, n, TB, RB, max_phases, cap, contig, 2, true));
            }
    }
    if (balance <= 0.0) {
        // fewest passes; the later candidate on ties
        size_t b = 0;
        for (size_t i = 1; i < cands.size(); ++i)
            if (cands[i].size() < cands[b].size() || (cands[i].size() == cands[b].size() && i < 3)) b = i;
        return cands[b];
    }
    // with a balance point: the lowest estimated time, sum over passes of
    // max(balance, arithmetic) plus a fifth of the smaller of the two (the
    // overlap of streaming and arithmetic is not perfect), after balancing
    // the three best distinct candidates
    auto estimate = [&](const std::vector<PassPlan>& c) {
        double t = 0.0;
        for (const PassPlan& P : c) {
            const double a = pass_cost(P, all);
            t += std::max(balance, a) + 0.2 * std::min(balance, a);
        }
        return t;
    };
    auto same = [](const std::vector<PassPlan>& x, const std::vector<PassPlan>& y) {
        if (x.size() != y.size()) return false;
        for (size_t p = 0; p < x.size(); ++p)
            if (x[p].S != y[p].S || x[p].ops != y[p].ops) return false;
        return true;
    };
    std::vector<std::pair<double, size_t>> order;
    for (size_t i = 0; i < cands.size(); ++i) {
        bool dup = false;
        for (auto& o : order) dup = dup || same(cands[o.second], cands[i]);
        if (!dup) order.push_back({estimate(cands[i]), i});
    }
    std::sort(order.begin(), order.end());
    size_t b = order[0].second;
    double best = 1e300;
    for (size_t r = 0; r < std::min<size_t>(3, order.size()); ++r) {
        const size_t i = order[r].second;
        rebalance(cands[i], all, TB, RB, max_phases, contig, balance);
        const double t = estimate(cands[i]);
        if (t < best - 1e-9) {
            best = t;
            b = i;
        }
    }
    return cands[b];
}

namespace {

using Cx = std::complex<double>;

// An operator on one or two qubits: index bit k of the 4x4 (or 2x2) matrix
// is qubit q[k].
struct LocalOp {
    int nb = 0;
    int q[2] = {-1, -1};
    Cx m[4][4];
};

bool has(const LocalOp& A, int qb) { return A.q[0] == qb || (A.nb == 2 && A.q[1] == qb); }

// The op as a LocalOp when all its qubits are register qubits (no thread or
// tile condition) and there are at most two of them.
bool soft_op(const OpRec& op, uint64_t regs, LocalOp& L)
{
    std::vector<int> sup;
    if (op.kind == 0 || op.kind == 1) {
        sup.push_back(op.target);
        sup.insert(sup.end(), op.ctrls.begin(), op.ctrls.end());
    } else if (op.kind == 2) {
        sup = op.ctrls;
    } else if (op.kind == 4) {
        if (!op.ctrls.empty()) return false;
        sup = {op.target, op.target2};
    } else {
        return false;
    }
    if (sup.empty() || sup.size() > 2) return false;
    for (int qb : sup)
        if (!((regs >> qb) & 1)) return false;
    L = LocalOp();
    L.nb = (int)sup.size();
    L.q[0] = sup[0];
    if (L.nb == 2) L.q[1] = sup[1];
    const int dim = 1 << L.nb;
    for (int i = 0; i < dim; ++i)
        for (int j = 0; j < dim; ++j) L.m[i][j] = 0.0;
    if (op.kind == 0 || op.kind == 1) {
        // bit 0: target; bit 1 (if any): the control
        Cx u[2][2];
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j)
                u[i][j] = op.kind == 1 ? Cx(i != j ? 1.0 : 0.0, 0.0) : Cx(op.u[2 * (2 * i + j)], op.u[2 * (2 * i + j) + 1]);
        for (int j = 0; j < dim; ++j) {
            if (L.nb == 2 && !((j >> 1) & 1)) {
                L.m[j][j] = 1.0;
                continue;
            }
            for (int i = 0; i < dim; ++i)
                if ((i >> 1) == (j >> 1)) L.m[i][j] = u[i & 1][j & 1];
        }
    } else if (op.kind == 2) {
        for (int j = 0; j < dim; ++j) L.m[j][j] = j == dim - 1 ? std::polar(1.0, op.angle) : Cx(1.0, 0.0);
    } else {
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) L.m[i][j] = Cx(op.m4[2 * (4 * i + j)], op.m4[2 * (4 * i + j) + 1]);
    }
    return true;
}

// A on qubits (q0[, q1]) whose qubits are a subset of them.
LocalOp embed(const LocalOp& A, int nb, int q0, int q1)
{
    LocalOp B;
    B.nb = nb;
    B.q[0] = q0;
    B.q[1] = q1;
    const int dim = 1 << nb;
    int pos[2] = {0, 0};  // bit of B's index holding A's bit k
    for (int k = 0; k < A.nb; ++k) pos[k] = A.q[k] == q0 ? 0 : 1;
    uint32_t amask = 0;
    for (int k = 0; k < A.nb; ++k) amask |= 1u << pos[k];
    auto sub = [&](int i) {
        int s = 0;
        for (int k = 0; k < A.nb; ++k) s |= ((i >> pos[k]) & 1) << k;
        return s;
    };
    for (int i = 0; i < dim; ++i)
        for (int j = 0; j < dim; ++j)
            B.m[i][j] = ((uint32_t)(i ^ j) & ~amask) ? Cx(0.0, 0.0) : A.m[sub(i)][sub(j)];
    return B;
}

LocalOp mul(const LocalOp& A, const LocalOp& B)  // A * B on the same qubits
{
    LocalOp C = A;
    const int dim = 1 << A.nb;
    for (int i = 0; i < dim; ++i)
        for (int j = 0; j < dim; ++j) {
            Cx s = 0.0;
            for (int k = 0; k < dim; ++k) s += A.m[i][k] * B.m[k][j];
            C.m[i][j] = s;
        }
    return C;
}

// Real multiply-adds per amplitude when an op is applied in registers.  An
// uncontrolled dense 2x2 runs as its unit-diagonal core (its diagonal part
// is deferred), a NOT as a register renaming (with at most a phase on the
// quarter where control and target are set, moving a deferred phase), a
// one-qubit phase not at all (deferred).
double op_cost(const OpRec& op, int nregctrl)
{
    switch (op.kind) {
    case 0: return nregctrl == 0 ? 4.0 : 8.0 / (1 << nregctrl);
    case 1: return nregctrl == 0 ? 0.0 : 1.0;
    case 2: return op.ctrls.size() == 1 ? 0.0 : 4.0 / (1 << op.ctrls.size());
    case 4: return 16.0 / (1 << nregctrl);
    default: return 1e9;
    }
}

struct Block {
    LocalOp acc;            // product of everything merged so far
    std::vector<int> plan;  // ops to emit, in order (originals or merged)
    double cost = 0.0;
};

}  // namespace

bool replan_phases_beam(PassPlan& P, const std::vector<OpRec>& all, int TB, int RB, int max_phases, int contig,
                        int width)
{
    const int K = TB + RB;
    std::vector<int> local(64, -1);
    for (int j = 0; j < K; ++j) local[P.S[j]] = j;
    auto ltargets = [&](const OpRec& op) -> uint32_t {
        if (op.kind == 2) return 0;
        uint32_t m = 1u << local[op.target];
        if (op.kind == 4) m |= 1u << local[op.target2];
        return m;
    };
    auto lmask = [&](const OpRec& op) {
        uint32_t m = 0;
        for (int q : op.ctrls)
            if (local[q] >= 0) m |= 1u << local[q];
        return m | ltargets(op);
    };
    std::vector<uint32_t> sets;  // every RB-subset of the tile qubits
    for (uint32_t x = 0; x < (1u << K); ++x)
        if (__builtin_popcount(x) == RB) sets.push_back(x);
    const uint32_t low = (1u << contig) - 1;
    struct St {
        std::vector<int> rem;
        std::vector<uint32_t> regs;
        std::vector<std::vector<int>> ops;
    };
    // ops a phase with register qubits regm takes from rem, and what is left
    auto split = [&](const std::vector<int>& rem, uint32_t regm, std::vector<int>& take, std::vector<int>& left) {
        uint32_t blocked = 0;
        for (int idx : rem) {
            const uint32_t m = lmask(all[idx]);
            if (!(m & blocked) && (ltargets(all[idx]) & ~regm) == 0)
                take.push_back(idx);
            else {
                blocked |= m;
                left.push_back(idx);
            }
        }
    };
    std::vector<St> beam(1);
    beam[0].rem = P.ops;
    const size_t best_known = P.phases.size();
    for (int step = 0; step < max_phases; ++step) {
        struct Kid {
            size_t left;
            size_t parent;
            uint32_t regm;
        };
        std::vector<Kid> kids;
        for (size_t b = 0; b < beam.size(); ++b)
            for (uint32_t x : sets) {
                if (step == 0 && (x & low)) continue;  // coalesced loads
                uint32_t blocked = 0;
                size_t left = 0, took = 0;
                for (int idx : beam[b].rem) {
                    const uint32_t m = lmask(all[idx]);
                    if (!(m & blocked) && (ltargets(all[idx]) & ~x) == 0)
                        ++took;
                    else {
                        blocked |= m;
                        ++left;
                    }
                }
                if (took) kids.push_back(Kid{left, b, x});
            }
        if (kids.empty()) return false;
        std::stable_sort(kids.begin(), kids.end(), [](const Kid& a, const Kid& c) { return a.left < c.left; });
        std::vector<St> next;
        std::vector<std::vector<int>> seen;
        for (const Kid& k : kids) {
            if ((int)next.size() == width) break;
            St st = beam[k.parent];
            std::vector<int> take, left;
            split(st.rem, k.regm, take, left);
            if (std::find(seen.begin(), seen.end(), left) != seen.end()) continue;
            seen.push_back(left);
            st.rem = left;
            st.regs.push_back(k.regm);
            st.ops.push_back(take);
            if (left.empty()) {
                if (st.regs.size() >= best_known) return false;
                // keep qubits 0..contig-1 out of the last phase's registers
                // where that admits the same ops (a store without re-layout)
                uint32_t& last = st.regs.back();
                if (last & low)
                    for (uint32_t x : sets)
                        if (!(x & low)) {
                            std::vector<int> t2, l2;
                            const std::vector<int>& before = st.regs.size() > 1 ? beam[k.parent].rem : P.ops;
                            split(before, x, t2, l2);
                            if (l2.empty()) {
                                last = x;
                                break;
                            }
                        }
                P.phases.clear();
                for (size_t i = 0; i < st.regs.size(); ++i) {
                    std::vector<int> regs;
                    for (int j = 0; j < K; ++j)
                        if ((st.regs[i] >> j) & 1) regs.push_back(j);
                    PhasePlan ph;
                    ph.lay = make_layout(TB, RB, regs);
                    ph.ops = st.ops[i];
                    P.phases.push_back(ph);
                }
                P.store = coalesced(P.phases.back().lay, contig) ? P.phases.back().lay : P.phases.front().lay;
                return true;
            }
            next.push_back(std::move(st));
        }
        beam.swap(next);
    }
    return false;
}

void assign_thread_positions(PassPlan& P, int TB, int contig)
{
    const int kWave = 6;  // thread bits from here on index the wave within the workgroup
    const size_t m = P.phases.size();
    auto in = [](const std::vector<int>& v, int j) { return std::find(v.begin(), v.end(), j) != v.end(); };
    // the next phase after phase i in which qubit j is a register qubit
    auto next_reg = [&](size_t i, int j) {
        for (size_t k = i + 1; k < m; ++k)
            if (in(P.phases[k].lay.reg, j)) return k;
        return m + 1;
    };
    std::vector<int> pos;  // pos[b]: qubit at thread bit b in the previous phase
    for (size_t i = 0; i < m; ++i) {
        Layout& L = P.phases[i].lay;
        const std::vector<int> tset = L.thr;
        std::vector<int> np(TB, -1);
        // wave bits: keep their qubits while they stay thread qubits;
        // otherwise (or in the first phase) give them the thread qubits
        // that stay out of the registers longest
        bool keep = i > 0;
        for (int b = kWave; b < TB && keep; ++b) keep = in(tset, pos[b]);
        if (keep) {
            for (int b = kWave; b < TB; ++b) np[b] = pos[b];
        } else if (TB > kWave) {
            std::vector<int> cand;
            for (int j : tset)
                if (j >= contig) cand.push_back(j);
            std::stable_sort(cand.begin(), cand.end(), [&](int a, int c) { return next_reg(i, a) > next_reg(i, c); });
            for (int b = kWave, k = 0; b < TB && k < (int)cand.size(); ++b, ++k) np[b] = cand[k];
        }
        // lane bits can be permuted freely by any re-layout: qubits
        // 0..contig-1 on their own lanes (coalesced loads and stores without
        // a final re-layout), the others in ascending order
        for (int j = 0; j < contig && j < TB; ++j)
            if (in(tset, j) && !in(np, j) && np[j] < 0) np[j] = j;
        std::vector<int> rest;
        for (int j : tset)
            if (!in(np, j)) rest.push_back(j);
        std::sort(rest.begin(), rest.end());
        for (int b = 0, k = 0; b < TB; ++b)
            if (np[b] < 0) np[b] = rest[k++];
        L.thr = np;
        pos = np;
    }
    // store layout: the last phase with qubits 0..contig-1 on thread bits 0..contig-1
    Layout st = P.phases.back().lay;
    for (int b = 0; b < contig && b < TB; ++b) {
        if (st.thr[b] == b) continue;
        auto t = std::find(st.thr.begin(), st.thr.end(), b);
        if (t != st.thr.end()) {
            std::swap(*t, st.thr[b]);
        } else {
            auto r = std::find(st.reg.begin(), st.reg.end(), b);
            std::swap(*r, st.thr[b]);
        }
    }
    P.store = st;
}

void merge_phase_ops(PassPlan& P, std::vector<OpRec>& ops)
{
    for (PhasePlan& ph : P.phases) {
        uint64_t regs = 0;
        for (int j : ph.lay.reg) regs |= 1ull << P.S[j];
        std::vector<Block> blocks;
        std::vector<int> out;
        auto flush_touching = [&](uint64_t qubits) {
            for (size_t b = 0; b < blocks.size();) {
                const LocalOp& A = blocks[b].acc;
                bool hit = false;
                for (int k = 0; k < A.nb; ++k) hit |= (qubits >> A.q[k]) & 1;
                if (hit) {
                    out.insert(out.end(), blocks[b].plan.begin(), blocks[b].plan.end());
                    blocks.erase(blocks.begin() + b);
                } else {
                    ++b;
                }
            }
        };
        for (int idx : ph.ops) {
            LocalOp L;
            if (!soft_op(ops[idx], regs, L)) {
                flush_touching(qubit_mask(ops[idx]));
                out.push_back(idx);
                continue;
            }
            const double c_op = op_cost(ops[idx], ops[idx].kind == 2 ? 0 : (int)ops[idx].ctrls.size());
            // blocks sharing a qubit with the op, and the union of qubits
            std::vector<size_t> hit;
            uint64_t uni = 0;
            for (int k = 0; k < L.nb; ++k) uni |= 1ull << L.q[k];
            for (size_t b = 0; b < blocks.size(); ++b) {
                const LocalOp& A = blocks[b].acc;
                bool h = false;
                for (int k = 0; k < L.nb; ++k) h |= has(A, L.q[k]);
                if (h) {
                    hit.push_back(b);
                    for (int k = 0; k < A.nb; ++k) uni |= 1ull << A.q[k];
                }
            }
            if (__builtin_popcountll(uni) > 2) {
                uint64_t qm = 0;
                for (int k = 0; k < L.nb; ++k) qm |= 1ull << L.q[k];
                flush_touching(qm);
                Block nbk;
                nbk.acc = L;
                nbk.plan = {idx};
                nbk.cost = c_op;
                blocks.push_back(nbk);
                continue;
            }
            const int nb = __builtin_popcountll(uni);
            const int q0 = __builtin_ctzll(uni);
            const int q1 = nb == 2 ? 63 - __builtin_clzll(uni) : -1;
            LocalOp acc = embed(L, nb, q0, q1);
            Block nbk;
            nbk.cost = c_op;
            for (size_t b : hit) {
                acc = mul(acc, embed(blocks[b].acc, nb, q0, q1));
                nbk.plan.insert(nbk.plan.end(), blocks[b].plan.begin(), blocks[b].plan.end());
                nbk.cost += blocks[b].cost;
            }
            nbk.plan.push_back(idx);
            nbk.acc = acc;
            const double full = nb == 1 ? 4.0 : 16.0;
            if (full < nbk.cost) {
                OpRec m{};
                m.target = q0;
                if (nb == 1) {
                    m.kind = 0;
                    for (int i = 0; i < 2; ++i)
                        for (int j = 0; j < 2; ++j) {
                            m.u[2 * (2 * i + j)] = acc.m[i][j].real();
                            m.u[2 * (2 * i + j) + 1] = acc.m[i][j].imag();
                        }
                } else {
                    m.kind = 4;
                    m.target2 = q1;
                    m.m4.resize(32);
                    for (int i = 0; i < 4; ++i)
                        for (int j = 0; j < 4; ++j) {
                            m.m4[2 * (4 * i + j)] = acc.m[i][j].real();
                            m.m4[2 * (4 * i + j) + 1] = acc.m[i][j].imag();
                        }
                }
                ops.push_back(m);
                nbk.plan = {(int)ops.size() - 1};
                nbk.cost = full;
            }
            std::sort(hit.begin(), hit.end());
            for (size_t k = hit.size(); k-- > 0;) blocks.erase(blocks.begin() + hit[k]);
            blocks.push_back(nbk);
        }
        for (const Block& b : blocks) out.insert(out.end(), b.plan.begin(), b.plan.end());
        ph.ops = out;
    }
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

namespace qs {
namespace {

using Super4 = std::vector<double>;  // 4x4 complex, row-major, re/im interleaved

Super4 mat4_mul(const Super4& A, const Super4& B)  // A * B
{
    Super4 C(32, 0.0);
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            double re = 0.0, im = 0.0;
            for (int k = 0; k < 4; ++k) {
                const double ar = A[2 * (4 * i + k)], ai = A[2 * (4 * i + k) + 1];
                const double br = B[2 * (4 * k + j)], bi = B[2 * (4 * k + j) + 1];
                re += ar * br - ai * bi;
                im += ar * bi + ai * br;
            }
            C[2 * (4 * i + j)] = re;
            C[2 * (4 * i + j) + 1] = im;
        }
    return C;
}

// conj(U) (x) U on (row bit r, column bit c), index r + 2c:
// M[r + 2c][r' + 2c'] = U[r][r'] conj(U[c][c']).
Super4 gate_superop(const double* u)
{
    Super4 M(32, 0.0);
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c)
            for (int r2 = 0; r2 < 2; ++r2)
                for (int c2 = 0; c2 < 2; ++c2) {
                    const double ar = u[2 * (2 * r + r2)], ai = u[2 * (2 * r + r2) + 1];
                    const double br = u[2 * (2 * c + c2)], bi = -u[2 * (2 * c + c2) + 1];
                    const int i = r + 2 * c, j = r2 + 2 * c2;
                    M[2 * (4 * i + j)] = ar * br - ai * bi;
                    M[2 * (4 * i + j) + 1] = ar * bi + ai * br;
                }
    return M;
}

// Channel superoperators on (rho00, rho10, rho01, rho11), the closed forms
// of the three Kraus maps.
Super4 channel_superop(int channel, double p)
{
    Super4 M(32, 0.0);
    auto set = [&](int i, int j, double v) { M[2 * (4 * i + j)] = v; };
    if (channel == QS_DEPHASING) {
        set(0, 0, 1.0);
        set(1, 1, 1.0 - 2.0 * p);
        set(2, 2, 1.0 - 2.0 * p);
        set(3, 3, 1.0);
    } else if (channel == QS_DEPOLARISING) {
        set(0, 0, 1.0 - 2.0 * p / 3.0);
        set(0, 3, 2.0 * p / 3.0);
        set(3, 3, 1.0 - 2.0 * p / 3.0);
        set(3, 0, 2.0 * p / 3.0);
        set(1, 1, 1.0 - 4.0 * p / 3.0);
        set(2, 2, 1.0 - 4.0 * p / 3.0);
    } else {
        const double s = sqrt(1.0 - p);
        set(0, 0, 1.0);
        set(0, 3, p);
        set(1, 1, s);
        set(2, 2, s);
        set(3, 3, 1.0 - p);
    }
    return M;
}

}  // namespace

std::vector<OpRec> dm_vector_ops(const std::vector<OpRec>& ops, int N)
{
    std::vector<OpRec> out;
    auto shifted = [&](const std::vector<int>& qs_) {
        std::vector<int> r;
        for (int q : qs_) r.push_back(q + N);
        return r;
    };
    auto push_pair = [&](int t, const Super4& M) {
        if (!out.empty()) {
            OpRec& prev = out.back();
            if (prev.kind == 4 && prev.ctrls.empty() && prev.target == t && prev.target2 == t + N) {
                prev.m4 = mat4_mul(M, prev.m4);  // M applied after prev
                return;
            }
        }
        OpRec op{};
        op.kind = 4;
        op.target = t;
        op.target2 = t + N;
        op.m4 = M;
        out.push_back(op);
    };
    for (const OpRec& op : ops) {
        if (op.kind == 0 && op.ctrls.empty()) {
            push_pair(op.target, gate_superop(op.u));
        } else if (op.kind == 0) {
            OpRec a = op, b = op;
            b.target = op.target + N;
            b.ctrls = shifted(op.ctrls);
            for (int k = 1; k < 8; k += 2) b.u[k] = -op.u[k];
            out.push_back(a);
            out.push_back(b);
        } else if (op.kind == 1) {
            OpRec a = op, b = op;
            b.target = op.target + N;
            b.ctrls = shifted(op.ctrls);
            out.push_back(a);
            out.push_back(b);
        } else if (op.kind == 2) {
            OpRec a = op, b = op;
            b.ctrls = shifted(op.ctrls);
            b.angle = -op.angle;
            out.push_back(a);
            out.push_back(b);
        } else if (op.kind == 3) {
            push_pair(op.target, channel_superop(op.channel, op.p));
        } else if (op.kind == 4) {
            // a two-qubit unitary: U on (t1, t2), conj(U) on (t1 + N, t2 + N)
            OpRec a = op, b = op;
            b.target = op.target + N;
            b.target2 = op.target2 + N;
            for (size_t k = 1; k < b.m4.size(); k += 2) b.m4[k] = -op.m4[k];
            out.push_back(a);
            out.push_back(b);
        }
    }
    return out;
}

}  // namespace qs
