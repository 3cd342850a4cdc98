// Planner for fused state-vector passes (see qs_plan.hip).
#pragma once

#include <stdint.h>

#include <vector>

#include "qs_host.h"

namespace qs {

constexpr int kPhMax = 24;  // register layouts per pass, at most

// A register layout of a 2^(TB+RB)-amplitude tile: local qubit of each
// thread bit and of each register bit.
struct Layout {
    std::vector<int> thr;
    std::vector<int> reg;
};

struct PhasePlan {
    Layout lay;
    std::vector<int> ops;  // indices into the circuit, in application order
};

struct PassPlan {
    std::vector<int> S;    // global qubits of the tile, ascending (local j <-> S[j])
    std::vector<int> ops;  // indices into the circuit, in application order
    std::vector<PhasePlan> phases;
    Layout store;          // layout written back to HBM (coalesced)
};

uint64_t qubit_mask(const OpRec& op);
bool coalesced(const Layout& L, int contig);
// contig: global qubits 0..contig-1 sit on the first lanes whenever the tile
// is read from or written to HBM (contiguous runs of 2^contig amplitudes).
// lookahead: also try a partition whose tile sets look one pass ahead
// (slower planning; for plans that are compiled and reused).
// balance > 0: then move ops between neighbouring passes so that no pass
// needs much more than `balance` multiply-adds per amplitude while its
// neighbour needs less (the arithmetic at which a pass stops being bound by
// HBM), see rebalance().
std::vector<PassPlan> plan_passes(const std::vector<OpRec>& all, int n, int TB, int RB, int max_phases,
                                  int max_ops, int contig, bool lookahead = false, double balance = 0.0);
// Re-order the thread bits of every phase of P (register sets unchanged) so
// that a re-layout keeps the qubits of the wave-index bits (thread bits 6
// and up) in place wherever it can: such a re-layout moves data only
// between lanes of one wave and needs no workgroup barrier.  The first
// phase keeps qubits 0..contig-1 on thread bits 0..contig-1; the store
// layout becomes the last phase's with qubits 0..contig-1 moved there.
void assign_thread_positions(PassPlan& P, int TB, int contig);
// Plan P's phases again by a beam search over register sets (the `width`
// partial plans that leave the fewest ops survive each phase); replaces
// P's phases and returns true only if that needs fewer phases than P has.
bool replan_phases_beam(PassPlan& P, const std::vector<OpRec>& all, int TB, int RB, int max_phases, int contig,
                        int width);
// Within every phase of P, replace runs of ops that act on at most two
// register qubits and carry no thread or tile condition by their product
// (a 2x2 dense op or a 4x4 kind-4 op), wherever that takes fewer
// multiply-adds than applying them one by one.  Merged ops are appended to
// `ops`; the phases' index lists are rewritten.  Ops on disjoint qubits
// commute, so ops may move past each other when their qubits are disjoint.
void merge_phase_ops(PassPlan& P, std::vector<OpRec>& ops);
// LDS images (K values) of the local bits for a re-layout from A to B.
std::vector<uint32_t> swizzle(const Layout& A, const Layout& B, int K);

}  // namespace qs
