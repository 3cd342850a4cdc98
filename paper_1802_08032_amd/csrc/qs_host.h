// Host-side structures behind the opaque C-ABI handles.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>
#include <vector>

#include "qs_internal.h"
#include "qstate.h"

struct qs_env_s {
    uint32_t magic;
    int device;
    bool profile;
    struct Rec {
        int klass;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    uint64_t launches[QS_K_COUNT];
    double ms[QS_K_COUNT];
    std::mutex mu;
    // measurement draw stream (qs_env_seed): Philox key and next draw index
    uint64_t rng_seed = 0, rng_stream = 0, rng_next = 0;
    // reduction scratch of destroyed registers, reused by new ones so that
    // register turnover never frees device memory (which would synchronise
    // the whole device)
    std::vector<std::pair<double*, double*>> scratch_pool;
};

struct qs_reg_s {
    uint32_t magic;
    qs_env env;
    int n;         // qubits (N for a density matrix)
    int nbits;     // index bits: n (state vector) or 2n (density matrix)
    int kind;
    int prec;
    void* amp;
    size_t bytes;
    bool owned;
    hipStream_t stream;
    double* scratch;     // device: reduction partials + 2 results
    double* host_res;    // pinned host: 2 doubles
};

// One recorded circuit operation.
struct OpRec {
    int kind;            // 0 dense, 1 not, 2 phase, 3 channel, 4 dense 4x4 on (target, target2)
    int target;
    int channel;
    std::vector<int> ctrls;  // controls (dense/not/4x4) or all qubits (phase)
    double u[8];
    double angle;
    double p;
    int target2 = -1;        // kind 4: second target (the high bit of the 4-index)
    std::vector<double> m4;  // kind 4: row-major 4x4 complex, index = bit(target) + 2 bit(target2)
};

namespace qs {
struct JitPlan;
void jit_plan_free(JitPlan* p);
struct BatchPlans;
void batch_plans_free(BatchPlans* p);
}  // namespace qs

struct qs_circuit_s {
    uint32_t magic;
    std::vector<OpRec> ops;
    uint64_t version = 0;  // bumped by every parameter change (qs_circuit_set_*)
    qs::JitPlan* jit = nullptr;  // cached run-time compiled form (qs_jit.hip)
};

// A batch of registers run together by one persistent launch (qs_fused.hip).
struct qs_batch_s {
    uint32_t magic;
    qs_env env;
    int prec;
    int TB, RB;
    int count;
    int grid;
    int passes_total;
    hipStream_t stream;            // the batch's own stream (capturable)
    std::vector<qs_reg> regs;
    std::vector<hipStream_t> reg_streams;  // distinct streams of the registers
    hipEvent_t ev_in, ev_out;
    void* dbuf = nullptr;          // BatchReg[] + BatchItem[] + FPass[] + FOp[] + 4x4 table
    size_t off_regs, off_order, off_passes, off_ops, off_m4;
    int nitems = 0;
    // launches in order: pass level by pass level, one per tile shape that
    // has items at that level (registers narrower than the batch tile are
    // one tile of their own width)
    struct Launch {
        int TB, RB, off, count, grid;
    };
    std::vector<Launch> launches;
    std::vector<int> reg_TB, reg_RB;  // tile shape of each register
    double* dprobs = nullptr;      // 2 doubles per register
    double* hprobs = nullptr;      // pinned copy
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // parameter updates (qs_batch_update): the circuits, their pass plans,
    // the range of op slots and 4x4 table entries each register's lowered
    // ops occupy, and host copies of the op table and the 4x4 table
    std::vector<const std::vector<OpRec>*> circ_ops;
    qs::BatchPlans* plans = nullptr;
    std::vector<size_t> reg_op_begin, reg_op_count, reg_m4_begin, reg_m4_count;
    std::vector<char> host_ops;
    std::vector<double> host_m4;
    // host sources of the asynchronous uploads on the batch stream (kept
    // until the batch is destroyed)
    std::vector<char> host_plan, host_m4b;
};

namespace qs {

qs_status set_error(qs_status s, const std::string& msg);
qs_status hip_error(hipError_t e, const char* what);

// Launch `f` on the register's stream, bracketed by profiling events when
// the environment profiles.  f(int* klass) returns hipError_t and may
// overwrite the kernel class.
template <class F>
qs_status profiled(qs_reg r, int klass, F&& f)
{
    qs_env env = r->env;
    hipEvent_t a = nullptr, b = nullptr;
    if (env->profile) {
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
            return hip_error(hipGetLastError(), "hipEventCreate");
        (void)hipEventRecord(a, r->stream);
    }
    const hipError_t e = f(&klass);
    if (env->profile) {
        (void)hipEventRecord(b, r->stream);
        std::lock_guard<std::mutex> g(env->mu);
        env->recs.push_back({klass, a, b});
    }
    if (e != hipSuccess) return hip_error(e, "kernel launch");
    return QS_OK;
}

// Fused execution of a state-vector circuit (qs_fused.hip): tiles of
// 2^(TB+RB) amplitudes, 2^TB threads, at most max_phases register layouts
// per pass.
struct FusedConfig {
    int TB, RB, max_phases;
    int contig = 6;  // low qubits kept on consecutive lanes for HBM access
};
bool fused_shape_supported(int prec, int TB, int RB);
FusedConfig default_fused_config(int prec, int k, int n);
qs_status run_fused_sv(qs_reg r, const std::vector<OpRec>& ops, FusedConfig cfg, int* passes);
// Batched registers (qs_fused.hip).
qs_status batch_build(qs_batch_s* b, const std::vector<qs_reg>& regs,
                      const std::vector<const std::vector<OpRec>*>& circs, int K);
hipError_t batch_launch(qs_batch_s* b, int init);
hipError_t batch_probs_launch(qs_batch_s* b, int q, double* dev_out);
// Rewrite the matrices and phase factors of the batch's op table from the
// circuits' current parameters and upload it on the batch stream.
qs_status batch_update(qs_batch_s* b);
// Eq. 2 on the 2N-qubit vector of a density matrix: gates become a gate on
// q and its conjugate on q+N, channels become 4x4 superoperators on
// (q, q+N); an uncontrolled gate and the channels that follow it on the same
// qubit are merged into one 4x4 (qs_plan.hip).
std::vector<OpRec> dm_vector_ops(const std::vector<OpRec>& ops, int N);
// Run-time compiled passes (qs_jit.hip).
// init_index != nullptr: the first pass forms the basis state |*init_index>
// (|j><j| for a density matrix) instead of reading the register.
// readout != nullptr (state vectors): the last pass also sums the total
// probability and P(q = 0) for every qubit q into readout[0], readout[1 + q]
// (synchronous).
qs_status run_compiled_sv(qs_reg r, qs_circuit_s* c, FusedConfig cfg, int* passes,
                          const uint64_t* init_index = nullptr, double* readout = nullptr);
// readout: the last source is that pass with the readout sums.
qs_status generate_sources(const std::vector<OpRec>& ops, int n, int kind, int prec, FusedConfig cfg,
                           std::vector<std::string>& out, std::vector<std::vector<double>>* mats = nullptr,
                           bool readout = false);
// Per-operation execution of one recorded op (qs_api.hip).
qs_status apply_op(qs_reg r, const OpRec& op);

}  // namespace qs
