/*
 * qstate -- C ABI of the MI355X (gfx950) state-vector / density-matrix gate
 * engine.  It implements the gate-application method of "QuEST and High
 * Performance Simulation of Quantum Computers" (Jones, Brown, Bush, Benjamin,
 * arXiv:1802.08032):
 *   - Sec. II.B.1, Eq. 1: a single-qubit gate G on qubit q updates every
 *     amplitude pair (alpha_a, alpha_{a + 2^q}) with bit q of a clear, in place;
 *     multi-controlled gates restrict this to pairs whose control bits are 1;
 *   - Sec. II.B.1, Eq. 2: an N-qubit density matrix rho is stored as a
 *     2N-qubit vector, rho[j][k] at index j + 2^N k, and G rho G^dagger is
 *     applied as G on qubit q and conj(G) on qubit q + N;
 *   - the decoherence channels named in the abstract and Sec. II.B.1
 *     (dephasing, depolarising) plus amplitude damping, as Kraus maps;
 *   - total probability, outcome probability and projective measurement.
 *
 * Conventions
 *   - Qubit q is bit q of the amplitude index (little endian).
 *   - Amplitudes are interleaved complex numbers in device memory:
 *     QS_C128 = two doubles (16 B), QS_C64 = two floats (8 B).  A register
 *     of n qubits holds 2^n amplitudes (QS_STATEVEC) or 4^n (QS_DENSITY).
 *   - Host-side 2x2 matrices are row-major qs_cplx[4] in double precision:
 *     u[2r + c] multiplies the bit=c amplitude into the bit=r amplitude.
 *     For QS_C64 registers the matrix is rounded to float once per call.
 *   - Every call returns a qs_status; QS_OK == 0.  Arguments are validated
 *     on the host before anything is launched, so a failed call leaves the
 *     register unchanged.  qs_last_error() gives the calling thread's last
 *     message.  Nothing in the library exits or aborts the process.
 *   - Gates, channels and initialisation are asynchronous on the register's
 *     HIP stream.  qs_calc_*, qs_measure* and qs_get_amps synchronise it
 *     (qs_measure* return once the outcome is known; the collapse that
 *     follows is queued on the stream like a gate).
 *   - The library is thread-safe across different registers; calls on one
 *     register must not overlap, nor calls that run one circuit handle (it
 *     keeps its compiled plan).
 */
#ifndef QSTATE_H
#define QSTATE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qs_env_s* qs_env;         /* device + profiling state            */
typedef struct qs_reg_s* qs_reg;         /* one quantum register (Qureg)        */
typedef struct qs_circuit_s* qs_circuit; /* recorded gate list + fusion plan    */
typedef struct qs_batch_s* qs_batch;     /* registers run by one launch         */

typedef enum { QS_STATEVEC = 0, QS_DENSITY = 1 } qs_kind;
typedef enum { QS_C64 = 1, QS_C128 = 2 } qs_prec;
typedef struct { double re, im; } qs_cplx;

typedef enum {
    QS_OK = 0,
    QS_E_ARG = -1,         /* qubit out of range, duplicate qubits, bad probability, ... */
    QS_E_KIND = -2,        /* operation not defined for this register kind               */
    QS_E_OOM = -3,         /* device allocation failed                                   */
    QS_E_DEVICE = -4,      /* a HIP call failed; qs_last_error() has hipGetErrorString   */
    QS_E_HANDLE = -5,      /* null, destroyed or foreign handle                          */
    QS_E_NOT_UNITARY = -6, /* max |U U^dagger - I| > 1e-10                               */
    QS_E_NOT_CPTP = -7     /* Kraus operators with max |sum K^dagger K - I| > 1e-10      */
} qs_status;

/* Channel kinds for qs_circuit_add_channel. */
typedef enum { QS_DEPHASING = 0, QS_DEPOLARISING = 1, QS_DAMPING = 2 } qs_channel;

/* Kernel classes for the per-launch profiler. */
typedef enum {
    QS_K_INIT = 0, QS_K_GATE = 1, QS_K_GATE_LOW = 2, QS_K_NOT = 3, QS_K_PHASE = 4,
    QS_K_DM_GATE = 5, QS_K_DM_CHANNEL = 6, QS_K_REDUCE = 7, QS_K_COLLAPSE = 8,
    QS_K_FUSED = 9, QS_K_COUNT = 10
} qs_kernel_class;

/* ---- environment ------------------------------------------------------- */

/* Bind HIP device `device` (createQuESTEnv, Sec. III.B.2).  *out is owned
 * by the caller and released with qs_env_destroy. */
qs_status qs_env_create(int device, qs_env* out);
qs_status qs_env_destroy(qs_env env);
/* Wait until all work on every register of this environment has finished
 * (syncQuESTEnv, Sec. III.B.2). */
qs_status qs_env_sync(qs_env env);
/* Text of the calling thread's most recent error (never NULL). */
const char* qs_last_error(void);

/* Per-launch timing: when enabled, every kernel launch is bracketed by two
 * HIP events on the register's stream.  qs_profile_read synchronises the
 * device, folds the recorded pairs into per-class totals and returns the
 * launch count and summed milliseconds of class `klass` since the last
 * reset. */
qs_status qs_profile_enable(qs_env env, int enable);
qs_status qs_profile_read(qs_env env, int klass, uint64_t* launches, double* total_ms);
qs_status qs_profile_reset(qs_env env);

/* ---- registers --------------------------------------------------------- */

/* Bytes of amplitude storage: (8 or 16) * 2^n for a state vector, * 4^n
 * for a density matrix (Sec. II.B.1: 16 x 2^n B in double precision).
 * Returns 0 for invalid arguments or sizes that overflow size_t. */
size_t qs_reg_bytes(int n, int kind, int prec);

/* Allocate a register of n qubits (1 <= n <= 40 for state vectors,
 * 1 <= n <= 20 for density matrices) on `hip_stream` (a hipStream_t, NULL
 * for the default stream).  Contents are undefined until an init call.
 * The library owns the memory; qs_reg_destroy frees it. */
qs_status qs_reg_create(qs_env env, int n, int kind, int prec, void* hip_stream, qs_reg* out);
/* As qs_reg_create, over caller-owned device memory `dev_ptr` of at least
 * qs_reg_bytes(n, kind, prec) bytes, 16-byte aligned.  The memory must
 * outlive the handle and is not freed by qs_reg_destroy. */
qs_status qs_reg_wrap(qs_env env, int n, int kind, int prec, void* dev_ptr, size_t bytes,
                      void* hip_stream, qs_reg* out);
qs_status qs_reg_destroy(qs_reg r);
/* Read back the register's shape; any output pointer may be NULL. */
qs_status qs_reg_info(qs_reg r, int* n, int* kind, int* prec, void** dev_ptr, void** hip_stream);

/* |0..0> (initZeroState, Sec. III.B.2), or |index><index| for a density matrix. */
qs_status qs_init_zero(qs_reg r);
/* Basis state |index>, 0 <= index < 2^n. */
qs_status qs_init_basis(qs_reg r, uint64_t index);
/* Direct amplitude access (Sec. II.B.1): copy `count` amplitudes starting
 * at raw vector index `start` (for a density matrix, index j + 2^N k) to or
 * from host memory.  Synchronous. */
qs_status qs_get_amps(qs_reg r, uint64_t start, uint64_t count, qs_cplx* host_out);
qs_status qs_set_amps(qs_reg r, uint64_t start, uint64_t count, const qs_cplx* host_in);

/* ---- gates (Eq. 1; on a density matrix, Eq. 2 with conj(u) on q + N) ---- */

/* Dense single-qubit unitary `u` on `target`. */
qs_status qs_unitary(qs_reg r, int target, const qs_cplx u[4]);
qs_status qs_controlled_unitary(qs_reg r, int control, int target, const qs_cplx u[4]);
/* Apply `u` on `target` to the pairs whose `n_controls` control bits are
 * all 1.  Controls must be distinct and differ from the target. */
qs_status qs_multi_controlled_unitary(qs_reg r, const int* controls, int n_controls,
                                      int target, const qs_cplx u[4]);
/* Multi-controlled NOT (CNOT for one control): a permutation of pairs. */
qs_status qs_multi_controlled_not(qs_reg r, const int* controls, int n_controls, int target);
/* Diagonal phase: amplitudes whose bits in `qubits` are all 1 are
 * multiplied by exp(i angle) (CZ is angle = pi on two qubits). */
qs_status qs_multi_controlled_phase(qs_reg r, const int* qubits, int n_qubits, double angle);

/* Named gates: thin wrappers over the calls above, with the same argument
 * checks and errors.
 *   qs_hadamard   H = [[1, 1], [1, -1]] / sqrt 2 on `target`
 *   qs_cnot       NOT on `target` where `control` is 1
 *   qs_cz         phase -1 where qubits q1 and q2 are both 1 (symmetric)
 *   qs_rotate_x   exp(-i theta X / 2) = [[c, -i s], [-i s, c]]
 *   qs_rotate_y   exp(-i theta Y / 2) = [[c, -s], [s, c]]
 *   qs_rotate_z   exp(-i theta Z / 2) = diag(e^(-i theta/2), e^(i theta/2))
 *   qs_t_gate     diag(1, e^(i pi/4))
 *   qs_sqrt_x     [[1+i, 1-i], [1-i, 1+i]] / 2   (its square is X)
 *   qs_sqrt_y     [[1+i, -1-i], [1+i, 1+i]] / 2  (its square is Y)
 * with c = cos(theta / 2), s = sin(theta / 2).  H, T, CZ, sqrt X and sqrt Y
 * are the gate set of the paper's random circuits (Sec. II.C). */
qs_status qs_hadamard(qs_reg r, int target);
qs_status qs_cnot(qs_reg r, int control, int target);
qs_status qs_cz(qs_reg r, int q1, int q2);
qs_status qs_rotate_x(qs_reg r, int target, double theta);
qs_status qs_rotate_y(qs_reg r, int target, double theta);
qs_status qs_rotate_z(qs_reg r, int target, double theta);
qs_status qs_t_gate(qs_reg r, int target);
qs_status qs_sqrt_x(qs_reg r, int target);
qs_status qs_sqrt_y(qs_reg r, int target);

/* ---- decoherence channels (density matrices only) ---------------------- */

/* rho -> (1-p) rho + p Z rho Z,                       0 <= p <= 1/2 */
qs_status qs_mix_dephasing(qs_reg r, int target, double p);
/* rho -> (1-p) rho + (p/3)(X rho X + Y rho Y + Z rho Z), 0 <= p <= 3/4 */
qs_status qs_mix_depolarising(qs_reg r, int target, double p);
/* Kraus {[[1,0],[0,sqrt(1-g)]], [[0,sqrt(g)],[0,0]]},   0 <= g <= 1 */
qs_status qs_mix_damping(qs_reg r, int target, double gamma);

/* ---- gates on several qubits and general Kraus maps --------------------- */
/* Sec. II.B.1: the pair update of Eq. 1 generalises to the group of 2^k
 * amplitudes that agree outside the k target bits, and the Eq. 2 identity
 * holds for multi-qubit gates.  Matrices are row-major 2^k x 2^k qs_cplx in
 * double precision; matrix index bit j corresponds to qubit targets[j]
 * (entry [r][c] maps the amplitude whose target bits spell c into the one
 * whose target bits spell r).  For QS_C64 registers they are rounded to
 * float once per call.  Each call copies its matrix to the register's
 * scratch memory on the register's stream and returns without waiting. */

/* Dense k-qubit unitary u on targets[0..k), k = 1..5, applied to the groups
 * whose `n_controls` control bits are all 1 (controls distinct and not
 * targets).  On a density matrix: u on the targets (controls as given), then
 * conj(u) on targets + N (controls + N), Eq. 2.  QS_E_ARG for a bad qubit
 * list or a non-finite entry, QS_E_NOT_UNITARY for max |u u^dagger - I| >
 * 1e-10. */
qs_status qs_multi_qubit_unitary(qs_reg r, const int* controls, int n_controls, const int* targets,
                                 int n_targets, const qs_cplx* u);
/* qs_multi_qubit_unitary on (target1, target2) with no controls: u is 4x4,
 * index = bit(target1) + 2 bit(target2). */
qs_status qs_two_qubit_unitary(qs_reg r, int target1, int target2, const qs_cplx u[16]);

/* General Kraus map rho -> sum_m K_m rho K_m^dagger on k = 1 or 2 target
 * qubits of a density matrix (the decoherence of Sec. II.B.1 in its general
 * form): `ops` holds n_ops operators of 2^k x 2^k, one after the other,
 * 1 <= n_ops <= 4^k.  Applied in one pass as the superoperator
 * S = sum_m conj(K_m) (x) K_m on (targets, targets + N), which the host forms
 * in double precision.  QS_E_KIND on a state vector; QS_E_NOT_CPTP when
 * max |sum_m K_m^dagger K_m - I| > 1e-10. */
qs_status qs_mix_multi_kraus(qs_reg r, const int* targets, int n_targets, const qs_cplx* ops, int n_ops);
qs_status qs_mix_kraus(qs_reg r, int target, const qs_cplx* ops, int n_ops);
qs_status qs_mix_two_qubit_kraus(qs_reg r, int target1, int target2, const qs_cplx* ops, int n_ops);

/* ---- initialisation variants, copies, overlaps, checkpoints -------------- */
/* Sec. II.B.1 allows direct reading and writing of the state; these build
 * common states on the device and read overlaps without copying the state
 * to the host.  Calls that take two registers need the same device,
 * precision and qubit count; they order the two registers' streams with
 * events (the reading call runs after earlier work on the other register,
 * and later work on that register runs after the read). */

/* |+>^n: every amplitude 2^(-n/2); on a density matrix |+><+|, every entry
 * 2^-N.  Write-only, asynchronous. */
qs_status qs_init_plus(qs_reg r);
/* r = |psi><psi| (density matrix r, entry j + 2^N k = psi_j conj(psi_k)) or
 * a copy of psi (state vector r), psi = the state vector `pure`.
 * Asynchronous. */
qs_status qs_init_pure_state(qs_reg r, qs_reg pure);
/* Copy the whole state of `src` into `dst` (same kind too).  Asynchronous. */
qs_status qs_clone(qs_reg dst, qs_reg src);
/* <bra|ket> = sum_i conj(bra_i) ket_i of two state vectors, accumulated in
 * double precision with compensated sums.  Synchronous. */
qs_status qs_calc_inner_product(qs_reg bra, qs_reg ket, qs_cplx* out);
/* Tr(rho^2) of a density matrix (the squared norm of its Eq. 2 vector, equal
 * to the purity for Hermitian rho), compensated, in double.  Synchronous. */
qs_status qs_calc_purity(qs_reg r, double* out);
/* Fidelity with the pure state `pure`: |<pure|r>|^2 for a state vector r,
 * <pure|rho|pure> (real part) for a density matrix r.  Synchronous. */
qs_status qs_calc_fidelity(qs_reg r, qs_reg pure, double* out);
/* Checkpoint: write the register to `path` (64-byte header: "QSTATE01",
 * int32 n, kind, prec, 0, uint64 amplitude count, 32 zero bytes; then the
 * raw amplitudes in the register's precision), streamed through two pinned
 * 64 MiB buffers so that device copies overlap file writes.  Synchronous;
 * QS_E_ARG on an I/O failure. */
qs_status qs_save_state(qs_reg r, const char* path);
/* Read a checkpoint written by qs_save_state into a register of the same
 * n, kind and precision.  The header and file size are checked before any
 * amplitude is written (QS_E_ARG, register unchanged); an I/O error later
 * leaves the register partly overwritten.  Synchronous. */
qs_status qs_load_state(qs_reg r, const char* path);

/* ---- probabilities and measurement -------------------------------------- */
/* The paper states no probability or measurement routine; these read the
 * state of Sec. II.B.1 in the standard way (Born rule), with the rounding
 * and draw conventions stated per call. */

/* sum |alpha|^2 (state vector) or trace (density matrix), accumulated in
 * double precision with compensated sums.  Synchronous. */
qs_status qs_calc_total_prob(qs_reg r, double* out);
/* Probability that `qubit` reads `outcome` (0 or 1).  Synchronous. */
qs_status qs_calc_prob_of_outcome(qs_reg r, int qubit, int outcome, double* out);
/* Projective measurement with the caller's uniform draw u01 in [0, 1):
 * p0 = P(qubit = 0) clamped to [0, 1]; outcome = (u01 < p0) ? 0 : 1; the
 * other branch is zeroed and the kept one scaled by 1/sqrt(p) (state
 * vector) or 1/p (density matrix), with the scale formed in double
 * precision.  *prob receives P(outcome).  Returns once the outcome is known
 * (the probabilities are read back); the collapse is queued on the
 * register's stream, so every later call sees the collapsed state. */
qs_status qs_measure(qs_reg r, int qubit, double u01, int* outcome, double* prob);
/* qs_measure with P(qubit = 0) = p0 and P(qubit = 1) = p1 supplied by the
 * caller instead of summed from the state: the probabilities the last pass
 * of qs_circuit_run_compiled_probs returns for the state it stored (p0 =
 * probs[1 + qubit], p1 = probs[0] - p0).  The outcome is (u01 < clamp(p0,
 * 0, 1)) ? 0 : 1 and the kept branch is scaled by 1/sqrt(p) (state vector)
 * or 1/p (density matrix) with p the supplied probability of that outcome.
 * QS_E_ARG for a negative or non-finite probability, a draw outside [0, 1)
 * or an outcome of probability 0.  Asynchronous: nothing is read back. */
qs_status qs_measure_given_probs(qs_reg r, int qubit, double p0, double p1, double u01, int* outcome,
                                 double* prob);
/* Measure every qubit, 0..n-1 in order, with draws u01[0..n-1] in [0, 1):
 * the result is that of n successive qs_measure calls (each qubit's
 * probability taken on the state its predecessors left; the outcomes are
 * the same up to draws within rounding of p0), computed from compensated
 * histograms of the unmeasured state (one full read, then reads of the
 * surviving 2^-10, 2^-20, ... of it) and one write-only collapse to the
 * measured basis entry.  outcomes[k] and probs[k] (either may be NULL)
 * receive qubit k's outcome and P(outcome).  u01 is read during the call
 * only.  QS_E_ARG for a NULL u01, a draw outside [0, 1) or an outcome of
 * zero probability; the register is unchanged then.  Returns once the
 * outcomes are known; the final collapse is queued on the register's
 * stream, as in qs_measure. */
qs_status qs_measure_all(qs_reg r, const double* u01, int* outcomes, double* probs);

/* ---- seeded draws (the paper leaves the source of measurement randomness
 * open; these calls give reproducible draws without caller-side RNG) ----- */

/* Uniform doubles in [0, 1) from the counter-based generator Philox4x64-10
 * (Salmon, Moraes, Dror and Shaw, SC'11) under key (seed, stream): draw k
 * is word k mod 4 of the ten-round Philox bijection of the 256-bit counter
 * k / 4 + 1, taken as (x >> 11) * 2^-53.  This is the stream of
 * numpy.random.Philox(key=[seed, stream]).  Writes out[0..count) = draws
 * first .. first + count - 1.  Host only; needs no device.  QS_E_ARG for a
 * NULL out or a negative count. */
qs_status qs_philox_draws(uint64_t seed, uint64_t stream, uint64_t first, int count, double* out);
/* Give `env` the draw stream (seed, stream) and rewind it to draw 0.  An
 * environment never seeded uses (0, 0). */
qs_status qs_env_seed(qs_env env, uint64_t seed, uint64_t stream);
/* qs_measure with the next draw of the register's environment stream.  The
 * stream advances by one draw when the call succeeds and not otherwise.
 * Registers sharing an environment take draws in call order (calls from
 * several threads at once take them in an unspecified order). */
qs_status qs_measure_seeded(qs_reg r, int qubit, int* outcome, double* prob);
/* qs_measure_all with the next n draws of the register's environment
 * stream (n = register qubits); advances the stream by n on success. */
qs_status qs_measure_all_seeded(qs_reg r, int* outcomes, double* probs);

/* ---- circuits: recorded gate lists with optional gate fusion ------------ */

qs_status qs_circuit_create(qs_circuit* out);
qs_status qs_circuit_destroy(qs_circuit c);
qs_status qs_circuit_add_unitary(qs_circuit c, const int* controls, int n_controls, int target,
                                 const qs_cplx u[4]);
qs_status qs_circuit_add_not(qs_circuit c, const int* controls, int n_controls, int target);
/* Record a dense two-qubit unitary u (4x4 row-major, index = bit(target1) +
 * 2 bit(target2), as qs_two_qubit_unitary; Sec. II.B.1 and, on a density
 * matrix, Eq. 2's conj(u) on target1 + N, target2 + N).  In fused runs it is
 * a 4x4 op of the pass that holds both targets.  QS_E_ARG for equal or
 * negative targets or a non-finite entry, QS_E_NOT_UNITARY for
 * max |u u^dagger - I| > 1e-10.  Not changed by qs_circuit_set_unitary. */
qs_status qs_circuit_add_two_qubit_unitary(qs_circuit c, int target1, int target2, const qs_cplx u[16]);
/* Change the parameters of recorded op `index` (0-based, in add order),
 * keeping its kind, target and controls: the matrix of a unitary, or the
 * angle of a phase.  QS_E_ARG if `index` holds another kind of op (or is out
 * of range); QS_E_NOT_UNITARY as for qs_circuit_add_unitary.  Later runs
 * use the new values (compiled passes are rebuilt from them; unchanged
 * kernel sources are reused); a batch sees them after qs_batch_update. */
qs_status qs_circuit_set_unitary(qs_circuit c, int index, const qs_cplx u[4]);
qs_status qs_circuit_set_phase(qs_circuit c, int index, double angle);
qs_status qs_circuit_add_phase(qs_circuit c, const int* qubits, int n_qubits, double angle);
qs_status qs_circuit_add_channel(qs_circuit c, int channel, int target, double p);
/* Number of recorded operations. */
qs_status qs_circuit_size(qs_circuit c, int* n_ops);
/* Apply the circuit to `r`.  fusion_qubits = 0 launches one kernel per
 * operation (the one-pass-per-gate method of Sec. II.B.1).  fusion_qubits
 * = k > 0 groups consecutive gates whose targets fit in a set of at most k
 * qubits and applies each group in one read and one write of the state
 * (gate fusion, Sec. II.B); density matrices use the run-time compiled
 * passes on their 2N-qubit vector (see qs_circuit_run_compiled), with k
 * counting vector qubits.  *n_passes (may be NULL) receives the number of
 * full-state kernel passes launched. */
qs_status qs_circuit_run(qs_reg r, qs_circuit c, int fusion_qubits, int* n_passes);
/* Fused run with an explicit tile shape through the generic pass kernel
 * (no run-time compilation, so any circuit starts at once): tiles of
 * 2^tile_qubits amplitudes held by 2^thread_bits threads, at most
 * max_phases register layouts per pass (0: default).  Uncontrolled dense
 * gates run as unit-diagonal cores with their diagonal part deferred to the
 * next op on the qubit (or the end of the circuit), as in the compiled
 * passes.  A density matrix runs as its 2N-qubit vector (Eq. 2: gates on q
 * and conj on q + N, channels as 4x4 superoperators on (q, q + N));
 * tile_qubits then counts vector qubits.  Shapes (thread_bits, tile_qubits
 * - thread_bits) compiled in: (6,3) (7,3) (8,3) (8,4) (9,3) (9,4) (10,3),
 * and for QS_C64 also (8,5) (9,5) (10,4).  QS_E_ARG for other shapes or a
 * tile wider than the register. */
qs_status qs_circuit_run_tiled(qs_reg r, qs_circuit c, int tile_qubits, int thread_bits,
                               int max_phases, int* n_passes);
/* As qs_circuit_run_tiled, but each pass runs a kernel generated for that
 * pass's structure (targets, controls, register layouts) and compiled for
 * gfx950 at run time; matrices and angles stay kernel data.  Each workgroup
 * loops over tiles and prefetches the next tile while computing the
 * current one.  contig_qubits (1..6, <= thread_bits; 0: 6) global qubits
 * 0..contig_qubits-1 stay on consecutive lanes whenever a tile is read or
 * written, i.e. HBM is accessed in contiguous runs of 2^contig_qubits
 * amplitudes; fewer pinned qubits leave more tile qubits for gates.  Compiled code
 * is cached in memory and on disk ($QS_JIT_CACHE, default
 * $HOME/.cache/qstate); the first run of a new structure pays the compile
 * time.  The compiled form is kept with the circuit until ops are added or
 * the register shape or tile changes.  Accepts 6..10 thread bits and 1..5
 * register bits with the tile in 160 KiB of LDS.  A density matrix runs as
 * its 2N-qubit vector (Eq. 2): a gate becomes the gate on q and its
 * conjugate on q + N, a channel a 4x4 superoperator on (q, q + N), and an
 * uncontrolled gate is merged with the channels that follow it on the same
 * qubit; tile_qubits then counts vector qubits (at most 2N). */
qs_status qs_circuit_run_compiled(qs_reg r, qs_circuit c, int tile_qubits, int thread_bits,
                                  int max_phases, int contig_qubits, int* n_passes);
/* qs_circuit_run_compiled starting from the basis state |basis_index>
 * (|j><j| for a density matrix): the first pass forms its tiles of that
 * state instead of reading the register, so the initialisation costs no
 * separate write pass and the first pass no read.  For an empty circuit
 * the register is simply set to the basis state.  QS_E_ARG for an index
 * outside [0, 2^n). */
qs_status qs_circuit_run_compiled_from_basis(qs_reg r, qs_circuit c, int tile_qubits, int thread_bits,
                                             int max_phases, int contig_qubits, uint64_t basis_index,
                                             int* n_passes);
/* qs_circuit_run_compiled (basis_index NULL) or
 * qs_circuit_run_compiled_from_basis (*basis_index) on a state vector whose
 * last pass also sums, as it stores the final state, the readouts of
 * Sec. II.B.1: probs[0] = sum of |alpha|^2 (calcTotalProb) and probs[1 + q]
 * = P(qubit q = 0) (calcProbOfOutcome) for q = 0..n-1, so that they cost no
 * further pass over the state.  Each lane adds |alpha|^2 in double
 * precision, the workgroups' sums are added in a fixed order with
 * compensation (results are reproducible run to run; they may differ from
 * qs_calc_total_prob / qs_calc_prob_of_outcome by rounding).  probs holds n
 * + 1 doubles; synchronous.  QS_E_KIND for a density matrix.  For an empty
 * circuit the sums come from the reduction kernels. */
qs_status qs_circuit_run_compiled_probs(qs_reg r, qs_circuit c, int tile_qubits, int thread_bits, int max_phases,
                                        int contig_qubits, const uint64_t* basis_index, double* probs,
                                        int* n_passes);
/* Host-only: the generated HIP source of pass `pass` for an n-qubit
 * register of kind `kind` and precision `prec` (copied into buf,
 * NUL-terminated, truncated to cap - 1 bytes; *len gets the full length,
 * *n_passes the pass count); pass -1 gives the last pass in the form
 * qs_circuit_run_compiled_probs runs (state vectors).  Needs no GPU. */
qs_status qs_circuit_source(qs_circuit c, int n, int kind, int prec, int tile_qubits, int thread_bits,
                            int max_phases, int contig_qubits, int pass, char* buf, size_t cap,
                            size_t* len, int* n_passes);
/* Host-only: the kernel data (matrices, core coefficients, deferred
 * factors) that pass `pass` of the same generated set reads through its
 * `mats` argument, as doubles (a QS_C64 pass receives them rounded to
 * float).  Copies min(cap, *len) values into buf (buf may be NULL when
 * cap is 0); *len gets the full count, *n_passes the pass count.  With the
 * source this lets a caller run or inspect a pass without a GPU.  Needs
 * no GPU. */
qs_status qs_circuit_pass_data(qs_circuit c, int n, int kind, int prec, int tile_qubits, int thread_bits,
                               int max_phases, int contig_qubits, int pass, double* buf, size_t cap,
                               size_t* len, int* n_passes);

/* ---- batches: many independent registers in one persistent launch ------- */

/* Bind `count` state-vector registers to `count` circuits (circuits[i] runs
 * on regs[i]).  All registers must share one environment and precision and
 * hold at least 9 qubits.  Every circuit is planned into fused passes of
 * tiles of tile_qubits qubits (9..13 for QS_C128, 9..14 for QS_C64); a
 * register narrower than that is a single tile of its own width.  A run is
 * one launch per pass level and tile shape: it applies pass p of every
 * register of that shape that has one, its tiles spread over all
 * workgroups (largest registers first); launch boundaries order a
 * register's passes, and no workgroup waits for another.  The batch keeps device copies of the
 * plans; registers and circuits must outlive it.  Parameter changes
 * (qs_circuit_set_*) are seen after qs_batch_update; adding ops to a
 * batched circuit is not supported.  Work runs on the batch's own stream, ordered after
 * and before the registers' streams. */
qs_status qs_batch_create(const qs_reg* regs, const qs_circuit* circuits, int count, int tile_qubits,
                          qs_batch* out);
qs_status qs_batch_destroy(qs_batch b);
/* Run every circuit once; init_zero != 0 first sets each register to |0..0>
 * inside the same launch.  Asynchronous. */
qs_status qs_batch_run(qs_batch b, int init_zero);
/* Record qs_batch_run(b, init_zero) into a HIP graph (replacing any earlier
 * one); qs_batch_replay launches it.  Asynchronous. */
qs_status qs_batch_capture(qs_batch b, int init_zero);
qs_status qs_batch_replay(qs_batch b);
/* Take the circuits' current parameters (qs_circuit_set_*) into the batch:
 * its device op table is rewritten on the batch stream, after earlier runs
 * and before later ones, so a captured graph replays with the new values
 * without being captured again.  Asynchronous (the host copy is taken
 * before the call returns). */
qs_status qs_batch_update(qs_batch b);
/* Per register i: p0[i] = P(qubit = 0), total[i] = total probability, in
 * double precision with compensated sums (either output may be NULL).
 * `qubit` must be below every register's size.  Synchronous. */
qs_status qs_batch_probs(qs_batch b, int qubit, double* p0, double* total);
/* Number of fused passes over all registers (for reporting). */
qs_status qs_batch_info(qs_batch b, int* n_regs, int* tile_qubits, int* n_passes);

#ifdef __cplusplus
}
#endif

#endif /* QSTATE_H */
