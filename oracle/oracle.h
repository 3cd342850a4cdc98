/*
 * Plain CPU oracle for the QuEST gate path -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the bench's CPU-baseline leg may load
 * this library.  It shares no source with the HIP library and is never on
 * the product path.
 *
 * Every routine is the direct definition of its operation, in complex128,
 * with no blocking, fusion or reordering:
 *   - single-qubit and multi-controlled gates: the amplitude-pair update of
 *     Eq. 1 (Sec. II.B.1), restricted to pairs whose control bits are all 1;
 *   - density matrices: rho stored as a 2N-qubit vector (Eq. 2) with
 *     rho[j][k] at index j + 2^N k; a gate G on qubit q is the two passes
 *     G on q, then conj(G) on q+N (the Choi-Jamiolkowski form of Sec. II.B.1);
 *   - decoherence channels: the Kraus sum  sum_m K_m B K_m^dagger  on every
 *     2x2 block B of rho selected by the target's row and column bit;
 *   - probabilities: Neumaier-compensated sums of |alpha|^2 or diag(rho);
 *   - measurement: p0 from the outcome-0 sum, outcome = (r < p0) ? 0 : 1,
 *     then collapse with the kept branch scaled by 1/sqrt(p) (state vector)
 *     or 1/p (density matrix).
 *
 * Qubit q is bit q of the amplitude index.  2x2 matrices are row-major,
 * element [r][c] at u[2r + c].  Complex numbers are C99 double complex
 * (two doubles: real, imaginary).
 *
 * Parity unpinned: none.  Every function is pinned by the tests against
 * Kronecker-product brute force, closed forms and invariants.
 */
#ifndef QUEST_ORACLE_H
#define QUEST_ORACLE_H

#include <complex.h>
#include <stdint.h>

typedef double complex or_cplx;

/* Gate record for the single-output evaluator or_sv_amp_after(). */
enum { OR_U = 0, OR_X = 1, OR_PHASE = 2 };
typedef struct {
    int kind;          /* OR_U, OR_X or OR_PHASE                       */
    int target;        /* target qubit (unused for OR_PHASE)           */
    uint64_t mask;     /* controls (OR_U, OR_X) or all qubits (PHASE)  */
    or_cplx u[4];      /* OR_U: row-major 2x2                          */
    double angle;      /* OR_PHASE: phase exp(i angle) on all-ones     */
} or_gate;

void or_init_basis(or_cplx* amp, uint64_t len, uint64_t index);

/* state vectors (n qubits, 2^n amplitudes) */
void or_sv_unitary(or_cplx* amp, int n, const int* ctrls, int nctrl, int t,
                   const or_cplx u[4]);
void or_sv_x(or_cplx* amp, int n, const int* ctrls, int nctrl, int t);
void or_sv_phase(or_cplx* amp, int n, const int* qubits, int nq, double angle);
double or_sv_total_prob(const or_cplx* amp, int n);
double or_sv_prob_outcome(const or_cplx* amp, int n, int q, int outcome);
int or_sv_measure(or_cplx* amp, int n, int q, double r, double* prob);

/* density matrices (N qubits, 4^N entries) */
void or_dm_unitary(or_cplx* rho, int N, const int* ctrls, int nctrl, int t,
                   const or_cplx u[4]);
void or_dm_x(or_cplx* rho, int N, const int* ctrls, int nctrl, int t);
void or_dm_phase(or_cplx* rho, int N, const int* qubits, int nq, double angle);
void or_dm_kraus(or_cplx* rho, int N, int t, const or_cplx* kraus, int nk);
void or_dm_dephasing(or_cplx* rho, int N, int t, double p);
void or_dm_depolarising(or_cplx* rho, int N, int t, double p);
void or_dm_damping(or_cplx* rho, int N, int t, double gamma);
double or_dm_total_prob(const or_cplx* rho, int N);
double or_dm_prob_outcome(const or_cplx* rho, int N, int q, int outcome);
int or_dm_measure(or_cplx* rho, int N, int q, double r, double* prob);

/* k-qubit gates (k = n_targets <= 5): U is 2^k x 2^k row-major, matrix
 * index bit j <-> qubit targets[j]; applied to every group of 2^k amplitudes
 * whose control bits are all 1.  On rho: U on the targets, then conj(U) on
 * targets + N (controls + N). */
void or_sv_multi_unitary(or_cplx* amp, int n, const int* ctrls, int nctrl, const int* targets, int nt,
                         const or_cplx* u);
void or_dm_multi_unitary(or_cplx* rho, int N, const int* ctrls, int nctrl, const int* targets, int nt,
                         const or_cplx* u);
/* Kraus map on k <= 2 qubits: nk row-major 2^k x 2^k operators. */
void or_dm_kraus_multi(or_cplx* rho, int N, const int* targets, int nt, const or_cplx* kraus, int nk);

/* Initialisation and overlaps. */
void or_init_uniform(or_cplx* amp, uint64_t len, double value);
void or_dm_init_pure(or_cplx* rho, int N, const or_cplx* psi);
or_cplx or_sv_inner_product(const or_cplx* bra, const or_cplx* ket, int n);
double or_dm_purity(const or_cplx* rho, int N);
double or_dm_fidelity_pure(const or_cplx* rho, int N, const or_cplx* psi);

/* One output amplitude of: product state (x)_q v_q, then gates[0..ng).
 * v holds n two-vectors, v[2q + b] = <b|v_q>.  Each gate is read as Eq. 1
 * for the single output element requested; cost 2^(#dense gates). */
or_cplx or_sv_amp_after(int n, const or_cplx* v, const or_gate* gates, int ng,
                        uint64_t index);

/* Thread count of the OpenMP loops, for timing only (results do not depend
 * on it).  Returns the previous count. */
int or_set_threads(int n);

/* Neumaier-compensated sum of x[0..len) (exposed for its own pin). */
double or_neumaier_sum(const double* x, uint64_t len);

#endif
