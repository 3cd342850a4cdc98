/*
 * Plain CPU oracle for the QuEST gate path -- TEST INFRASTRUCTURE ONLY.
 * Only the tests, the smoke check and the bench's CPU-baseline leg use it.
 * Definitions and conventions are listed in oracle.h.
 *
 * Loops over independent amplitude pairs may run under OpenMP; every pair
 * is still computed by the same expression, so the result does not depend
 * on the thread count.  Sums are sequential and Neumaier-compensated.
 */
#include "oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>

static uint64_t mask_of(const int* qs, int nq)
{
    uint64_t m = 0;
    for (int k = 0; k < nq; ++k) m |= (uint64_t)1 << qs[k];
    return m;
}

void or_init_basis(or_cplx* amp, uint64_t len, uint64_t index)
{
    for (uint64_t i = 0; i < len; ++i) amp[i] = 0;
    amp[index] = 1;
}

/* Eq. 1 (Sec. II.B.1): for every i in [0, 2^(n-1)),
 *   n_i = floor(i / 2^t) * 2^(t+1) + (i mod 2^t)
 * and the pair (alpha_{n_i}, alpha_{n_i + 2^t}) is replaced by G times it.
 * Multi-control generalisation: only pairs whose control bits are all 1. */
void or_sv_unitary(or_cplx* amp, int n, const int* ctrls, int nctrl, int t,
                   const or_cplx u[4])
{
    const uint64_t half = (uint64_t)1 << (n - 1);
    const uint64_t step = (uint64_t)1 << t;
    const uint64_t cmask = mask_of(ctrls, nctrl);
    const or_cplx g00 = u[0], g01 = u[1], g10 = u[2], g11 = u[3];
#pragma omp parallel for schedule(static) if (half >= 65536)
    for (int64_t ii = 0; ii < (int64_t)half; ++ii) {
        const uint64_t i = (uint64_t)ii;
        const uint64_t ni = (i / step) * (2 * step) + (i % step);
        if ((ni & cmask) != cmask) continue;
        const or_cplx a = amp[ni];
        const or_cplx b = amp[ni + step];
        amp[ni] = g00 * a + g01 * b;
        amp[ni + step] = g10 * a + g11 * b;
    }
}

void or_sv_x(or_cplx* amp, int n, const int* ctrls, int nctrl, int t)
{
    const or_cplx x[4] = {0, 1, 1, 0};
    or_sv_unitary(amp, n, ctrls, nctrl, t, x);
}

/* Diagonal multi-controlled phase: the amplitudes whose listed bits are all
 * 1 are multiplied by exp(i angle); every other amplitude is unchanged. */
void or_sv_phase(or_cplx* amp, int n, const int* qubits, int nq, double angle)
{
    const uint64_t len = (uint64_t)1 << n;
    const uint64_t m = mask_of(qubits, nq);
    const or_cplx f = cexp(I * angle);
#pragma omp parallel for schedule(static) if (len >= 65536)
    for (int64_t ii = 0; ii < (int64_t)len; ++ii) {
        const uint64_t i = (uint64_t)ii;
        if ((i & m) == m) amp[i] *= f;
    }
}

/* Neumaier (improved Kahan-Babuska) summation, Z. Angew. Math. Mech. 54
 * (1974) 39: carry the rounding error of every addition in c. */
double or_neumaier_sum(const double* x, uint64_t len)
{
    double s = 0.0, c = 0.0;
    for (uint64_t i = 0; i < len; ++i) {
        const double t = s + x[i];
        if (fabs(s) >= fabs(x[i])) c += (s - t) + x[i];
        else c += (x[i] - t) + s;
        s = t;
    }
    return s + c;
}

typedef struct { double s, c; } nsum;

static void nsum_add(nsum* a, double v)
{
    const double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}

static double abs2(or_cplx z) { return creal(z) * creal(z) + cimag(z) * cimag(z); }

double or_sv_total_prob(const or_cplx* amp, int n)
{
    nsum acc = {0.0, 0.0};
    const uint64_t len = (uint64_t)1 << n;
    for (uint64_t i = 0; i < len; ++i) nsum_add(&acc, abs2(amp[i]));
    return acc.s + acc.c;
}

double or_sv_prob_outcome(const or_cplx* amp, int n, int q, int outcome)
{
    nsum acc = {0.0, 0.0};
    const uint64_t len = (uint64_t)1 << n;
    for (uint64_t i = 0; i < len; ++i)
        if ((int)((i >> q) & 1) == outcome) nsum_add(&acc, abs2(amp[i]));
    return acc.s + acc.c;
}

/* Measurement of qubit q with the uniform draw r in [0, 1):
 * p0 = P(q = 0) clamped to [0, 1]; outcome 0 iff r < p0; p = P(q = outcome)
 * summed directly; kept amplitudes scaled by 1/sqrt(p), the rest zeroed. */
int or_sv_measure(or_cplx* amp, int n, int q, double r, double* prob)
{
    double p0 = or_sv_prob_outcome(amp, n, q, 0);
    if (p0 < 0.0) p0 = 0.0;
    if (p0 > 1.0) p0 = 1.0;
    const int outcome = (r < p0) ? 0 : 1;
    const double p = or_sv_prob_outcome(amp, n, q, outcome);
    const double scale = 1.0 / sqrt(p);
    const uint64_t len = (uint64_t)1 << n;
    for (uint64_t i = 0; i < len; ++i) {
        if ((int)((i >> q) & 1) == outcome) amp[i] *= scale;
        else amp[i] = 0;
    }
    if (prob) *prob = p;
    return outcome;
}

/* ---- density matrices: rho as the 2N-qubit vector of Eq. 2 ----------- */

/* G rho G^dagger as conj(G) on qubit t+N after G on qubit t (Sec. II.B.1);
 * controls c act on rows in the first pass and as c+N on columns in the
 * second. */
void or_dm_unitary(or_cplx* rho, int N, const int* ctrls, int nctrl, int t,
                   const or_cplx u[4])
{
    int* cshift = (int*)malloc(sizeof(int) * (nctrl > 0 ? nctrl : 1));
    for (int k = 0; k < nctrl; ++k) cshift[k] = ctrls[k] + N;
    const or_cplx uc[4] = {conj(u[0]), conj(u[1]), conj(u[2]), conj(u[3])};
    or_sv_unitary(rho, 2 * N, ctrls, nctrl, t, u);
    or_sv_unitary(rho, 2 * N, cshift, nctrl, t + N, uc);
    free(cshift);
}

void or_dm_x(or_cplx* rho, int N, const int* ctrls, int nctrl, int t)
{
    const or_cplx x[4] = {0, 1, 1, 0};
    or_dm_unitary(rho, N, ctrls, nctrl, t, x);
}

void or_dm_phase(or_cplx* rho, int N, const int* qubits, int nq, double angle)
{
    int* qshift = (int*)malloc(sizeof(int) * (nq > 0 ? nq : 1));
    for (int k = 0; k < nq; ++k) qshift[k] = qubits[k] + N;
    or_sv_phase(rho, 2 * N, qubits, nq, angle);
    or_sv_phase(rho, 2 * N, qshift, nq, -angle);
    free(qshift);
}

/* Kraus map on qubit t: every 2x2 block B of rho that varies only the row
 * bit t and the column bit t is replaced by sum_m K_m B K_m^dagger, with
 * plain 2x2 matrix products. */
void or_dm_kraus(or_cplx* rho, int N, int t, const or_cplx* kraus, int nk)
{
    const uint64_t dim = (uint64_t)1 << N;
    const uint64_t tb = (uint64_t)1 << t;
    /* column blocks outermost, so that the inner loop walks rows, which are
     * contiguous in the vector; every block is computed the same way */
#pragma omp parallel for schedule(static) if (dim >= 256)
    for (int64_t kk = 0; kk < (int64_t)dim; ++kk) {
        const uint64_t k = (uint64_t)kk;
        if (k & tb) continue;
        for (uint64_t j = 0; j < dim; ++j) {
            if (j & tb) continue;
            or_cplx B[2][2], S[2][2] = {{0, 0}, {0, 0}};
            for (int r = 0; r < 2; ++r)
                for (int c = 0; c < 2; ++c)
                    B[r][c] = rho[(j | (r ? tb : 0)) + dim * (k | (c ? tb : 0))];
            for (int m = 0; m < nk; ++m) {
                const or_cplx* K = kraus + 4 * m;
                or_cplx KB[2][2];
                for (int r = 0; r < 2; ++r)
                    for (int c = 0; c < 2; ++c)
                        KB[r][c] = K[2 * r + 0] * B[0][c] + K[2 * r + 1] * B[1][c];
                /* (K B K^dagger)[r][c] = sum_s (K B)[r][s] conj(K[c][s]) */
                for (int r = 0; r < 2; ++r)
                    for (int c = 0; c < 2; ++c)
                        S[r][c] += KB[r][0] * conj(K[2 * c + 0]) + KB[r][1] * conj(K[2 * c + 1]);
            }
            for (int r = 0; r < 2; ++r)
                for (int c = 0; c < 2; ++c)
                    rho[(j | (r ? tb : 0)) + dim * (k | (c ? tb : 0))] = S[r][c];
        }
    }
}

/* Dephasing: rho -> (1-p) rho + p Z rho Z, Kraus {sqrt(1-p) I, sqrt(p) Z}. */
void or_dm_dephasing(or_cplx* rho, int N, int t, double p)
{
    const double a = sqrt(1.0 - p), b = sqrt(p);
    const or_cplx K[8] = {a, 0, 0, a,   b, 0, 0, -b};
    or_dm_kraus(rho, N, t, K, 2);
}

/* Depolarising: rho -> (1-p) rho + (p/3)(X rho X + Y rho Y + Z rho Z). */
void or_dm_depolarising(or_cplx* rho, int N, int t, double p)
{
    const double a = sqrt(1.0 - p), b = sqrt(p / 3.0);
    const or_cplx K[16] = {a, 0, 0, a,
                           0, b, b, 0,
                           0, -I * b, I * b, 0,
                           b, 0, 0, -b};
    or_dm_kraus(rho, N, t, K, 4);
}

/* Amplitude damping: K0 = [[1, 0], [0, sqrt(1-g)]], K1 = [[0, sqrt(g)], [0, 0]]. */
void or_dm_damping(or_cplx* rho, int N, int t, double gamma)
{
    const or_cplx K[8] = {1, 0, 0, sqrt(1.0 - gamma),   0, sqrt(gamma), 0, 0};
    or_dm_kraus(rho, N, t, K, 2);
}

/* Total probability of a density matrix: its trace, sum_j Re rho[j][j]. */
double or_dm_total_prob(const or_cplx* rho, int N)
{
    const uint64_t dim = (uint64_t)1 << N;
    nsum acc = {0.0, 0.0};
    for (uint64_t j = 0; j < dim; ++j) nsum_add(&acc, creal(rho[j + dim * j]));
    return acc.s + acc.c;
}

double or_dm_prob_outcome(const or_cplx* rho, int N, int q, int outcome)
{
    const uint64_t dim = (uint64_t)1 << N;
    nsum acc = {0.0, 0.0};
    for (uint64_t j = 0; j < dim; ++j)
        if ((int)((j >> q) & 1) == outcome) nsum_add(&acc, creal(rho[j + dim * j]));
    return acc.s + acc.c;
}

/* Projective measurement of qubit q: rho -> P rho P / p with P the
 * projector on the outcome; entries with row or column bit q != outcome
 * vanish, the rest are divided by p. */
int or_dm_measure(or_cplx* rho, int N, int q, double r, double* prob)
{
    double p0 = or_dm_prob_outcome(rho, N, q, 0);
    if (p0 < 0.0) p0 = 0.0;
    if (p0 > 1.0) p0 = 1.0;
    const int outcome = (r < p0) ? 0 : 1;
    const double p = or_dm_prob_outcome(rho, N, q, outcome);
    const double scale = 1.0 / p;
    const uint64_t dim = (uint64_t)1 << N;
    for (uint64_t k = 0; k < dim; ++k)
        for (uint64_t j = 0; j < dim; ++j) {
            const int keep = ((int)((j >> q) & 1) == outcome) && ((int)((k >> q) & 1) == outcome);
            if (keep) rho[j + dim * k] *= scale;
            else rho[j + dim * k] = 0;
        }
    if (prob) *prob = p;
    return outcome;
}

/* ---- multi-qubit gates and maps ----------------------------------------- */

/* Offset of matrix index a on the target qubits: bit j of a sits at bit
 * targets[j] of the amplitude index. */
static uint64_t spread(uint64_t a, const int* targets, int nt)
{
    uint64_t o = 0;
    for (int j = 0; j < nt; ++j)
        if ((a >> j) & 1) o |= (uint64_t)1 << targets[j];
    return o;
}

/* A k-qubit gate (Sec. II.B.1: the pair update of Eq. 1 holds for
 * multi-qubit gates with groups of 2^k amplitudes in place of pairs): for
 * every index b whose target bits are all 0 and whose control bits are all
 * 1, the 2^k amplitudes x_a = alpha_{b + spread(a)} are replaced by U x.
 * u is 2^k x 2^k row-major, u[r * 2^k + c]. */
void or_sv_multi_unitary(or_cplx* amp, int n, const int* ctrls, int nctrl, const int* targets, int nt,
                         const or_cplx* u)
{
    const uint64_t len = (uint64_t)1 << n;
    const uint64_t tmask = mask_of(targets, nt), cmask = mask_of(ctrls, nctrl);
    const int d = 1 << nt;
#pragma omp parallel for schedule(static) if (len >= 65536)
    for (int64_t bb = 0; bb < (int64_t)len; ++bb) {
        const uint64_t b = (uint64_t)bb;
        if ((b & tmask) != 0 || (b & cmask) != cmask) continue;
        or_cplx x[32], y[32];
        for (int a = 0; a < d; ++a) x[a] = amp[b + spread((uint64_t)a, targets, nt)];
        for (int r = 0; r < d; ++r) {
            or_cplx acc = 0;
            for (int c = 0; c < d; ++c) acc += u[r * d + c] * x[c];
            y[r] = acc;
        }
        for (int a = 0; a < d; ++a) amp[b + spread((uint64_t)a, targets, nt)] = y[a];
    }
}

/* Eq. 2 for a k-qubit gate: U on the row qubits, then conj(U) on the column
 * qubits (targets + N, controls + N). */
void or_dm_multi_unitary(or_cplx* rho, int N, const int* ctrls, int nctrl, const int* targets, int nt,
                         const or_cplx* u)
{
    const int d = 1 << nt;
    int cs[64], ts[8];
    for (int k = 0; k < nctrl; ++k) cs[k] = ctrls[k] + N;
    for (int k = 0; k < nt; ++k) ts[k] = targets[k] + N;
    or_cplx* uc = (or_cplx*)malloc(sizeof(or_cplx) * (size_t)d * (size_t)d);
    for (int k = 0; k < d * d; ++k) uc[k] = conj(u[k]);
    or_sv_multi_unitary(rho, 2 * N, ctrls, nctrl, targets, nt, u);
    or_sv_multi_unitary(rho, 2 * N, cs, nctrl, ts, nt, uc);
    free(uc);
}

/* Kraus map on the qubits `targets` (k of them, k <= 2): every 2^k x 2^k
 * block B of rho whose row and column indices vary only in the target bits
 * is replaced by sum_m K_m B K_m^dagger, by plain matrix products.  kraus
 * holds nk row-major 2^k x 2^k matrices one after the other. */
void or_dm_kraus_multi(or_cplx* rho, int N, const int* targets, int nt, const or_cplx* kraus, int nk)
{
    const uint64_t dim = (uint64_t)1 << N;
    const uint64_t tmask = mask_of(targets, nt);
    const int d = 1 << nt;
#pragma omp parallel for schedule(static) if (dim >= 256)
    for (int64_t kk = 0; kk < (int64_t)dim; ++kk) {
        const uint64_t k = (uint64_t)kk;
        if (k & tmask) continue;
        for (uint64_t j = 0; j < dim; ++j) {
            if (j & tmask) continue;
            or_cplx B[4][4], S[4][4];
            for (int r = 0; r < d; ++r)
                for (int c = 0; c < d; ++c) {
                    B[r][c] = rho[(j | spread((uint64_t)r, targets, nt)) + dim * (k | spread((uint64_t)c, targets, nt))];
                    S[r][c] = 0;
                }
            for (int m = 0; m < nk; ++m) {
                const or_cplx* K = kraus + (size_t)m * d * d;
                or_cplx KB[4][4];
                for (int r = 0; r < d; ++r)
                    for (int c = 0; c < d; ++c) {
                        or_cplx acc = 0;
                        for (int s = 0; s < d; ++s) acc += K[r * d + s] * B[s][c];
                        KB[r][c] = acc;
                    }
                for (int r = 0; r < d; ++r)
                    for (int c = 0; c < d; ++c) {
                        or_cplx acc = 0;
                        for (int s = 0; s < d; ++s) acc += KB[r][s] * conj(K[c * d + s]);
                        S[r][c] += acc;
                    }
            }
            for (int r = 0; r < d; ++r)
                for (int c = 0; c < d; ++c)
                    rho[(j | spread((uint64_t)r, targets, nt)) + dim * (k | spread((uint64_t)c, targets, nt))] = S[r][c];
        }
    }
}

/* ---- state initialisation and overlaps ---------------------------------- */

/* |+>^n = H^(x)n |0..0>: every amplitude 2^(-n/2).  For a density matrix
 * (len = 4^N) the same routine with value 2^(-N) gives |+><+|. */
void or_init_uniform(or_cplx* amp, uint64_t len, double value)
{
    for (uint64_t i = 0; i < len; ++i) amp[i] = value;
}

/* rho = |psi><psi|: rho[j][k] = psi_j conj(psi_k), stored at j + 2^N k. */
void or_dm_init_pure(or_cplx* rho, int N, const or_cplx* psi)
{
    const uint64_t dim = (uint64_t)1 << N;
    for (uint64_t k = 0; k < dim; ++k)
        for (uint64_t j = 0; j < dim; ++j) rho[j + dim * k] = psi[j] * conj(psi[k]);
}

/* <bra|ket> = sum_i conj(bra_i) ket_i, real and imaginary parts summed
 * with Neumaier compensation. */
or_cplx or_sv_inner_product(const or_cplx* bra, const or_cplx* ket, int n)
{
    const uint64_t len = (uint64_t)1 << n;
    nsum re = {0.0, 0.0}, im = {0.0, 0.0};
    for (uint64_t i = 0; i < len; ++i) {
        const or_cplx z = conj(bra[i]) * ket[i];
        nsum_add(&re, creal(z));
        nsum_add(&im, cimag(z));
    }
    return (re.s + re.c) + I * (im.s + im.c);
}

/* Purity Tr(rho^2) = sum_jk rho_jk rho_kj = sum_jk |rho_jk|^2 for Hermitian
 * rho (Neumaier sum over every entry). */
double or_dm_purity(const or_cplx* rho, int N)
{
    const uint64_t len = (uint64_t)1 << (2 * N);
    nsum acc = {0.0, 0.0};
    for (uint64_t i = 0; i < len; ++i) nsum_add(&acc, abs2(rho[i]));
    return acc.s + acc.c;
}

/* Fidelity of rho with the pure state psi: <psi|rho|psi> =
 * sum_jk conj(psi_j) rho_jk psi_k (its real part; the imaginary part
 * vanishes for Hermitian rho). */
double or_dm_fidelity_pure(const or_cplx* rho, int N, const or_cplx* psi)
{
    const uint64_t dim = (uint64_t)1 << N;
    nsum acc = {0.0, 0.0};
    for (uint64_t k = 0; k < dim; ++k)
        for (uint64_t j = 0; j < dim; ++j) nsum_add(&acc, creal(conj(psi[j]) * rho[j + dim * k] * psi[k]));
    return acc.s + acc.c;
}

/* ---- single output amplitude ------------------------------------------ */

static or_cplx amp_rec(int n, const or_cplx* v, const or_gate* g, int ng, uint64_t i)
{
    if (ng == 0) {
        or_cplx a = 1;
        for (int q = 0; q < n; ++q) a *= v[2 * q + (int)((i >> q) & 1)];
        return a;
    }
    const or_gate* G = &g[ng - 1];
    if (G->kind == OR_PHASE) {
        const or_cplx a = amp_rec(n, v, g, ng - 1, i);
        return ((i & G->mask) == G->mask) ? a * cexp(I * G->angle) : a;
    }
    if ((i & G->mask) != G->mask) return amp_rec(n, v, g, ng - 1, i);
    const uint64_t tb = (uint64_t)1 << G->target;
    if (G->kind == OR_X) return amp_rec(n, v, g, ng - 1, i ^ tb);
    /* Eq. 1 read for one element: alpha'_i = G[b][0] alpha_{i, t=0} + G[b][1] alpha_{i, t=1} */
    const int b = (int)((i >> G->target) & 1);
    const or_cplx a0 = amp_rec(n, v, g, ng - 1, i & ~tb);
    const or_cplx a1 = amp_rec(n, v, g, ng - 1, i | tb);
    return G->u[2 * b + 0] * a0 + G->u[2 * b + 1] * a1;
}

or_cplx or_sv_amp_after(int n, const or_cplx* v, const or_gate* gates, int ng,
                        uint64_t index)
{
    return amp_rec(n, v, gates, ng, index);
}

int or_set_threads(int n)
{
    const int prev = omp_get_max_threads();
    omp_set_num_threads(n);
    return prev;
}
