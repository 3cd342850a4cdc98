// Internal declarations shared by the C-ABI layer and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qstate.h"

namespace qs {

// Up to 64 bit positions to insert into a compact loop index, ascending.
// After insertion the bits in `ones` are set (controls), the rest are 0.
struct BitInsert {
    int count;
    int pos[63];
    uint64_t ones;
};

// 2x2 complex matrix, row-major, real/imag interleaved.
template <typename T>
struct Mat2 {
    T m[8];
};

struct Launch {
    hipStream_t stream;
    int device;
};

// Builds the insertion spec for the given positions (any order) and ones mask.
BitInsert make_insert(const int* positions, int count, uint64_t ones);

// --- state-vector kernels -------------------------------------------------
// Every amplitude 0 except `index`, which becomes (re, im).  Write-only.
template <typename T> hipError_t launch_init_basis(const Launch& L, void* amp, uint64_t len, uint64_t index,
                                                   double re, double im);
template <typename T> hipError_t launch_gate(const Launch& L, void* amp, int nbits, int t,
                                             const int* ctrls, int nc, const Mat2<T>& u, int* klass);
template <typename T> hipError_t launch_not(const Launch& L, void* amp, int nbits, int t,
                                            const int* ctrls, int nc);
// Multiply by f every amplitude with all bits of `mask` set, except those
// that also have all bits of `skip` set (skip == 0: no exception).
template <typename T> hipError_t launch_phase(const Launch& L, void* amp, int nbits, uint64_t mask,
                                              uint64_t skip, double fre, double fim);

// --- density-matrix kernels ------------------------------------------------
template <typename T> hipError_t launch_dm_gate(const Launch& L, void* rho, int N, int t,
                                                const int* ctrls, int nc, const Mat2<T>& u);
template <typename T> hipError_t launch_dm_channel(const Launch& L, void* rho, int N, int t,
                                                   int channel, double p);

// --- reductions and collapse ----------------------------------------------
// Sum of |alpha|^2 split by bit q (q < 0: one total sum in out[0]).  Writes
// {sum over bit q == 0, sum over bit q == 1} as doubles to `dev_out`.
// `partials` must hold 2 * 2 * kReduceBlocks doubles.
constexpr int kReduceBlocks = 1024;
template <typename T> hipError_t launch_prob_sv(const Launch& L, const void* amp, int nbits, int q,
                                                double* partials, double* dev_out);
// Sum of |alpha|^2 over the indices whose bit q equals `outcome`, reading
// only those (half the state when q is at least the line bits: 3 for
// complex128, 4 for complex64).  Writes {sum, 0} to `dev_out`.
template <typename T> hipError_t launch_prob_half_sv(const Launch& L, const void* amp, int nbits, int q,
                                                     int outcome, double* partials, double* dev_out);
template <typename T> hipError_t launch_prob_dm(const Launch& L, const void* rho, int N, int q,
                                                double* partials, double* dev_out);
// out[j] = sum of part[i * cols + j] over rows i = 0..rows-1 (compensated,
// in row order).
hipError_t launch_sum_columns(const Launch& L, const double* part, int rows, int cols, double* out);
template <typename T> hipError_t launch_collapse_sv(const Launch& L, void* amp, int nbits, int q,
                                                    int outcome, double scale);
template <typename T> hipError_t launch_collapse_dm(const Launch& L, void* rho, int N, int q,
                                                    int outcome, double scale);

// Register scratch (device doubles): reduction partials, two results, then
// two k-qubit matrices of up to 32 x 32 complex entries (a gate and its
// conjugate, or a superoperator).
constexpr int kScratchMatOff = 4 * kReduceBlocks + 8;
constexpr int kScratchMatDoubles = 2 * 32 * 32 * 2;
constexpr int kScratchDoubles = kScratchMatOff + kScratchMatDoubles;

// --- k-qubit groups, initialisation variants, overlaps ---------------------
// Replace every group of 2^k amplitudes (k = 1..5 targets; matrix index bit j
// <-> targets[j]) whose control bits are all 1 by dev_m times it; dev_m is a
// device array of 2^k x 2^k complex T pairs, row-major.
template <typename T> hipError_t launch_group_gate(const Launch& L, void* amp, int nbits, const int* targets,
                                                   int k, const int* ctrls, int nc, const T* dev_m);
// Every amplitude set to (re, im).  Write-only.
template <typename T> hipError_t launch_init_fill(const Launch& L, void* amp, uint64_t len, double re, double im);
// rho = |psi><psi| in the Eq. 2 layout; psi holds 2^N amplitudes.
template <typename T> hipError_t launch_dm_from_pure(const Launch& L, void* rho, int N, const void* psi);
// dev_out = {Re, Im} of sum_i conj(a_i) b_i (compensated, in double).
template <typename T> hipError_t launch_inner_sv(const Launch& L, const void* a, const void* b, int nbits,
                                                 double* partials, double* dev_out);
// dev_out = {Re, Im} of <psi| rho |psi> (compensated, in double).
template <typename T> hipError_t launch_fid_dm(const Launch& L, const void* rho, int N, const void* psi,
                                               double* partials, double* dev_out);

// --- measure-all ----------------------------------------------------------
// |alpha|^2 of the items j < 2^(nbits - shift) at index fixed + (j << shift),
// summed per bin j mod 2^mbits (mbits <= 10) with compensated sums: dev_out
// receives 2^mbits (sum, compensation) pairs.  `partials` holds
// 2 * 1024 * max_blocks doubles.
constexpr int kHistBlocks = 256;
template <typename T> hipError_t launch_hist_sv(const Launch& L, const void* amp, int nbits, int shift,
                                                uint64_t fixed, int mbits, double* partials, int max_blocks,
                                                double* dev_out);
// Real parts of the 2^N diagonal entries of a density matrix, as doubles.
template <typename T> hipError_t launch_diag_dm(const Launch& L, const void* rho, int N, double* dev_out);

}  // namespace qs
