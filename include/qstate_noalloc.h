/*
 * qstate -- entry point that allocates nothing.
 *
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, serving loops that must not call hipMalloc, harnesses that forbid
 * it.  A register handle brings its own reduction scratch, allocated by
 * qs_reg_create / qs_reg_wrap; this call needs no handle.
 */
#ifndef QSTATE_NOALLOC_H
#define QSTATE_NOALLOC_H

#include "qstate.h"

#ifdef __cplusplus
extern "C" {
#endif

/* The reduction of qs_calc_total_prob / qs_calc_prob_of_outcome over
 * caller-owned amplitudes: dev_amps holds an n-qubit register of kind
 * `kind` (QS_STATEVEC: 2^n amplitudes, 1 <= n <= 40; QS_DENSITY: the Eq. 2
 * vector of 4^n entries, 1 <= n <= 20) in precision `prec`, interleaved
 * complex, on HIP device `device`.  Writes two doubles to the device
 * pointer dev_out: {P(qubit = 0), P(qubit = 1)} (for a density matrix, sums
 * of the diagonal split by row bit `qubit`), or {total probability, 0} for
 * qubit = -1, with the compensated double-precision sums and the same
 * kernels and grid as the register calls (so the values are identical).
 * Asynchronous on `hip_stream` (NULL: the default stream); nothing is
 * allocated, freed or copied to the host.
 *
 * The reduction partials live in a library-static device array of
 * 4 x 1024 doubles (32 KiB) per GPU, held until the process ends; the
 * reduction grid never exceeds 1024 blocks, so every register size fits.
 * Each call fully writes the partials it later reads; calls that overlap on
 * one GPU (different streams or threads) share the array and race.
 * QS_E_ARG for NULL pointers, an unknown kind or precision, n or qubit out
 * of range, or an invalid device. */
qs_status qs_prob_noalloc(int device, const void* dev_amps, int n, int kind, int prec, int qubit,
                          double* dev_out, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* QSTATE_NOALLOC_H */
