"""The run-time compiled passes, executed on the CPU (tests/pass_emu.py),
against the oracle.

Every generated pass set of a circuit is compiled for the host and applied
to a seeded random state in order: the register renames, unit-diagonal
cores, deferred diagonal factors (within a pass and handed from pass to
pass), pending flips, LDS re-layouts and HBM addressing of the generated
code all take part.  The result must equal the oracle's Eq. 1 updates to
the tolerance of the precision.  The workgroup count is varied, so tiles
also run through the persistent loop with its prefetch."""
import numpy as np
import pytest

import oracle as O
from tests import pass_emu
from workloads import layered_circuit, noisy_circuit, paper_random_circuit, random_gate_ops, random_state

pytestmark = pytest.mark.skipif(not pass_emu.available(), reason='host clang++ not found')


def _run_sv(ops, n, prec, shape, grid_div=4, seed=5):
    import paper_1802_08032_amd as q
    K, TB, L = shape
    psi = random_state(n, seed)
    ref = psi.astype(np.complex128).copy()
    for op in ops:
        O.apply_sv(ref, n, op)
    amp = psi.astype(np.complex128 if prec == q.C128 else np.complex64).copy()
    c = q.Circuit(ops)
    npass = pass_emu.run_passes(c, amp, n, prec, K, TB, L, q.STATEVEC, grid_div=grid_div)
    c.close()
    return np.abs(amp.astype(np.complex128) - ref).max(), npass


@pytest.mark.parametrize('shape,grid_div', [((12, 8, 4), 16), ((11, 8, 4), 1), ((12, 9, 4), 4)])
def test_layered_circuit_with_multi_controlled_phase(shape, grid_div):
    """Haar layers, CNOT bricks and a 4-qubit controlled phase per layer on
    18 qubits: several passes, 4x4 cores with pair factors, factors carried
    between passes."""
    import paper_1802_08032_amd as q
    err, npass = _run_sv(layered_circuit(18, 4, 31, mcphase=True), 18, q.C128, shape, grid_div)
    assert npass >= 2
    assert err <= 1e-12


def test_layered_circuit_complex64():
    import paper_1802_08032_amd as q
    err, npass = _run_sv(layered_circuit(17, 5, 3, mcphase=True), 17, q.C64, (12, 8, 4), 4)
    assert npass >= 2
    assert err <= 2e-5


def test_random_controlled_gates():
    """Dense gates, NOTs and phases with up to three controls on random
    qubits: controls on register, thread and tile-index bits, flips pending
    on register bits, full-matrix fallbacks keeping deferred factors."""
    import paper_1802_08032_amd as q
    for seed in (1, 2, 3):
        err, _ = _run_sv(random_gate_ops(16, 120, seed, max_controls=3), 16, q.C128, (12, 8, 4), 4, seed=seed)
        assert err <= 1e-12, seed


def test_paper_random_circuit():
    """The paper's gate set (H, T, CZ, X^1/2, Y^1/2): deferred one-qubit
    phases and controlled phases between all kinds of bits."""
    import paper_1802_08032_amd as q
    err, npass = _run_sv(paper_random_circuit(16, 24, 7), 16, q.C128, (12, 8, 4), 2)
    assert npass >= 2
    assert err <= 1e-12


def test_density_matrix_passes():
    """A noisy layered circuit on an 8-qubit density matrix: the 16-qubit
    vector of Eq. 2 with the conjugate gates and 4x4 channel
    superoperators (non-unitary unit-diagonal cores)."""
    import paper_1802_08032_amd as q
    N = 8
    ops = noisy_circuit(N, 2, 1)
    psi = random_state(N, 9)
    rho0 = O.dm_pure(N, psi)
    ref = rho0.copy()
    for op in ops:
        O.apply_dm(ref, N, op)
    amp = rho0.astype(np.complex128).copy()
    c = q.Circuit(ops)
    npass = pass_emu.run_passes(c, amp, 2 * N, q.C128, 12, 8, 4, q.DENSITY, grid_div=2)
    c.close()
    assert npass >= 1
    assert np.abs(amp - ref).max() <= 1e-12


def test_two_qubit_unitaries_in_circuits():
    """Recorded two-qubit unitaries (4x4 ops of the pass holding both
    targets, unit-diagonal 4x4 cores) mixed with one-qubit gates, on a state
    vector and on a density matrix (conj(U) on the column qubits)."""
    import paper_1802_08032_amd as q
    from workloads import random_multi_ops
    n = 16
    ops = (random_multi_ops(n, 40, 3, max_targets=2, max_controls=0) + layered_circuit(n, 2, 4)
           + random_multi_ops(n, 20, 5, max_targets=1, max_controls=2))
    err, npass = _run_sv(ops, n, q.C128, (12, 8, 4), 4)
    assert npass >= 2
    assert err <= 1e-12
    N = 7
    dops = random_multi_ops(N, 16, 6, max_targets=2, max_controls=0) + noisy_circuit(N, 1, 2)
    rho0 = O.dm_pure(N, random_state(N, 4))
    ref = rho0.copy()
    for op in dops:
        O.apply_dm(ref, N, op)
    amp = rho0.astype(np.complex128).copy()
    c = q.Circuit(dops)
    pass_emu.run_passes(c, amp, 2 * N, q.C128, 12, 8, 4, q.DENSITY, grid_div=2)
    c.close()
    assert np.abs(amp - ref).max() <= 1e-12


@pytest.mark.parametrize('prec_name,shape,n,grid_div', [('C128', (12, 8, 4), 17, 4), ('C64', (12, 8, 4), 17, 2),
                                                        ('C128', (11, 8, 4), 15, 1)])
def test_readout_sums_of_the_last_pass(prec_name, shape, n, grid_div):
    """The last pass in its readout form: each workgroup's sums of
    |alpha|^2 in total and over bit q = 0 for every qubit (register bits
    with pending flips, thread bits, tile-index bits), added over the
    workgroups, against the oracle's total probability and outcome
    probabilities of its final state (Sec. II.B.1); the stored state is
    unchanged by the readout."""
    import paper_1802_08032_amd as q
    prec = getattr(q, prec_name)
    K, TB, L = shape
    from workloads.circuits import Op
    ops = layered_circuit(n, 3, 11, mcphase=True) + random_gate_ops(n, 40, 5, max_controls=2)
    # NOTs conditioned on tile-index qubits: flips still pending at the store
    ops += [Op('x', target=t, controls=(n - 1,)) for t in range(4, 9)] + [Op('x', target=2, controls=(n - 2, 1))]
    psi = random_state(n, 3)
    ref = psi.astype(np.complex128).copy()
    for op in ops:
        O.apply_sv(ref, n, op)
    amp = psi.astype(np.complex128 if prec == q.C128 else np.complex64).copy()
    c = q.Circuit(ops)
    if (prec_name, n) == ('C64', 17):
        assert '? t - s0 : s0' in c.source(n, prec, K, TB, -1, 0, L)[0]
    npass, part = pass_emu.run_passes(c, amp, n, prec, K, TB, L, q.STATEVEC, grid_div=grid_div, readout=True)
    c.close()
    assert npass >= 2
    assert not np.isnan(part).any()
    got = part.sum(axis=0)
    want = np.array([O.sv_total_prob(ref, n)] + [O.sv_prob_outcome(ref, n, k, 0) for k in range(n)])
    tol = 1e-12 if prec == q.C128 else 2e-5
    assert np.abs(got - want).max() <= tol
    assert np.abs(amp.astype(np.complex128) - ref).max() <= tol
