"""Pins for the oracle's state-vector routines (no GPU).

The oracle is checked against things other than itself: dense Kronecker
products (tests/brute.py), closed forms (GHZ, QFT of a basis state, H^n|0>),
invariants, and library routines (math.fsum) for its compensated sums.
"""
import math

import numpy as np
import pytest

import oracle as O
from tests import brute as B
from workloads import (Op, haar_unitary, layered_circuit, param_circuit, H, X,
                       product_layer)

TOL = 1e-13


def rand_state(n, seed):
    rng = np.random.default_rng(seed)
    psi = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return np.ascontiguousarray(psi / np.linalg.norm(psi))


@pytest.mark.parametrize('n', [1, 2, 3, 5, 8])
def test_single_qubit_gate_every_target_matches_kron(n):
    rng = np.random.default_rng(n)
    for t in range(n):
        u = haar_unitary(rng)
        psi = rand_state(n, 100 + t)
        ref = B.gate_matrix(n, (), t, u) @ psi
        O.sv_unitary(psi, n, (), t, u)
        assert np.max(np.abs(psi - ref)) < TOL


def test_controlled_and_multicontrolled_match_kron():
    rng = np.random.default_rng(7)
    n = 7
    for trial in range(40):
        k = int(rng.integers(1, 5))
        qs = [int(q) for q in rng.choice(n, size=k + 1, replace=False)]
        ctrls, t = qs[:k], qs[k]
        u = haar_unitary(rng)
        psi = rand_state(n, trial)
        ref = B.gate_matrix(n, ctrls, t, u) @ psi
        O.sv_unitary(psi, n, ctrls, t, u)
        assert np.max(np.abs(psi - ref)) < TOL, (ctrls, t)


def test_x_and_phase_match_kron():
    rng = np.random.default_rng(8)
    n = 6
    for trial in range(20):
        qs = [int(q) for q in rng.choice(n, size=3, replace=False)]
        psi = rand_state(n, trial)
        ref = B.gate_matrix(n, qs[:2], qs[2], B.PX) @ psi
        O.sv_x(psi, n, qs[:2], qs[2])
        assert np.max(np.abs(psi - ref)) < TOL
        phi = float(rng.uniform(0, 2 * np.pi))
        ref = B.phase_matrix(n, qs, phi) @ psi
        O.sv_phase(psi, n, qs, phi)
        assert np.max(np.abs(psi - ref)) < TOL


@pytest.mark.parametrize('n,depth,seed', [(6, 5, 0), (9, 4, 1), (10, 3, 2)])
def test_layered_circuit_matches_kron(n, depth, seed):
    ops = layered_circuit(n, depth, seed, mcphase=True)
    assert np.max(np.abs(O.run_sv(n, ops) - B.run_sv(n, ops))) < 1e-12


def test_param_circuit_matches_kron():
    ops = param_circuit(8, 3, 5)
    assert np.max(np.abs(O.run_sv(8, ops) - B.run_sv(8, ops))) < 1e-12


def test_eq1_pair_index_formula_against_bit_insertion():
    """n_i of Eq. 1 is i with a 0 inserted at bit q; its partner sets bit q.
    Checked through the gate: X on q swaps exactly those pairs."""
    n = 5
    for q in range(n):
        psi = np.arange(1 << n, dtype=np.complex128)
        O.sv_x(psi, n, (), q)
        assert np.array_equal(psi.real.astype(int), np.arange(1 << n) ^ (1 << q))


def test_ghz_closed_form():
    for n in (2, 5, 11):
        ops = [Op('u', target=0, u=H)] + [Op('x', target=q + 1, controls=(q,)) for q in range(n - 1)]
        psi = O.run_sv(n, ops)
        expect = np.zeros(1 << n, dtype=np.complex128)
        expect[0] = expect[-1] = 1 / math.sqrt(2)
        assert np.max(np.abs(psi - expect)) < TOL


def qft_ops(n):
    """Textbook QFT on little-endian qubits: for q = n-1..0, H(q) then a
    controlled phase 2 pi / 2^(q-m+1) from every lower qubit m, then reverse
    the qubit order with swaps (3 CNOTs each)."""
    ops = []
    for q in reversed(range(n)):
        ops.append(Op('u', target=q, u=H))
        for m in reversed(range(q)):
            ops.append(Op('phase', qubits=(m, q), angle=2 * math.pi / 2 ** (q - m + 1)))
    for q in range(n // 2):
        a, b = q, n - 1 - q
        ops += [Op('x', target=b, controls=(a,)), Op('x', target=a, controls=(b,)),
                Op('x', target=b, controls=(a,))]
    return ops


@pytest.mark.parametrize('n,x', [(3, 5), (6, 37), (9, 300)])
def test_qft_of_basis_state_closed_form(n, x):
    psi = O.run_sv(n, qft_ops(n), init_index=x)
    k = np.arange(1 << n)
    expect = np.exp(2j * math.pi * x * k / 2 ** n) / math.sqrt(2 ** n)
    assert np.max(np.abs(psi - expect)) < 1e-12


def test_hadamard_all_uniform():
    n = 12
    psi = O.run_sv(n, [Op('u', target=q, u=H) for q in range(n)])
    assert np.max(np.abs(psi - 2 ** (-n / 2))) < TOL


def test_x_on_basis_is_permutation():
    n = 7
    psi = O.run_sv(n, [Op('x', target=q) for q in (0, 3, 6)], init_index=5)
    assert psi[5 ^ 1 ^ 8 ^ 64] == 1 and np.count_nonzero(psi) == 1


def test_norm_preserved_by_unitaries():
    n = 14
    psi = O.run_sv(n, layered_circuit(n, 3, 11, mcphase=True))
    assert abs(O.sv_total_prob(psi, n) - 1) < 1e-13


def test_prob_outcome_and_expectation_z():
    n = 6
    psi = rand_state(n, 3)
    for q in range(n):
        p0 = O.sv_prob_outcome(psi, n, q, 0)
        p1 = O.sv_prob_outcome(psi, n, q, 1)
        bits = (np.arange(1 << n) >> q) & 1
        assert abs(p0 - np.sum(np.abs(psi[bits == 0]) ** 2)) < 1e-15
        assert abs(p0 + p1 - 1) < 1e-14
        # <Z_q> = 2 P(q=0) - 1, with Z_q materialised by Kronecker product
        zq = B.kron_factors(n, {q: B.PZ})
        assert abs(np.vdot(psi, zq @ psi).real - (2 * p0 - 1)) < 1e-14


def test_measure_collapse_rule():
    n = 5
    psi0 = rand_state(n, 9)
    for q in range(n):
        p0 = O.sv_prob_outcome(psi0, n, q, 0)
        for r, expect in ((0.0, 0), (p0 - 1e-9, 0), (p0 + 1e-9, 1), (0.999999, 1)):
            psi = psi0.copy()
            o, p = O.sv_measure(psi, n, q, r)
            assert o == expect
            bits = (np.arange(1 << n) >> q) & 1
            kept = np.where(bits == o, psi0, 0) / math.sqrt(p)
            assert np.max(np.abs(psi - kept)) < 1e-14
            assert abs(O.sv_prob_outcome(psi, n, q, o) - 1) < 1e-14


def test_measure_deterministic_outcomes():
    n = 3
    psi = O.zero_state(n, 0b101)
    o, p = O.sv_measure(psi.copy(), n, 0, 0.999999999)
    assert o == 1 and abs(p - 1) < 1e-15      # p0 = 0: always 1
    o, p = O.sv_measure(psi.copy(), n, 1, 0.999999999)
    assert o == 0 and abs(p - 1) < 1e-15      # p0 = 1: always 0


def test_measure_frequency_within_5_sigma():
    n = 3
    ops = [Op('u', target=q, u=haar_unitary(np.random.default_rng(q))) for q in range(n)]
    base = O.run_sv(n, ops)
    p0 = O.sv_prob_outcome(base, n, 1, 0)
    rng = np.random.default_rng(123)
    trials = 10000
    zeros = sum(O.sv_measure(base.copy(), n, 1, r)[0] == 0 for r in rng.random(trials))
    sigma = math.sqrt(trials * p0 * (1 - p0))
    assert abs(zeros - trials * p0) < 5 * sigma


def test_neumaier_sum_against_fsum():
    rng = np.random.default_rng(0)
    x = rng.standard_normal(200000) * 10.0 ** rng.integers(-12, 12, 200000)
    assert O.neumaier_sum(x) == pytest.approx(math.fsum(x), rel=1e-15, abs=1e-300)
    assert O.neumaier_sum([1e16, 1.0, -1e16]) == 1.0
    assert O.neumaier_sum([1.0, 1e100, 1.0, -1e100]) == 2.0


def test_amps_after_matches_full_state():
    """The single-output evaluator agrees with the full oracle run."""
    n = 9
    prod = product_layer(n, 3)
    vecs = np.array([op.u[:, 0] for op in prod])
    rest = [Op('x', target=4, controls=(3,)), Op('u', target=2, controls=(7, 8), u=haar_unitary(np.random.default_rng(1))),
            Op('phase', qubits=(0, 5, 6), angle=1.1), Op('u', target=8, u=H), Op('x', target=0, controls=(8,))]
    full = O.run_sv(n, prod + rest)
    idx = np.arange(1 << n)
    assert np.max(np.abs(O.amps_after(n, vecs, rest, idx) - full)) < 1e-14


def test_haar_inputs_are_unitary_and_uniform():
    rng = np.random.default_rng(42)
    us = [haar_unitary(rng) for _ in range(4000)]
    for u in us[:200]:
        assert np.max(np.abs(u @ u.conj().T - np.eye(2))) < 4e-15
    m = np.mean([abs(u[0, 0]) ** 2 for u in us])
    assert abs(m - 0.5) < 0.02
    assert np.array_equal(X @ X, np.eye(2))


def test_oracle_result_independent_of_thread_count():
    """Every amplitude pair is computed by one expression whatever the
    OpenMP split, so one thread and all threads give identical bits (17
    qubits: large enough for the parallel loops)."""
    n = 17
    ops = layered_circuit(n, 2, 5, mcphase=True)
    prev = O.set_threads(1)
    try:
        one = O.run_sv(n, ops)
    finally:
        O.set_threads(prev)
    many = O.run_sv(n, ops)
    assert np.array_equal(one, many)
    assert O.sv_prob_outcome(one, n, 16, 1) == O.sv_prob_outcome(many, n, 16, 1)
