"""Pins for the oracle's density-matrix routines (no GPU).

Eq. 2 maps rho to a 2N-qubit vector; the oracle applies G on q then conj(G)
on q+N.  Here that is checked against the plain matrix product G rho G^dagger,
the Kraus channels against full Kraus sums, their single-qubit closed forms,
the vectorisation identity vec(K rho K^dagger) = (conj(K) (x) K) vec(rho),
and the invariants trace = 1, Hermiticity and positivity.
"""
import math

import numpy as np
import pytest

import oracle as O
from tests import brute as B
from workloads import Op, haar_unitary, layered_circuit, noisy_circuit


def rand_density(N, seed, rank=3):
    rng = np.random.default_rng(seed)
    dim = 1 << N
    A = rng.standard_normal((dim, rank)) + 1j * rng.standard_normal((dim, rank))
    rho = A @ A.conj().T
    return rho / np.trace(rho).real


@pytest.mark.parametrize('N', [1, 2, 3, 4])
def test_dm_unitary_is_g_rho_gdagger(N):
    rng = np.random.default_rng(N)
    for trial in range(12):
        k = int(rng.integers(0, N))
        qs = [int(q) for q in rng.choice(N, size=k + 1, replace=False)]
        u = haar_unitary(rng)
        rho = rand_density(N, trial)
        vec = B.dm_to_vector(rho)
        O.dm_unitary(vec, N, qs[:k], qs[k], u)
        G = B.gate_matrix(N, qs[:k], qs[k], u)
        assert np.max(np.abs(O.dm_matrix(vec, N) - G @ rho @ G.conj().T)) < 1e-14


def test_dm_phase_and_x():
    N = 4
    rho = rand_density(N, 5)
    vec = B.dm_to_vector(rho)
    O.dm_phase(vec, N, (0, 2, 3), 0.77)
    O.dm_x(vec, N, (1,), 3)
    G = B.gate_matrix(N, (1,), 3, B.PX) @ B.phase_matrix(N, (0, 2, 3), 0.77)
    assert np.max(np.abs(O.dm_matrix(vec, N) - G @ rho @ G.conj().T)) < 1e-14


@pytest.mark.parametrize('kind,p', [('dephasing', 0.13), ('depolarising', 0.21), ('damping', 0.37),
                                    ('dephasing', 0.5), ('depolarising', 0.75), ('damping', 1.0)])
def test_channels_match_full_kraus_sum(kind, p):
    N = 3
    for t in range(N):
        rho = rand_density(N, 10 + t)
        vec = B.dm_to_vector(rho)
        O.apply_dm(vec, N, Op(kind, target=t, p=p))
        Ks = [B.kron_factors(N, {t: K}) for K in B.kraus_ops(kind, p)]
        ref = sum(K @ rho @ K.conj().T for K in Ks)
        assert np.max(np.abs(O.dm_matrix(vec, N) - ref)) < 1e-14


def test_channels_through_eq2_superoperator():
    """K on qubit t and conj(K) on qubit t+N of the 2N-qubit vector, summed
    over the Kraus operators, is the same map (the Eq. 2 route)."""
    N = 3
    for kind, p in (('dephasing', 0.2), ('depolarising', 0.3), ('damping', 0.4)):
        t = 1
        rho = rand_density(N, 3)
        vec = B.dm_to_vector(rho)
        sup = sum(B.kron_factors(2 * N, {t: K, t + N: K.conj()}) for K in B.kraus_ops(kind, p))
        ref = sup @ vec
        O.apply_dm(vec, N, Op(kind, target=t, p=p))
        assert np.max(np.abs(vec - ref)) < 1e-14


def test_single_qubit_channel_closed_forms():
    rho = rand_density(1, 4, rank=2)
    a, b, c, d = rho[0, 0], rho[0, 1], rho[1, 0], rho[1, 1]
    p = 0.3

    def run(kind, p):
        v = B.dm_to_vector(rho)
        O.apply_dm(v, 1, Op(kind, target=0, p=p))
        return O.dm_matrix(v, 1)

    r = run('dephasing', p)
    assert np.allclose(r, [[a, (1 - 2 * p) * b], [(1 - 2 * p) * c, d]], atol=1e-15)
    r = run('depolarising', p)
    assert np.allclose(r, [[(1 - 2 * p / 3) * a + 2 * p / 3 * d, (1 - 4 * p / 3) * b],
                           [(1 - 4 * p / 3) * c, (1 - 2 * p / 3) * d + 2 * p / 3 * a]], atol=1e-15)
    r = run('damping', p)
    s = math.sqrt(1 - p)
    assert np.allclose(r, [[a + p * d, s * b], [s * c, (1 - p) * d]], atol=1e-15)
    # fully depolarising at p = 3/4 gives I/2; damping at gamma = 1 empties |1>
    assert np.allclose(run('depolarising', 0.75), np.eye(2) / 2, atol=1e-15)
    one = np.array([[0, 0], [0, 1]], dtype=np.complex128)
    v = B.dm_to_vector(one)
    O.apply_dm(v, 1, Op('damping', target=0, p=1.0))
    assert np.allclose(O.dm_matrix(v, 1), [[1, 0], [0, 0]], atol=1e-15)


@pytest.mark.parametrize('N,depth,seed', [(3, 3, 0), (4, 2, 1), (5, 1, 2)])
def test_noisy_circuit_matches_brute_force(N, depth, seed):
    ops = noisy_circuit(N, depth, seed, p_depol=0.05, p_deph=0.04, gamma=0.06)
    got = O.dm_matrix(O.run_dm(N, ops), N)
    ref = B.run_dm(N, ops)
    assert np.max(np.abs(got - ref)) < 1e-13


def test_noisy_invariants_trace_hermitian_psd():
    N = 6
    ops = noisy_circuit(N, 3, 4, p_depol=0.02, p_deph=0.03, gamma=0.05)
    vec = O.run_dm(N, ops)
    rho = O.dm_matrix(vec, N)
    assert abs(O.dm_total_prob(vec, N) - 1) < 1e-13
    assert np.max(np.abs(rho - rho.conj().T)) < 1e-15
    assert np.min(np.linalg.eigvalsh(rho)) > -1e-12
    purity = np.trace(rho @ rho).real
    assert purity < 1 - 1e-3


def test_pure_dm_equals_outer_product_of_sv():
    N = 6
    ops = layered_circuit(N, 4, 9, mcphase=True)
    psi = O.run_sv(N, ops)
    vec = O.run_dm(N, ops)
    assert np.max(np.abs(O.dm_matrix(vec, N) - np.outer(psi, psi.conj()))) < 1e-13
    # Eq. 2 vector of a pure state is psi (x) conj(psi) in the 2N-qubit index
    assert np.max(np.abs(vec - np.kron(psi.conj(), psi))) < 1e-13
    rho = O.dm_matrix(vec, N)
    assert abs(np.trace(rho @ rho).real - 1) < 1e-12


def test_dm_probabilities_and_measure():
    N = 4
    rho = rand_density(N, 8)
    vec = B.dm_to_vector(rho)
    for q in range(N):
        bits = (np.arange(1 << N) >> q) & 1
        p0 = O.dm_prob_outcome(vec, N, q, 0)
        assert abs(p0 - np.sum(np.diag(rho)[bits == 0].real)) < 1e-15
    p0 = O.dm_prob_outcome(vec, N, 2, 0)
    v = vec.copy()
    o, p = O.dm_measure(v, N, 2, p0 + 1e-6)
    assert o == 1 and abs(p - (1 - p0)) < 1e-14
    P = B.kron_factors(N, {2: B.P1})
    assert np.max(np.abs(O.dm_matrix(v, N) - P @ rho @ P / p)) < 1e-14
    assert abs(O.dm_total_prob(v, N) - 1) < 1e-14
