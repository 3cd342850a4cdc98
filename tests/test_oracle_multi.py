"""Pins for the oracle's k-qubit gates, general Kraus maps, initialisations
and overlaps (no GPU).

Sec. II.B.1 states that the pair update of Eq. 1 and the Eq. 2 route for
density matrices hold for multi-qubit gates; decoherence is a Kraus map.
The oracle's k-qubit routines gather groups of 2^k amplitudes; here they are
checked against full 2^n x 2^n operators built a different way (qubits
permuted so that the targets come first, then a Kronecker product, then
permuted back), against products of the already-pinned single-qubit
routines (U_a (x) U_b, SWAP, CNOT as a 4x4), and against the vectorisation
identity vec(K rho K^dagger) = (conj(K) (x) K) vec(rho).
"""
import math

import numpy as np
import pytest

import oracle as O
from tests import brute as B
from workloads import Op, haar_unitary, haar_unitary_k, random_kraus, random_multi_ops, random_state


def permutation(n, order):
    """P with P|i> = |j>, where bit s of j is bit order[s] of i (qubit
    order[s] moves to position s)."""
    dim = 1 << n
    P = np.zeros((dim, dim))
    for i in range(dim):
        j = 0
        for s, q in enumerate(order):
            j |= ((i >> q) & 1) << s
        P[j, i] = 1.0
    return P


def full_operator(n, controls, targets, u):
    """Controlled k-qubit U as a dense matrix: move targets to positions
    0..k-1 and controls to k..k+c-1, build |1..1><1..1| (x) U + (I - proj)
    (x) I there with np.kron, move back."""
    k, c = len(targets), len(controls)
    rest = [q for q in range(n) if q not in targets and q not in controls]
    order = list(targets) + list(controls) + rest
    P = permutation(n, order)
    dk = 1 << k
    proj = np.zeros((1 << c, 1 << c))
    proj[-1, -1] = 1.0
    ctrl_part = np.kron(proj, np.asarray(u)) + np.kron(np.eye(1 << c) - proj, np.eye(dk))
    local = np.kron(np.eye(1 << len(rest)), ctrl_part)
    return P.T @ local @ P


def rand_density(N, seed, rank=3):
    rng = np.random.default_rng(seed)
    dim = 1 << N
    A = rng.standard_normal((dim, rank)) + 1j * rng.standard_normal((dim, rank))
    rho = A @ A.conj().T
    return rho / np.trace(rho).real


def test_full_operator_reproduces_single_qubit_gates():
    # the construction itself, against the Kronecker brute force of Eq. 1
    rng = np.random.default_rng(0)
    u = haar_unitary(rng)
    assert np.max(np.abs(full_operator(5, (1, 3), (4,), u) - B.gate_matrix(5, (1, 3), 4, u))) < 1e-15
    assert np.max(np.abs(full_operator(5, (), (0,), u) - B.gate_matrix(5, (), 0, u))) < 1e-15


@pytest.mark.parametrize('n', [3, 5, 7])
def test_multi_unitary_matches_full_operator(n):
    rng = np.random.default_rng(n)
    for trial in range(10):
        k = int(rng.integers(1, min(3, n) + 1))
        c = int(rng.integers(0, min(2, n - k) + 1))
        qs = [int(v) for v in rng.choice(n, size=k + c, replace=False)]
        u = haar_unitary_k(rng, k)
        psi = random_state(n, 100 * n + trial)
        got = psi.copy()
        O.sv_multi_unitary(got, n, qs[k:], qs[:k], u)
        ref = full_operator(n, qs[k:], qs[:k], u) @ psi
        assert np.max(np.abs(got - ref)) < 1e-14


def test_five_target_unitary():
    n = 6
    rng = np.random.default_rng(11)
    u = haar_unitary_k(rng, 5)
    targets = (4, 0, 5, 2, 1)
    psi = random_state(n, 12)
    got = psi.copy()
    O.sv_multi_unitary(got, n, (3,), targets, u)
    assert np.max(np.abs(got - full_operator(n, (3,), targets, u) @ psi)) < 1e-14


def test_two_qubit_products_swap_and_cnot():
    n = 5
    rng = np.random.default_rng(3)
    ua, ub = haar_unitary(rng), haar_unitary(rng)
    psi = random_state(n, 4)
    # U_a on qubit 3 (matrix bit 0), U_b on qubit 1 (matrix bit 1): kron(ub, ua)
    got = psi.copy()
    O.sv_multi_unitary(got, n, (), (3, 1), np.kron(ub, ua))
    ref = psi.copy()
    O.sv_unitary(ref, n, (), 3, ua)
    O.sv_unitary(ref, n, (), 1, ub)
    assert np.max(np.abs(got - ref)) < 1e-15
    # SWAP exchanges the two qubits' bits of every index
    swap = np.eye(4)[[0, 2, 1, 3]]
    got = psi.copy()
    O.sv_multi_unitary(got, n, (), (0, 4), swap)
    for i in range(1 << n):
        j = (i & ~0b10001) | ((i & 1) << 4) | ((i >> 4) & 1)
        assert got[j] == psi[i]
    # CNOT(control 2, target 0) as a 4x4 on (0, 2) equals the pinned NOT:
    # matrix bit 1 (qubit 2) controls a flip of matrix bit 0 (qubit 0)
    cnot = np.eye(4)[[0, 1, 3, 2]]
    got = psi.copy()
    O.sv_multi_unitary(got, n, (), (0, 2), cnot)
    ref = psi.copy()
    O.sv_x(ref, n, (2,), 0)
    assert np.max(np.abs(got - ref)) == 0.0


def test_multi_unitary_ghz_closed_form():
    # H (x) I then CNOT on qubits (0,1), as one 4x4, then CNOT chain: GHZ
    n = 4
    cnot = np.eye(4)[[0, 3, 2, 1]]  # control = matrix bit 0, target = bit 1
    h_then_cnot = cnot @ np.kron(np.eye(2), np.array([[1, 1], [1, -1]]) / math.sqrt(2))
    psi = O.zero_state(n)
    O.sv_multi_unitary(psi, n, (), (0, 1), h_then_cnot)
    for q in range(1, n - 1):
        O.sv_multi_unitary(psi, n, (), (q, q + 1), cnot)
    want = np.zeros(1 << n, dtype=np.complex128)
    want[0] = want[-1] = 1 / math.sqrt(2)
    assert np.max(np.abs(psi - want)) < 1e-15


@pytest.mark.parametrize('N', [2, 3, 4])
def test_dm_multi_unitary_is_u_rho_udagger(N):
    rng = np.random.default_rng(20 + N)
    for trial in range(6):
        k = int(rng.integers(1, min(2, N) + 1))
        c = int(rng.integers(0, min(1, N - k) + 1))
        qs = [int(v) for v in rng.choice(N, size=k + c, replace=False)]
        u = haar_unitary_k(rng, k)
        rho = rand_density(N, trial)
        vec = B.dm_to_vector(rho)
        O.dm_multi_unitary(vec, N, qs[k:], qs[:k], u)
        G = full_operator(N, qs[k:], qs[:k], u)
        assert np.max(np.abs(O.dm_matrix(vec, N) - G @ rho @ G.conj().T)) < 1e-14


@pytest.mark.parametrize('N', [2, 3, 4])
def test_kraus_multi_matches_full_kraus_sum(N):
    rng = np.random.default_rng(40 + N)
    for trial in range(6):
        k = int(rng.integers(1, min(2, N) + 1))
        ts = [int(v) for v in rng.choice(N, size=k, replace=False)]
        Ks = random_kraus(rng, k, int(rng.integers(1, 5)))
        # completeness of the generated set
        assert np.max(np.abs(sum(K.conj().T @ K for K in Ks) - np.eye(1 << k))) < 1e-14
        rho = rand_density(N, 50 + trial)
        vec = B.dm_to_vector(rho)
        O.dm_kraus_multi(vec, N, ts, Ks)
        full = [full_operator(N, (), ts, K) for K in Ks]
        ref = sum(F @ rho @ F.conj().T for F in full)
        got = O.dm_matrix(vec, N)
        assert np.max(np.abs(got - ref)) < 1e-14
        assert abs(np.trace(got) - 1.0) < 1e-14
        assert np.max(np.abs(got - got.conj().T)) < 1e-15


def test_kraus_multi_vectorisation_identity():
    # vec(K rho K^dagger) = (conj(K) (x) K) vec(rho) on the Eq. 2 vector, with
    # K acting on the row qubits t and conj(K) on the column qubits t + N
    N = 3
    rng = np.random.default_rng(7)
    Ks = random_kraus(rng, 2, 3)
    ts = (2, 0)
    rho = rand_density(N, 8)
    vec = B.dm_to_vector(rho)
    got = vec.copy()
    O.dm_kraus_multi(got, N, ts, Ks)
    ref = sum(full_operator(2 * N, (), (ts[0] + N, ts[1] + N), K.conj()) @ full_operator(2 * N, (), ts, K) @ vec
              for K in Ks)
    assert np.max(np.abs(got - ref)) < 1e-14


def test_kraus_multi_reduces_to_the_named_channels():
    N = 3
    for kind, p in (('dephasing', 0.2), ('depolarising', 0.3), ('damping', 0.45)):
        for t in range(N):
            rho = rand_density(N, 60 + t)
            a = B.dm_to_vector(rho)
            b = a.copy()
            O.dm_kraus_multi(a, N, (t,), B.kraus_ops(kind, p))
            O.apply_dm(b, N, Op(kind, target=t, p=p))
            assert np.max(np.abs(a - b)) < 1e-15
    # a product channel on two qubits = the two single-qubit channels
    Ka, Kb = B.kraus_ops('damping', 0.3), B.kraus_ops('depolarising', 0.2)
    prod = [np.kron(kb, ka) for kb in Kb for ka in Ka]  # ka on targets[0], kb on targets[1]
    rho = rand_density(N, 70)
    a = B.dm_to_vector(rho)
    b = a.copy()
    O.dm_kraus_multi(a, N, (1, 2), prod)
    O.apply_dm(b, N, Op('damping', target=1, p=0.3))
    O.apply_dm(b, N, Op('depolarising', target=2, p=0.2))
    assert np.max(np.abs(a - b)) < 1e-15


def test_random_multi_ops_circuit_against_brute_force():
    n = 6
    ops = random_multi_ops(n, 20, 5, max_targets=3, max_controls=2)
    psi = O.zero_state(n)
    for op in ops:
        O.apply_sv(psi, n, op)
    ref = np.zeros(1 << n, dtype=np.complex128)
    ref[0] = 1
    for op in ops:
        ref = full_operator(n, op.controls, op.targets, op.u) @ ref
    assert np.max(np.abs(psi - ref)) < 1e-14
    assert abs(O.sv_total_prob(psi, n) - 1.0) < 1e-14


def test_init_pure_and_uniform():
    N = 4
    psi = random_state(N, 9)
    rho = O.dm_pure(N, psi)
    assert np.max(np.abs(O.dm_matrix(rho, N) - np.outer(psi, psi.conj()))) < 1e-16
    plus = O.uniform_state(5, 2 ** -2.5)
    assert np.all(plus == 2 ** -2.5)
    # H on every qubit of |0..0> is the uniform state
    h = O.zero_state(5)
    for q in range(5):
        O.sv_unitary(h, 5, (), q, np.array([[1, 1], [1, -1]]) / math.sqrt(2))
    assert np.max(np.abs(h - plus)) < 1e-15


def test_inner_product_purity_fidelity():
    n = 7
    a, b = random_state(n, 1), random_state(n, 2)
    z = O.sv_inner_product(a, b, n)
    assert abs(z - np.vdot(a, b)) < 1e-15
    assert abs(O.sv_inner_product(a, a, n) - 1.0) < 1e-15
    N = 4
    psi = random_state(N, 3)
    pure = O.dm_pure(N, psi)
    assert abs(O.dm_purity(pure, N) - 1.0) < 1e-14
    mixed = B.dm_to_vector(np.eye(1 << N, dtype=np.complex128) / (1 << N))
    assert abs(O.dm_purity(mixed, N) - 2.0 ** -N) < 1e-16
    rho = rand_density(N, 4)
    vec = B.dm_to_vector(rho)
    assert abs(O.dm_purity(vec, N) - np.trace(rho @ rho).real) < 1e-14
    assert abs(O.dm_fidelity_pure(pure, N, psi) - 1.0) < 1e-14
    assert abs(O.dm_fidelity_pure(vec, N, psi) - np.vdot(psi, rho @ psi).real) < 1e-14
