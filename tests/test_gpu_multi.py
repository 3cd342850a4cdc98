"""GPU parity of the k-qubit calls and the state-building / overlap calls
against the oracle.

* qs_multi_qubit_unitary (k = 1..5 targets, 0..2 controls; state vectors and,
  through Eq. 2, density matrices) and qs_mix_multi_kraus (1- and 2-qubit
  Kraus maps applied as superoperators) against the oracle's group gather
  and explicit Kraus sums, element by element at 1e-12 in complex128 and by
  fidelity deficit in complex64.
* qs_init_plus, qs_init_pure_state, qs_clone, qs_calc_inner_product,
  qs_calc_purity, qs_calc_fidelity, qs_save_state / qs_load_state.
* Error paths: bad qubit lists, non-unitary matrices, non-trace-preserving
  Kraus sets, Kraus maps on a state vector; the register is unchanged after
  every rejected call.
"""
import os

import numpy as np
import pytest

import oracle as O
from tests.gpu_util import fidelity_deficit, log, max_abs
from workloads import Op, haar_unitary_k, random_kraus, random_multi_ops, random_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope='module')
def q():
    import paper_1802_08032_amd as q
    return q


@pytest.fixture(scope='module')
def env(q):
    e = q.Env(0)
    yield e
    e.close()


def run_ops(q, env, n, ops, kind, prec, state=None):
    reg = q.Register(env, n, kind, prec)
    if state is None:
        reg.init_zero()
    else:
        reg.set_amps(state)
    for op in ops:
        reg.apply(op)
    amps = reg.get_amps()
    reg.close()
    return amps


@pytest.mark.parametrize('n', [5, 6, 9, 13])
def test_multi_qubit_unitary_every_k(q, env, n):
    """Every group size k = 1..min(5, n) with targets at low and high bits,
    from a random state, against the oracle's group update."""
    rng = np.random.Generator(np.random.PCG64(100 + n))
    psi = random_state(n, 7 + n)
    ops = []
    for k in range(1, min(5, n) + 1):
        for placement in ('low', 'high', 'random'):
            if placement == 'low':
                ts = list(range(k))
            elif placement == 'high':
                ts = list(range(n - k, n))[::-1]
            else:
                ts = [int(v) for v in rng.choice(n, size=k, replace=False)]
            rest = [x for x in range(n) if x not in ts]
            nc = int(rng.integers(0, min(2, len(rest)) + 1))
            cs = [int(v) for v in rng.choice(rest, size=nc, replace=False)] if nc else []
            ops.append(Op('unitary', targets=tuple(ts), controls=tuple(cs), u=haar_unitary_k(rng, k)))
    ref = psi.copy()
    for op in ops:
        O.apply_sv(ref, n, op)
    got = run_ops(q, env, n, ops, q.STATEVEC, q.C128, state=psi)
    log(f'multi-qubit unitaries n={n}: {len(ops)} ops, max abs error {max_abs(got, ref):.2e}')
    assert max_abs(got, ref) <= 1e-12


@pytest.mark.parametrize('n,seed', [(8, 1), (12, 2), (16, 3)])
def test_random_multi_qubit_circuits_sv(q, env, n, seed):
    ops = random_multi_ops(n, 40, seed, max_targets=5, max_controls=2)
    ref = O.run_sv(n, ops)
    got = run_ops(q, env, n, ops, q.STATEVEC, q.C128)
    assert max_abs(got, ref) <= 1e-12
    got64 = run_ops(q, env, n, ops, q.STATEVEC, q.C64)
    assert abs(fidelity_deficit(ref, got64)) <= 1e-5


def test_multi_qubit_unitary_grid_stride_24q(q, env):
    """2^22 groups of 4 (more than the 4096-block grid covers at once, so
    every thread loops), and a 5-qubit group straddling low and high bits."""
    n = 24
    rng = np.random.Generator(np.random.PCG64(24))
    psi = random_state(n, 24)
    ops = [Op('unitary', targets=(0, 23), u=haar_unitary_k(rng, 2)),
           Op('unitary', targets=(1, 5, 12, 17, 22), controls=(3,), u=haar_unitary_k(rng, 5)),
           Op('unitary', targets=(7,), controls=(0, 20), u=haar_unitary_k(rng, 1))]
    ref = psi.copy()
    for op in ops:
        O.apply_sv(ref, n, op)
    got = run_ops(q, env, n, ops, q.STATEVEC, q.C128, state=psi)
    log(f'multi-qubit unitaries n=24: max abs error {max_abs(got, ref):.2e}')
    assert max_abs(got, ref) <= 1e-12


@pytest.mark.parametrize('N,seed', [(1, 4), (3, 5), (5, 6), (7, 7)])
def test_density_multi_unitary_and_kraus(q, env, N, seed):
    """Eq. 2 for k-qubit gates (conj(U) on targets + N) and general Kraus
    maps against the oracle's two literal passes and explicit Kraus sums."""
    ops = random_multi_ops(N, 24, seed, max_targets=min(3, N), max_controls=2, kraus=True)
    ref = O.run_dm(N, ops)
    got = run_ops(q, env, N, ops, q.DENSITY, q.C128)
    log(f'density matrix N={N}: {len(ops)} ops, max abs error {max_abs(got, ref):.2e}')
    assert max_abs(got, ref) <= 1e-12
    got64 = run_ops(q, env, N, ops, q.DENSITY, q.C64)
    assert max_abs(got64, ref) <= 1e-5


def test_kraus_matches_named_channels(q, env):
    """The depolarising and damping channels given as Kraus sets through
    qs_mix_kraus equal the closed-form kernels (and the oracle)."""
    N, p, g = 6, 0.2, 0.3
    rho0 = O.dm_pure(N, random_state(N, 61))
    s = np.sqrt
    X = np.array([[0, 1], [1, 0]], complex)
    Y = np.array([[0, -1j], [1j, 0]])
    Z = np.diag([1.0, -1.0]).astype(complex)
    depol = [s(1 - p) * np.eye(2), s(p / 3) * X, s(p / 3) * Y, s(p / 3) * Z]
    damp = [np.array([[1, 0], [0, s(1 - g)]], complex), np.array([[0, s(g)], [0, 0]], complex)]
    a = q.Register(env, N, q.DENSITY)
    b = q.Register(env, N, q.DENSITY)
    a.set_amps(rho0)
    b.set_amps(rho0)
    a.mix_kraus(2, np.stack(depol))
    a.mix_kraus(4, np.stack(damp))
    b.mix_depolarising(2, p)
    b.mix_damping(4, g)
    ref = rho0.copy()
    O.dm_depolarising(ref, N, 2, p)
    O.dm_damping(ref, N, 4, g)
    assert max_abs(a.get_amps(), ref) <= 1e-12
    assert max_abs(a.get_amps(), b.get_amps()) <= 1e-12
    a.close()
    b.close()


def test_two_qubit_calls_and_kraus_on_12q_density_matrix(q, env):
    """qs_two_qubit_unitary and qs_mix_two_qubit_kraus (16 x 16
    superoperator) on a 24-bit vector: many grid-stride iterations."""
    N = 12
    rng = np.random.Generator(np.random.PCG64(12))
    u = haar_unitary_k(rng, 2)
    ks = random_kraus(rng, 2, 3)
    rho0 = O.dm_pure(N, random_state(N, 12))
    reg = q.Register(env, N, q.DENSITY)
    reg.set_amps(rho0)
    reg.two_qubit_unitary(3, 10, u)
    reg.mix_two_qubit_kraus(11, 0, np.stack(ks))
    ref = rho0.copy()
    O.dm_multi_unitary(ref, N, (), (3, 10), u)
    O.dm_kraus_multi(ref, N, (11, 0), ks)
    err = max_abs(reg.get_amps(), ref)
    log(f'two-qubit unitary + Kraus on N=12: max abs error {err:.2e}')
    assert err <= 1e-12
    assert abs(reg.calc_total_prob() - 1.0) <= 1e-12
    reg.close()


def test_rejected_calls_leave_the_register_unchanged(q, env):
    n = 6
    psi = random_state(n, 3)
    reg = q.Register(env, n)
    reg.set_amps(psi)
    rng = np.random.Generator(np.random.PCG64(3))
    u2 = haar_unitary_k(rng, 2)
    bad = [
        (lambda: reg.multi_qubit_unitary((1, 1), u2), 'QS_E_ARG'),             # duplicate target
        (lambda: reg.multi_qubit_unitary((1, 2), u2, (2,)), 'QS_E_ARG'),       # control is a target
        (lambda: reg.multi_qubit_unitary((1, 6), u2), 'QS_E_ARG'),             # qubit out of range
        (lambda: reg.multi_qubit_unitary((0, 1), 2 * u2), 'QS_E_NOT_UNITARY'),
        (lambda: reg.multi_qubit_unitary(tuple(range(6)), np.eye(64)), 'QS_E_ARG'),  # k = 6
        (lambda: reg.mix_kraus(0, np.stack([np.eye(2)])), 'QS_E_KIND'),        # Kraus map on a state vector
    ]
    for call, code in bad:
        with pytest.raises(q.QStateError, match=code):
            call()
    assert max_abs(reg.get_amps(), psi) == 0.0
    reg.close()
    N = 3
    rho0 = O.dm_pure(N, random_state(N, 4))
    dm = q.Register(env, N, q.DENSITY)
    dm.set_amps(rho0)
    with pytest.raises(q.QStateError, match='QS_E_NOT_CPTP'):
        dm.mix_kraus(1, np.stack([0.9 * np.eye(2)]))
    with pytest.raises(q.QStateError, match='QS_E_ARG'):
        dm.mix_kraus(1, np.stack([np.eye(2)] * 5) / np.sqrt(5))                # more than 4^k operators
    assert max_abs(dm.get_amps(), rho0) == 0.0
    dm.close()


@pytest.mark.parametrize('prec_name', ['C128', 'C64'])
def test_init_plus_and_pure_state(q, env, prec_name):
    prec = getattr(q, prec_name)
    tol = 1e-15 if prec == q.C128 else 1e-7
    for n in (1, 7, 15):
        reg = q.Register(env, n, q.STATEVEC, prec)
        reg.init_plus()
        assert max_abs(reg.get_amps(), O.uniform_state(n, 2.0 ** (-n / 2))) <= tol
        reg.close()
    for N in (1, 4, 9):
        dm = q.Register(env, N, q.DENSITY, prec)
        dm.init_plus()
        assert max_abs(dm.get_amps(), O.uniform_state(2 * N, 2.0 ** -N)) <= tol
        psi = random_state(N, 20 + N)
        sv = q.Register(env, N, q.STATEVEC, prec)
        sv.set_amps(psi)
        dm.init_pure_state(sv)
        ref = O.dm_pure(N, psi if prec == q.C128 else psi.astype(np.complex64).astype(np.complex128))
        err = max_abs(dm.get_amps(), ref)
        assert err <= (1e-15 if prec == q.C128 else 1e-7), err
        # a state vector initialised from the pure state is its copy
        sv2 = q.Register(env, N, q.STATEVEC, prec)
        sv2.init_pure_state(sv)
        assert max_abs(sv2.get_amps(), sv.get_amps()) == 0.0
        sv.close()
        sv2.close()
        dm.close()


@pytest.mark.parametrize('prec_name', ['C128', 'C64'])
def test_overlaps_against_the_oracle(q, env, prec_name):
    prec = getattr(q, prec_name)
    dbl = prec == q.C128
    for n in (3, 11, 20):
        a, b = random_state(n, 30 + n), random_state(n, 40 + n)
        if not dbl:  # the registers hold the float-rounded states
            a = a.astype(np.complex64).astype(np.complex128)
            b = b.astype(np.complex64).astype(np.complex128)
        ra, rb = q.Register(env, n, q.STATEVEC, prec), q.Register(env, n, q.STATEVEC, prec)
        ra.set_amps(a)
        rb.set_amps(b)
        ip = ra.calc_inner_product(rb)
        ref = O.sv_inner_product(a, b, n)
        assert abs(ip - ref) <= 1e-14, (n, ip, ref)
        assert abs(rb.calc_fidelity(ra) - abs(ref) ** 2) <= 1e-14
        assert abs(ra.calc_inner_product(ra) - 1.0) <= (1e-14 if dbl else 1e-6)
        rc = q.Register(env, n, q.STATEVEC, prec)
        rc.clone_from(ra)
        assert max_abs(rc.get_amps(), ra.get_amps()) == 0.0
        for r in (ra, rb, rc):
            r.close()
    for N in (2, 6, 10):
        ops = random_multi_ops(N, 12, 50 + N, max_targets=2, max_controls=1, kraus=True)
        rho = O.run_dm(N, ops)
        psi = random_state(N, 60 + N)
        if not dbl:
            rho = rho.astype(np.complex64).astype(np.complex128)
            psi = psi.astype(np.complex64).astype(np.complex128)
        dm = q.Register(env, N, q.DENSITY, prec)
        dm.set_amps(rho)
        sv = q.Register(env, N, q.STATEVEC, prec)
        sv.set_amps(psi)
        pur, pur_ref = dm.calc_purity(), O.dm_purity(rho, N)
        fid, fid_ref = dm.calc_fidelity(sv), O.dm_fidelity_pure(rho, N, psi)
        log(f'N={N} {prec_name}: purity {pur:.15f} (oracle {pur_ref:.15f}), fidelity {fid:.3e}')
        assert abs(pur - pur_ref) <= 1e-14
        assert abs(fid - fid_ref) <= 1e-14
        dm.close()
        sv.close()


@pytest.mark.parametrize('kind_name,prec_name,n', [('STATEVEC', 'C128', 23), ('STATEVEC', 'C64', 24),
                                                   ('DENSITY', 'C128', 12), ('DENSITY', 'C64', 5)])
def test_checkpoint_round_trip(q, env, tmp_path, kind_name, prec_name, n):
    """qs_save_state / qs_load_state restore the state bit for bit (states
    above 64 MiB take several staging chunks); a checkpoint of another shape
    or a truncated file is rejected before anything is written."""
    kind, prec = getattr(q, kind_name), getattr(q, prec_name)
    reg = q.Register(env, n, kind, prec)
    reg.init_plus()
    reg.apply(Op('u', target=1, u=haar_unitary_k(np.random.Generator(np.random.PCG64(1)), 1)))
    before = reg.get_amps()
    path = str(tmp_path / 'state.qs')
    reg.save_state(path)
    assert os.path.getsize(path) == 64 + q.reg_bytes(n, kind, prec)
    reg.init_zero()
    reg.load_state(path)
    assert np.array_equal(reg.get_amps(), before)
    other = q.Register(env, n - 1, kind, prec)
    other.init_zero()
    with pytest.raises(q.QStateError, match='QS_E_ARG'):
        other.load_state(path)
    assert other.get_amps()[0] == 1.0
    other.close()
    with open(path, 'r+b') as f:
        f.truncate(64 + 100)
    reg.init_zero()
    with pytest.raises(q.QStateError, match='QS_E_ARG'):
        reg.load_state(path)
    assert reg.get_amps()[0] == 1.0
    reg.close()


@pytest.mark.parametrize('kind_name,n', [('STATEVEC', 15), ('DENSITY', 7)])
def test_two_qubit_unitaries_in_circuits_every_path(q, env, kind_name, n):
    """Recorded two-qubit unitaries mixed with one-qubit and controlled
    gates, run one kernel per op, through the generic fused kernel and
    through the run-time compiled passes (on ρ's 2N-qubit vector for a
    density matrix), each against the oracle at 1e-12."""
    from workloads import layered_circuit
    kind = getattr(q, kind_name)
    ops = (random_multi_ops(n, 24, 11, max_targets=2, max_controls=0) + layered_circuit(n, 2, 12)
           + random_multi_ops(n, 12, 13, max_targets=1, max_controls=2))
    if kind == q.DENSITY:
        ref = O.run_dm(n, ops)
    else:
        ref = O.run_sv(n, ops)
    c = q.Circuit(ops)
    runs = {'per-op': lambda r: c.run(r, 0), 'fused': lambda r: c.run(r, 12)}
    if kind == q.STATEVEC:
        runs['tiled'] = lambda r: c.run_tiled(r, 12, 8)
        runs['compiled'] = lambda r: c.run_compiled(r, 12, 8, 0, 4)
    for name, fn in runs.items():
        log(f'two-qubit circuit {kind_name} n={n} {name}')
        reg = q.Register(env, n, kind, q.C128)
        reg.init_zero()
        fn(reg)
        err = max_abs(reg.get_amps(), ref)
        reg.close()
        assert err <= 1e-12, (name, err)
    c.close()
    # a 4x4 that is not unitary is rejected when recorded
    bad = Op('unitary', targets=(0, 1), u=2.0 * np.eye(4))
    with pytest.raises(q.QStateError):
        q.Circuit([bad])
