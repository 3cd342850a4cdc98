"""State-vector parity: the HIP path through the C ABI against the oracle,
element by element.  Tolerance: 1e-12 max absolute amplitude error in
complex128; 1e-5 fidelity deficit in complex64; measurement outcomes exact."""
import math

import numpy as np
import pytest

import oracle as O
from tests.gpu_util import fidelity_deficit, log, max_abs, run_gpu
from workloads import (H, Op, haar_unitary, layered_circuit, measurement_draws, param_circuit,
                       random_gate_ops, random_state)

pytestmark = pytest.mark.gpu
TOL128 = 1e-12
TOL64_FID = 1e-5


@pytest.fixture(scope='module')
def q():
    import paper_1802_08032_amd as q
    return q


@pytest.fixture(scope='module')
def env(q):
    e = q.Env(0)
    yield e
    e.close()


def oracle_run(n, ops, state=None, init=0):
    if state is None:
        return O.run_sv(n, ops, init_index=init)
    a = state.copy()
    for op in ops:
        O.apply_sv(a, n, op)
    return a


@pytest.mark.parametrize('seed', [0, 1, 2, 3, 4])
def test_c0_random_circuit_per_gate_and_fused(q, env, seed):
    """16 qubits, depth 20, Haar layers + CNOT bricks: amplitudes and total
    probability, unfused and fused."""
    n, depth = 16, 20
    ops = layered_circuit(n, depth, seed)
    ref = O.run_sv(n, ops)
    for fusion in (None, 13, 11, 9):
        log(f'c0 seed={seed} fusion={fusion}')
        got, reg = run_gpu(q, env, n, ops, fusion=fusion, keep=True)
        assert max_abs(got, ref) <= TOL128, fusion
        assert abs(reg.calc_total_prob() - O.sv_total_prob(ref, n)) <= TOL128
        reg.close()


@pytest.mark.parametrize('n', [6, 9, 13])
def test_every_op_every_target(q, env, n):
    """Each gate kind on each target, with random controls, from a random
    state; compared after every op (several tiles and the low-target path)."""
    rng = np.random.default_rng(n)
    state = random_state(n, 100 + n)
    reg = q.Register(env, n)
    reg.set_amps(state)
    ref = state.copy()
    for t in range(n):
        for kind in ('u', 'x', 'phase'):
            k = int(rng.integers(0, min(3, n - 1) + 1))
            others = [int(v) for v in rng.choice([j for j in range(n) if j != t], size=k, replace=False)]
            if kind == 'u':
                op = Op('u', target=t, controls=tuple(others), u=haar_unitary(rng))
            elif kind == 'x':
                op = Op('x', target=t, controls=tuple(others))
            else:
                op = Op('phase', qubits=tuple(others + [t]), angle=float(rng.uniform(0, 6.28)))
            log(f'n={n} t={t} {kind} ctrls={others}')
            reg.apply(op)
            O.apply_sv(ref, n, op)
            assert max_abs(reg.get_amps(), ref) <= TOL128, (t, kind, others)
    reg.close()


@pytest.mark.parametrize('n', [1, 2, 3, 4, 5])
def test_small_registers(q, env, n):
    ops = random_gate_ops(n, 40, seed=n, max_controls=n - 1)
    state = random_state(n, n)
    log(f'small n={n}')
    assert max_abs(run_gpu(q, env, n, ops, state=state), oracle_run(n, ops, state)) <= TOL128
    assert max_abs(run_gpu(q, env, n, ops, state=state, fusion=13), oracle_run(n, ops, state)) <= TOL128


@pytest.mark.parametrize('fusion', [9, 10, 11, 12, 13])
@pytest.mark.parametrize('n,seed', [(14, 1), (17, 2)])
def test_fused_random_gates(q, env, n, seed, fusion):
    """Mixed dense / NOT / phase gates with up to 4 controls anywhere (inside
    and outside the tile), fused at every tile width."""
    ops = random_gate_ops(n, 300, seed=seed, max_controls=4)
    state = random_state(n, seed)
    log(f'fused n={n} seed={seed} k={fusion}')
    assert max_abs(run_gpu(q, env, n, ops, state=state, fusion=fusion), oracle_run(n, ops, state)) <= TOL128


def test_fused_layered_with_mcphase_and_param(q, env):
    n = 18
    for ops in (layered_circuit(n, 6, 5, mcphase=True), param_circuit(n, 4, 6)):
        ref = O.run_sv(n, ops)
        for fusion in (None, 13, 10):
            log(f'layered/param n={n} fusion={fusion}')
            assert max_abs(run_gpu(q, env, n, ops, fusion=fusion), ref) <= TOL128


def test_ragged_and_empty_circuits(q, env):
    n = 12
    state = random_state(n, 7)
    # empty circuit leaves the state untouched
    got = run_gpu(q, env, n, [], state=state, fusion=13)
    assert max_abs(got, state) == 0.0
    # a single phase (no dense target) and a single gate on the top qubit
    for ops in ([Op('phase', qubits=(3,), angle=0.3)], [Op('u', target=n - 1, u=H)]):
        assert max_abs(run_gpu(q, env, n, ops, state=state, fusion=12), oracle_run(n, ops, state)) <= TOL128


def test_probabilities_and_measurement_bit_exact(q, env):
    n = 12
    ops = layered_circuit(n, 5, 8, mcphase=True)
    ref = O.run_sv(n, ops)
    got, reg = run_gpu(q, env, n, ops, keep=True)
    for qb in range(n):
        for o in (0, 1):
            assert abs(reg.calc_prob_of_outcome(qb, o) - O.sv_prob_outcome(ref, n, qb, o)) <= TOL128
    draws = measurement_draws(11, 0, n)
    for qb in range(n):
        o_gpu, p_gpu = reg.measure(qb, draws[qb])
        o_ref, p_ref = O.sv_measure(ref, n, qb, draws[qb])
        assert o_gpu == o_ref, qb
        assert abs(p_gpu - p_ref) <= TOL128
    assert max_abs(reg.get_amps(), ref) <= TOL128
    assert abs(reg.calc_total_prob() - 1.0) <= TOL128
    reg.close()


@pytest.mark.parametrize('prec,n', [('C128', 4), ('C128', 23), ('C64', 5), ('C64', 23)])
def test_prob_of_outcome_half_and_full_reads(q, env, prec, n):
    """calcProbOfOutcome for every qubit and outcome.  Qubits below the
    128-byte line sum over the whole state; the others read only the
    outcome's half: a register whose half is shorter than one workgroup
    step, and 23 qubits, where the large-step kernel instance runs."""
    log(f'prob of outcome {prec} n={n}')
    state = random_state(n, 40 + n)
    reg = q.Register(env, n, q.STATEVEC, getattr(q, prec))
    reg.set_amps(state)
    # the register holds the state rounded to its precision
    ref = state if prec == 'C128' else state.astype(np.complex64).astype(np.complex128)
    for qb in range(n):
        for o in (0, 1):
            assert abs(reg.calc_prob_of_outcome(qb, o) - O.sv_prob_outcome(ref, n, qb, o)) <= TOL128, (qb, o)
    reg.close()


def test_measure_deterministic_edges(q, env):
    reg = q.Register(env, 4)
    reg.init_basis(0b0101)
    assert reg.measure(0, 0.999999999) == (1, 1.0)
    assert reg.measure(1, 0.999999999)[0] == 0
    reg.close()


@pytest.mark.parametrize('fusion', [None, 14])
def test_complex64_fidelity(q, env, fusion):
    n = 16
    ops = layered_circuit(n, 20, 3, mcphase=True)
    ref = O.run_sv(n, ops)
    got, reg = run_gpu(q, env, n, ops, prec=q.C64, fusion=fusion, keep=True)
    assert fidelity_deficit(ref, got) <= TOL64_FID
    # reductions accumulate in double
    assert abs(reg.calc_total_prob() - float(np.sum(np.abs(got) ** 2))) <= 1e-12
    draws = measurement_draws(5, 1, 4)
    for qb in range(4):
        p0_ref = O.sv_prob_outcome(ref, n, qb, 0)
        o, _ = reg.measure(qb, draws[qb])
        if abs(draws[qb] - p0_ref) > 1e-4:  # outside the complex64 near-tie band
            assert o == O.sv_measure(ref, n, qb, draws[qb])[0]
    reg.close()


def test_error_codes_leave_state_unchanged(q, env):
    n = 5
    state = random_state(n, 1)
    reg = q.Register(env, n)
    reg.set_amps(state)
    bad_u = np.array([[1, 1], [0, 1]], dtype=np.complex128)
    cases = [
        (lambda: reg.unitary(n, H), 'QS_E_ARG'),
        (lambda: reg.unitary(-1, H), 'QS_E_ARG'),
        (lambda: reg.multi_controlled_unitary([1, 1], 0, H), 'QS_E_ARG'),
        (lambda: reg.multi_controlled_unitary([0], 0, H), 'QS_E_ARG'),
        (lambda: reg.multi_controlled_not([7], 0), 'QS_E_ARG'),
        (lambda: reg.unitary(0, bad_u), 'QS_E_NOT_UNITARY'),
        (lambda: reg.mix_dephasing(0, 0.1), 'QS_E_KIND'),
        (lambda: reg.multi_controlled_phase([], 0.1), 'QS_E_ARG'),
        (lambda: reg.calc_prob_of_outcome(0, 2), 'QS_E_ARG'),
        (lambda: reg.measure(0, 1.0), 'QS_E_ARG'),
        (lambda: reg.init_basis(1 << n), 'QS_E_ARG'),
        (lambda: reg.get_amps(30, 3), 'QS_E_ARG'),
    ]
    for fn, name in cases:
        with pytest.raises(q.QStateError) as ei:
            fn()
        assert ei.value.name == name
    c = q.Circuit([Op('u', target=n + 2, u=H)])
    with pytest.raises(q.QStateError):
        c.run(reg, 0)
    c.close()
    assert max_abs(reg.get_amps(), state) == 0.0
    stale = reg.h
    reg.close()
    assert q.lib().qs_reg_destroy(stale) == -5      # double destroy
    assert q.lib().qs_reg_destroy(None) == -5
    assert q.lib().qs_init_zero(stale) == -5


def test_owned_and_wrapped_registers_agree(q, env):
    n = 10
    ops = layered_circuit(n, 4, 2)
    a = run_gpu(q, env, n, ops)
    reg = q.Register(env, n, owned=True)
    reg.init_zero()
    for op in ops:
        reg.apply(op)
    assert max_abs(reg.get_amps(), a) == 0.0
    reg.close()


def test_profiler_counts_launches(q, env):
    n = 12
    env.profile(True)
    env.profile_reset()
    ops = layered_circuit(n, 2, 1)
    run_gpu(q, env, n, ops, fusion=12)
    launches, ms = env.profile_read(q.qstate.K_FUSED)
    env.profile(False)
    assert launches >= 1 and ms > 0.0


def flip_circuit(n: int, seed: int):
    """NOTs controlled by low (thread) qubits on every other qubit, each
    followed by a gate on its target, a gate controlled by its target, a
    4-qubit phase over flipped qubits, and flips left open at the end."""
    rng = np.random.default_rng(seed)
    ops = [Op('u', target=t, u=haar_unitary(rng)) for t in range(n)]
    for t in range(4, n):
        c = int(rng.integers(0, 4))
        ops.append(Op('x', target=t, controls=(c,)))
        ops.append(Op('x', target=t, controls=((c + 1) % 4,)))
        ops.append(Op('u', target=t, u=haar_unitary(rng)))
        ops.append(Op('x', target=t, controls=(c,)))
        if t + 1 < n:
            ops.append(Op('u', target=t + 1, controls=(t,), u=haar_unitary(rng)))
    ops.append(Op('phase', qubits=(4, 5, 6, 7), angle=0.7, controls=(4, 5, 6), target=7))
    for t in range(4, n):
        ops.append(Op('x', target=t, controls=(t % 4, (t + 1) % 4)))
        ops.append(Op('x', target=t, controls=(n - 1 - t % 3,)) if t < n - 3 else Op('x', target=t, controls=(0,)))
    return ops


@pytest.mark.parametrize('prec_name,tile,tb,contig', [('C128', 12, 8, 4), ('C128', 13, 9, 4), ('C128', 11, 8, 6),
                                                      ('C64', 13, 9, 4), ('C64', 14, 10, 5)])
def test_compiled_deferred_flips(q, env, prec_name, tile, tb, contig):
    """Thread- and tile-controlled NOTs kept as per-lane flips: folded into
    later gate matrices, applied before their target is used as a control,
    and folded into the LDS and HBM write addresses."""
    prec = getattr(q, prec_name)
    n = 15
    ops = flip_circuit(n, 11)
    state = random_state(n, 5)
    ref = oracle_run(n, ops, state)
    reg = q.Register(env, n, q.STATEVEC, prec)
    reg.set_amps(state)
    c = q.Circuit(ops)
    log(f'flips {prec_name} tile={tile} tb={tb} contig={contig}')
    c.run_compiled(reg, tile, tb, 0, contig)
    got = reg.get_amps()
    if prec == q.C128:
        assert max_abs(got, ref) <= TOL128
    else:
        assert fidelity_deficit(ref, got) <= TOL64_FID
    c.close()
    reg.close()


@pytest.mark.parametrize('prec_name,tile,tb,contig', [('C128', 13, 10, 6), ('C128', 12, 9, 6), ('C128', 11, 8, 6),
                                                      ('C128', 9, 6, 6), ('C128', 13, 9, 4), ('C128', 12, 8, 3),
                                                      ('C64', 14, 10, 6), ('C64', 13, 9, 4)])
def test_compiled_passes_match_oracle(q, env, prec_name, tile, tb, contig):
    """Run-time specialised pass kernels: random gates with controls inside
    and outside the tile, plus a layered circuit with multi-controlled phases."""
    prec = getattr(q, prec_name)
    n = 16
    ops = random_gate_ops(n, 200, seed=tile + tb, max_controls=4) + layered_circuit(n, 3, 4, mcphase=True)
    state = random_state(n, 3)
    ref = oracle_run(n, ops, state)
    reg = q.Register(env, n, q.STATEVEC, prec)
    reg.set_amps(state)
    c = q.Circuit(ops)
    log(f'compiled {prec_name} tile={tile} tb={tb} contig={contig}')
    passes = c.run_compiled(reg, tile, tb, 0, contig)
    got = reg.get_amps()
    if prec == q.C128:
        assert max_abs(got, ref) <= TOL128
    else:
        assert fidelity_deficit(ref, got) <= TOL64_FID
    # the cached compiled form is reused on a second run
    reg.set_amps(state)
    assert c.run_compiled(reg, tile, tb, 0, contig) == passes
    got2 = reg.get_amps()
    assert max_abs(got2, got) == 0.0
    c.close()
    reg.close()


def oracle_measure_all(state, n, draws):
    """The definition: qubits 0..n-1 measured one after another."""
    ref = state.copy()
    outs, probs = [], []
    for k in range(n):
        o, p = O.sv_measure(ref, n, k, draws[k])
        outs.append(o)
        probs.append(p)
    return ref, outs, probs


@pytest.mark.parametrize('n', [1, 2, 5, 10, 11, 13, 21, 23])
def test_measure_all_matches_sequential_measurement(q, env, n):
    """One histogram stage (n <= 10), two (11..20) and three (21..30)."""
    state = random_state(n, 40 + n)
    draws = measurement_draws(9, n, n)
    ref, outs, probs = oracle_measure_all(state, n, draws)
    reg = q.Register(env, n)
    reg.set_amps(state)
    log(f'measure_all n={n}')
    o, p = reg.measure_all(draws)
    assert o == outs
    assert max(abs(a - b) for a, b in zip(p, probs)) <= TOL128
    assert max_abs(reg.get_amps(), ref) <= TOL128
    reg.close()


def test_measure_all_circuit_basis_and_errors(q, env):
    n = 12
    ops = layered_circuit(n, 6, 3, mcphase=True)
    state = O.run_sv(n, ops)
    draws = measurement_draws(4, 1, n)
    ref, outs, probs = oracle_measure_all(state, n, draws)
    reg = q.Register(env, n)
    reg.set_amps(state)
    # a draw outside [0, 1) is rejected before anything runs
    with pytest.raises(q.QStateError):
        reg.measure_all(np.concatenate([draws[:-1], [1.0]]))
    assert max_abs(reg.get_amps(), state) == 0.0
    o, p = reg.measure_all(draws)
    assert o == outs and max(abs(a - b) for a, b in zip(p, probs)) <= TOL128
    assert max_abs(reg.get_amps(), ref) <= TOL128
    # a basis state measures to its own bits with probability 1
    reg.init_basis(0b101100111001)
    o, p = reg.measure_all(measurement_draws(4, 2, n))
    assert o == [(0b101100111001 >> k) & 1 for k in range(n)]
    assert all(abs(v - 1.0) <= 1e-15 for v in p)
    reg.close()


def test_measure_all_complex64(q, env):
    n = 15
    state = random_state(n, 77)
    draws = measurement_draws(5, 3, n)
    ref, outs, probs = oracle_measure_all(state, n, draws)
    reg = q.Register(env, n, q.STATEVEC, q.C64)
    reg.set_amps(state)
    o, p = reg.measure_all(draws)
    # outcomes agree unless a draw falls within the c64 error of p0
    assert o == outs
    assert max(abs(a - b) for a, b in zip(p, probs)) <= 1e-5
    assert fidelity_deficit(ref, reg.get_amps()) <= TOL64_FID
    reg.close()


COMPILED_SHAPES = [(12, 8, 4), (13, 9, 4), (12, 9, 4), (13, 10, 4), (11, 8, 4), (12, 9, 6), (10, 7, 3), (9, 6, 6),
                   (12, 8, 5), (13, 8, 5)]


@pytest.mark.parametrize('seed', range(8))
def test_compiled_random_sweep(q, env, seed):
    """Tile shapes and circuit families in turn, seeded register sizes, through
    the compiled passes (pass partition with window candidates, merged
    register-only ops, deferred flips), against the oracle."""
    rng = np.random.default_rng(500 + seed)
    K, TB, L = COMPILED_SHAPES[(3 * seed + 1) % len(COMPILED_SHAPES)]
    n = int(rng.integers(max(K, 12), 17))
    fam = seed % 4
    if fam == 0:
        ops = layered_circuit(n, int(rng.integers(3, 9)), seed, mcphase=True)
    elif fam == 1:
        ops = param_circuit(n, int(rng.integers(3, 9)), seed)
    elif fam == 2:
        ops = random_gate_ops(n, 250, seed, max_controls=3)
    else:
        ops = layered_circuit(n, 4, seed) + random_gate_ops(n, 120, seed + 1, max_controls=2) + flip_circuit(n, seed)
    state = random_state(n, 900 + seed)
    ref = oracle_run(n, ops, state)
    reg = q.Register(env, n)
    reg.set_amps(state)
    c = q.Circuit(ops)
    log(f'sweep seed={seed} n={n} tile={K},{TB},{L} family={fam} ops={len(ops)}')
    passes = c.run_compiled(reg, K, TB, 0, L)
    assert 1 <= passes <= len(ops)
    assert max_abs(reg.get_amps(), ref) <= TOL128
    c.close()
    reg.close()


def test_seeded_measurement_takes_the_environment_stream(q):
    """qs_measure_seeded / qs_measure_all_seeded give exactly what
    qs_measure / qs_measure_all give with numpy's Philox draws of the same
    (seed, stream); a rejected call does not advance the stream, and
    reseeding rewinds it."""
    n = 10
    ops = layered_circuit(n, 4, 12, mcphase=True)
    e = q.Env(0)
    e.seed(21, 4)
    draws = measurement_draws(21, 4, 3 + n + 1)

    def fresh():
        r = q.Register(e, n, q.STATEVEC, q.C128)
        r.init_zero()
        c = q.Circuit(ops)
        c.run(r, 0)
        c.close()
        return r

    a, b = fresh(), fresh()
    for k, qb in enumerate((3, 7, 0)):
        assert a.measure_seeded(qb) == b.measure(qb, draws[k])
    with pytest.raises(q.QStateError):
        a.measure_seeded(n)  # no such qubit: rejected, no draw taken
    assert max_abs(a.get_amps(), b.get_amps()) == 0.0
    c, d = fresh(), fresh()
    assert c.measure_all_seeded() == d.measure_all(draws[3:3 + n])
    assert max_abs(c.get_amps(), d.get_amps()) == 0.0
    e.seed(21, 4)
    f, g = fresh(), fresh()
    assert f.measure_seeded(5) == g.measure(5, draws[0])
    for r in (a, b, c, d, f, g):
        r.close()
    e.close()


def test_named_gates_match_the_oracle(q, env):
    """qs_hadamard, qs_cnot, qs_cz, qs_rotate_x/y/z, qs_t_gate and
    qs_sqrt_x/y apply the matrices they name: on a state vector from a random state, and on a density matrix
    (Eq. 2) from a basis state; argument errors pass through."""
    from workloads import ry, rz
    th = 0.7
    c, s = math.cos(th / 2), math.sin(th / 2)
    rx = np.array([[c, -1j * s], [-1j * s, c]])
    SX = np.array([[1 + 1j, 1 - 1j], [1 - 1j, 1 + 1j]]) / 2
    SY = np.array([[1 + 1j, -1 - 1j], [1 + 1j, 1 + 1j]]) / 2
    assert np.allclose(SX @ SX, [[0, 1], [1, 0]]) and np.allclose(SY @ SY, [[0, -1j], [1j, 0]])

    def seq(n):
        return [('hadamard', (3,), Op('u', target=3, u=H)),
                ('cnot', (2, n - 2), Op('x', target=n - 2, controls=(2,))),
                ('cz', (n - 1, 1), Op('phase', qubits=(n - 1, 1), angle=math.pi)),
                ('rotate_x', (0, th), Op('u', target=0, u=rx)),
                ('rotate_y', (n - 3, th), Op('u', target=n - 3, u=ry(th))),
                ('rotate_z', (1, th), Op('u', target=1, u=rz(th))),
                ('t_gate', (4,), Op('phase', qubits=(4,), angle=math.pi / 4)),
                ('sqrt_x', (2,), Op('u', target=2, u=SX)),
                ('sqrt_y', (0,), Op('u', target=0, u=SY)),
                ('hadamard', (n - 1,), Op('u', target=n - 1, u=H))]

    n = 9
    state = random_state(n, 77)
    reg = q.Register(env, n)
    reg.set_amps(state)
    ref = state.copy()
    for name, args, op in seq(n):
        getattr(reg, name)(*args)
        O.apply_sv(ref, n, op)
    assert max_abs(reg.get_amps(), ref) <= TOL128
    for bad in (lambda: reg.cnot(3, 3), lambda: reg.hadamard(n), lambda: reg.cz(2, 2)):
        with pytest.raises(q.QStateError):
            bad()
    assert max_abs(reg.get_amps(), ref) <= TOL128  # rejected calls change nothing
    reg.close()

    N = 5
    rho = q.Register(env, N, q.DENSITY, q.C128)
    rho.init_basis(6)
    ref = O.dm_zero(N, 6)
    for name, args, op in seq(N):
        getattr(rho, name)(*args)
        O.apply_dm(ref, N, op)
    assert max_abs(rho.get_amps(), ref) <= TOL128
    rho.close()


def test_compiled_ragged_and_empty_circuits(q, env):
    """Compiled passes on degenerate circuits: an empty circuit launches no
    pass and leaves the state untouched; a lone phase gate and a lone gate on
    the top qubit match the oracle."""
    n = 14
    state = random_state(n, 9)
    reg = q.Register(env, n)
    reg.set_amps(state)
    c = q.Circuit([])
    assert c.run_compiled(reg, 12, 8, 0, 4) == 0
    assert max_abs(reg.get_amps(), state) == 0.0
    c.close()
    for ops in ([Op('phase', qubits=(3, 13), angle=0.3)], [Op('u', target=n - 1, u=H)]):
        reg.set_amps(state)
        c = q.Circuit(ops)
        assert c.run_compiled(reg, 12, 8, 0, 4) == 1
        assert max_abs(reg.get_amps(), oracle_run(n, ops, state)) <= TOL128
        c.close()
    reg.close()
