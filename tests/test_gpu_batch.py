"""Batched registers: many independent state vectors of uneven size, each
with its own circuit, run by one persistent launch and replayed from a HIP
graph; every register against the oracle."""
import numpy as np
import pytest

import oracle as O
from tests.gpu_util import fidelity_deficit, log, max_abs
from workloads import Op, param_circuit, random_gate_ops, ry, rz

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


def make_batch(q, env, sizes, prec, depth, seed0, tile):
    regs = [q.Register(env, n, q.STATEVEC, prec) for n in sizes]
    ops = [param_circuit(n, depth, seed0 + i) + random_gate_ops(n, 20, seed0 + 500 + i, max_controls=2)
           for i, n in enumerate(sizes)]
    circs = [q.Circuit(o) for o in ops]
    b = q.Batch(regs, circs, tile)
    return regs, ops, circs, b


def close_all(b, regs, circs):
    b.close()
    for c in circs:
        c.close()
    for r in regs:
        r.close()


@pytest.mark.parametrize('tile', [9, 10, 12])
def test_batch_c128_matches_oracle(q, env, tile):
    rng = np.random.default_rng(tile)
    sizes = [int(v) for v in rng.integers(max(tile, 9), 15, 20)]
    regs, ops, circs, b = make_batch(q, env, sizes, q.C128, 3, 100, tile)
    log(f'batch c128 tile={tile} sizes={sizes}')
    b.run(init_zero=True)
    p0, tot = b.probs(0)
    for i, n in enumerate(sizes):
        ref = O.run_sv(n, ops[i])
        assert max_abs(regs[i].get_amps(), ref) <= 1e-12, (i, n)
        assert abs(p0[i] - O.sv_prob_outcome(ref, n, 0, 0)) <= 1e-12
        assert abs(tot[i] - 1.0) <= 1e-12
    close_all(b, regs, circs)


def test_batch_c64_fidelity(q, env):
    sizes = [9, 10, 11, 12, 13, 14, 15, 16, 10, 12]
    regs, ops, circs, b = make_batch(q, env, sizes, q.C64, 4, 7, 10)
    b.run(init_zero=True)
    for i, n in enumerate(sizes):
        assert fidelity_deficit(O.run_sv(n, ops[i]), regs[i].get_amps()) <= 1e-5, (i, n)
    close_all(b, regs, circs)


def test_graph_replay_matches_eager(q, env):
    """Replays of the captured launch, with eager work in between, give the
    eager result every time."""
    sizes = [9, 11, 13, 10, 12, 14]
    regs, ops, circs, b = make_batch(q, env, sizes, q.C128, 3, 40, 9)
    b.run(init_zero=True)
    eager = [r.get_amps() for r in regs]
    b.capture(init_zero=True)
    for rep in range(3):
        for r in regs:  # eager work on the registers between replays
            r.unitary(0, np.eye(2))
            r.calc_total_prob()
        b.replay()
        for i, r in enumerate(regs):
            assert max_abs(r.get_amps(), eager[i]) == 0.0, (rep, i)
    close_all(b, regs, circs)


def test_batch_rejects_bad_input(q, env):
    r8 = q.Register(env, 8)
    r12 = q.Register(env, 12, q.STATEVEC, q.C64)
    r10 = q.Register(env, 10)
    c = q.Circuit(param_circuit(8, 1, 0))
    c10 = q.Circuit(param_circuit(10, 1, 0))
    with pytest.raises(q.QStateError):      # below 9 qubits
        q.Batch([r8], [c], 9)
    with pytest.raises(q.QStateError):      # mixed precision
        q.Batch([r10, r12], [c10, c10], 9)
    with pytest.raises(q.QStateError):      # circuit wider than the register
        q.Batch([r10], [q.Circuit(param_circuit(12, 1, 0))], 9)
    for x in (c, c10):
        x.close()
    for r in (r8, r12, r10):
        r.close()


@pytest.mark.parametrize('prec_name', ['C128', 'C64'])
def test_c3_workload_512_registers(q, env, prec_name):
    """512 registers of 10..20 qubits (uniform, seed 3), depth-16 RY/RZ + CZ
    ladder circuits (register i: seed 1000 + i).  Registers up to 13 qubits,
    and the first register of each larger size, are compared with the
    oracle amplitude by amplitude and by P(q0 = 0); every register's total
    probability with 1."""
    prec = getattr(q, prec_name)
    rng = np.random.Generator(np.random.PCG64(3))
    sizes = [int(v) for v in rng.integers(10, 21, 512)]
    regs = [q.Register(env, n, q.STATEVEC, prec) for n in sizes]
    ops = [param_circuit(n, 16, 1000 + i) for i, n in enumerate(sizes)]
    circs = [q.Circuit(o) for o in ops]
    log(f'c3 {prec_name}: 512 registers')
    # registers of 10 and 11 qubits are single tiles of their own width
    b = q.Batch(regs, circs, 12)
    b.capture(init_zero=True)
    b.replay()
    p0, tot = b.probs(0)
    tol_tot = 1e-12 if prec == q.C128 else 1e-5
    assert np.max(np.abs(tot - 1.0)) <= tol_tot
    checked = 0
    large_seen = set()
    for i, n in enumerate(sizes):
        if n > 13:
            if n in large_seen:
                continue
            large_seen.add(n)
        ref = O.run_sv(n, ops[i])
        got = regs[i].get_amps()
        if prec == q.C128:
            assert max_abs(got, ref) <= 1e-12, (i, n)
            assert abs(p0[i] - O.sv_prob_outcome(ref, n, 0, 0)) <= 1e-12
        else:
            assert fidelity_deficit(ref, got) <= 1e-5, (i, n)
        checked += 1
    assert checked > 100 and large_seen == set(range(14, 21))
    b.close()
    for c in circs:
        c.close()
    for r in regs:
        r.close()


def test_batch_parameter_update_replays_new_values(q, env):
    """A captured batch replays with new gate parameters after
    qs_batch_update, without being captured again: every register matches
    the oracle run of its circuit with the new values, including matrices
    that become diagonal and diagonal ones that become dense; setters reject
    ops of another kind."""
    import dataclasses
    from workloads import H, haar_unitary, rz
    rng = np.random.default_rng(5)
    sizes = [10, 12, 9, 11, 13, 10]
    # the last register's circuit is empty (the batch runs a placeholder
    # pass for it, which an update must leave alone)
    ops = [param_circuit(n, 3, 300 + i) for i, n in enumerate(sizes[:-1])] + [[]]
    regs = [q.Register(env, n) for n in sizes]
    circs = [q.Circuit(o) for o in ops]
    b = q.Batch(regs, circs, 10)
    b.capture(init_zero=True)
    b.replay()
    for r, n, o in zip(regs, sizes, ops):
        assert max_abs(r.get_amps(), O.run_sv(n, o)) <= 1e-12
    new_ops = []
    for c, o in zip(circs, ops):
        no = list(o)
        for k, op in enumerate(no):
            if op.kind == 'u':
                u = (haar_unitary(rng), np.eye(2), rz(float(rng.uniform(0, 6))), H)[k % 4]
                c.set_unitary(k, u)
                no[k] = dataclasses.replace(op, u=np.asarray(u, dtype=np.complex128))
            elif op.kind == 'phase':
                a = float(rng.uniform(0, 6))
                c.set_phase(k, a)
                no[k] = dataclasses.replace(op, angle=a)
        new_ops.append(no)
    b.update()
    b.replay()
    for r, n, o in zip(regs, sizes, new_ops):
        assert max_abs(r.get_amps(), O.run_sv(n, o)) <= 1e-12
    assert max_abs(regs[-1].get_amps(), O.zero_state(sizes[-1])) == 0.0
    # errors: wrong op kind, index out of range, not unitary
    k_u = next(k for k, op in enumerate(ops[0]) if op.kind == 'u')
    k_p = next(k for k, op in enumerate(ops[0]) if op.kind == 'phase')
    for bad in (lambda: circs[0].set_unitary(k_p, H), lambda: circs[0].set_phase(k_u, 0.1),
                lambda: circs[0].set_unitary(len(ops[0]), H), lambda: circs[0].set_unitary(k_u, 2 * H)):
        with pytest.raises(q.QStateError):
            bad()
    close_all(b, regs, circs)


def test_compiled_circuit_sees_parameter_changes(q, env):
    """Compiled passes are rebuilt after qs_circuit_set_*: the second run
    uses the new matrices (one turned diagonal) and matches the oracle."""
    import dataclasses
    from workloads import haar_unitary, layered_circuit
    rng = np.random.default_rng(6)
    n = 14
    ops = layered_circuit(n, 3, 4, mcphase=True)
    reg = q.Register(env, n)
    c = q.Circuit(ops)
    reg.init_zero()
    c.run_compiled(reg, 12, 8, 0, 4)
    assert max_abs(reg.get_amps(), O.run_sv(n, ops)) <= 1e-12
    no = list(ops)
    for k, op in enumerate(no):
        if op.kind == 'u' and k % 2 == 0:
            u = haar_unitary(rng) if k % 4 == 0 else np.diag([1.0, np.exp(0.4j)])
            c.set_unitary(k, u)
            no[k] = dataclasses.replace(op, u=np.asarray(u, dtype=np.complex128))
        elif op.kind == 'phase':
            c.set_phase(k, 1.3)
            no[k] = dataclasses.replace(op, angle=1.3)
    reg.init_zero()
    c.run_compiled(reg, 12, 8, 0, 4)
    assert max_abs(reg.get_amps(), O.run_sv(n, no)) <= 1e-12
    c.close()
    reg.close()


@pytest.mark.parametrize('prec_name', ['C128', 'C64'])
def test_registers_narrower_than_the_batch_tile(q, env, prec_name):
    """A batch tile wider than some registers: those run as single tiles of
    their own width (own kernel shape, own launches), the rest with the
    batch tile; eager runs, graph replays and parameter updates all match
    the oracle."""
    prec = getattr(q, prec_name)
    sizes = [9, 14, 10, 11, 13, 12, 15, 9, 12]
    regs, ops, circs, b = make_batch(q, env, sizes, prec, 3, 60, 13)
    log(f'batch narrower registers {prec_name}: {b.info()}')
    tol = 1e-12 if prec == q.C128 else 1e-5

    def check(op_lists):
        for i, n in enumerate(sizes):
            ref = O.run_sv(n, op_lists[i])
            got = regs[i].get_amps()
            if prec == q.C128:
                assert max_abs(got, ref) <= tol, (i, n, max_abs(got, ref))
            else:
                assert fidelity_deficit(ref, got) <= tol, (i, n)
    b.run(init_zero=True)
    check(ops)
    b.capture(init_zero=True)
    b.replay()
    check(ops)
    # new angles for every rotation, taken into the captured graph
    rng = np.random.default_rng(5)
    new_ops = []
    for c, o in zip(circs, ops):
        lst = list(o)
        for k, op in enumerate(lst):
            if op.kind == 'u':
                u = ry(float(rng.uniform(0, 6.28))) if abs(op.u[0, 1]) > 0 else rz(float(rng.uniform(0, 6.28)))
                c.set_unitary(k, u)
                lst[k] = Op('u', target=op.target, controls=op.controls, u=u)
        new_ops.append(lst)
    b.update()
    b.replay()
    check(new_ops)
    close_all(b, regs, circs)
