"""Whole-state oracle parity of the run-time compiled passes at sizes where
every workgroup loops over many tiles.

The compiled pass launches a persistent grid of at most (resident workgroups
per CU) x 256 workgroups, each looping over tiles and prefetching the next
one.  With 2^12-amplitude tiles that loop only runs more than once per
workgroup when the register holds far more than 256 x 2^12 amplitudes, so
the registers here are 2^24..2^27 entries: the bench circuit's shape at 26
qubits (complex128, the bench's tile), the same shape at 27 qubits in
complex64 (the 33-qubit leg's tile), and the noisy 12-qubit density matrix
(a 24-bit vector) through compiled passes.  Each is compared with the
oracle over the whole state.

Also: a compiled plan is keyed by the register kind, so one channel-free
circuit run on a 2N-qubit state vector and then on an N-qubit density matrix
(same index width, different op lists under Eq. 2) gives each its own result.
"""
import gc

import numpy as np
import pytest

import oracle as O
from tests.gpu_util import fidelity_deficit, log, max_abs
from workloads import layered_circuit, noisy_circuit, random_gate_ops

pytestmark = pytest.mark.gpu

from bench import C64_TILE, DEFAULT_TILE as BENCH_TILE  # noqa: E402


@pytest.fixture(scope='module')
def q():
    import paper_1802_08032_amd as q
    return q


@pytest.fixture(scope='module')
def env(q):
    e = q.Env(0)
    yield e
    e.close()


def release():
    import torch
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def tiles_per_workgroup_at_least(nbits, tile_qubits, threads):
    """Lower bound on the tiles each workgroup of the persistent grid walks:
    at most 2048 threads are resident per CU, so the grid has at most
    256 * 2048 / threads workgroups."""
    return (1 << (nbits - tile_qubits)) // (256 * 2048 // threads)


def test_bench_circuit_26q_c128_whole_state(q, env):
    n = 26
    K, TB, L = BENCH_TILE
    assert tiles_per_workgroup_at_least(n, K, 1 << TB) >= 2
    ops = layered_circuit(n, 10, 1, mcphase=True)
    log(f'tiled parity: bench circuit n={n} c128 tile={BENCH_TILE} ({len(ops)} gates)')
    reg = q.Register(env, n)
    reg.init_zero()
    c = q.Circuit(ops)
    passes = c.run_compiled(reg, K, TB, 0, L)
    got = reg.get_amps()
    c.close()
    reg.close()
    release()
    ref = O.run_sv(n, ops)
    err = max_abs(got, ref)
    log(f'  {passes} passes, max abs error {err:.2e}')
    assert passes < len(ops)
    assert err <= 1e-12


def test_bench_circuit_27q_c64_whole_state(q, env):
    n = 27
    K, TB, L = C64_TILE
    assert tiles_per_workgroup_at_least(n, K, 1 << TB) >= 2
    ops = layered_circuit(n, 10, 1, mcphase=True)
    log(f'tiled parity: bench circuit n={n} c64 tile={C64_TILE} ({len(ops)} gates)')
    reg = q.Register(env, n, q.STATEVEC, q.C64)
    reg.init_zero()
    c = q.Circuit(ops)
    passes = c.run_compiled(reg, K, TB, 0, L)
    got = reg.get_amps()
    c.close()
    reg.close()
    release()
    ref = O.run_sv(n, ops)
    deficit = fidelity_deficit(ref, got)
    rel = float(np.sqrt(np.sum(np.abs(got - ref) ** 2) / np.sum(np.abs(ref) ** 2)))
    log(f'  {passes} passes, fidelity deficit {deficit:.2e}, relative l2 error {rel:.2e}')
    assert abs(deficit) <= 1e-5
    assert rel <= 1e-5


def test_noisy_dm_12q_compiled_whole_state(q, env):
    N = 12
    K, TB, L = 12, 8, 4
    assert tiles_per_workgroup_at_least(2 * N, K, 1 << TB) >= 2
    ops = noisy_circuit(N, 10, 2)
    log(f'tiled parity: noisy density matrix N={N} ({len(ops)} ops) through compiled passes')
    reg = q.Register(env, N, q.DENSITY)
    reg.init_zero()
    c = q.Circuit(ops)
    passes = c.run_compiled(reg, K, TB, 0, L)
    got = reg.get_amps()
    trace = reg.calc_total_prob()
    c.close()
    reg.close()
    release()
    ref = O.run_dm(N, ops)
    err = max_abs(got, ref)
    log(f'  {passes} passes, max abs error {err:.2e}')
    assert err <= 1e-12
    assert abs(trace - O.dm_total_prob(ref, N)) <= 1e-12


@pytest.mark.parametrize('first', ['statevec', 'density'])
def test_compiled_plan_is_keyed_by_register_kind(q, env, first):
    N = 5
    ops = layered_circuit(N, 3, 11, mcphase=True) + random_gate_ops(N, 12, 12, max_controls=2)
    c = q.Circuit(ops)
    sv = q.Register(env, 2 * N)
    dm = q.Register(env, N, q.DENSITY)
    order = (sv, dm) if first == 'statevec' else (dm, sv)
    for reg in order:
        reg.init_zero()
        c.run_compiled(reg, 8, 6, 0, 4)
    log(f'plan kind key: {first} first')
    assert max_abs(sv.get_amps(), O.run_sv(2 * N, ops)) <= 1e-12
    assert max_abs(dm.get_amps(), O.run_dm(N, ops)) <= 1e-12
    c.close()
    sv.close()
    dm.close()


@pytest.mark.parametrize('kind_name,prec_name,n,index', [('STATEVEC', 'C128', 14, 0), ('STATEVEC', 'C128', 14, 5),
                                                         ('STATEVEC', 'C128', 20, (1 << 20) - 1),
                                                         ('STATEVEC', 'C64', 16, 9), ('DENSITY', 'C128', 6, 3)])
def test_compiled_run_from_basis_state(q, env, kind_name, prec_name, n, index):
    """qs_circuit_run_compiled_from_basis: the first pass forms |index>
    (|index><index| for a density matrix) instead of reading the register,
    which holds garbage beforehand; the result equals the oracle's run from
    that basis state, and an empty circuit just sets the basis state."""
    kind, prec = getattr(q, kind_name), getattr(q, prec_name)
    if kind == q.DENSITY:
        ops = noisy_circuit(n, 3, 21)
        ref = O.run_dm(n, ops, init_index=index)
        tile = (10, 7, 0, 3)
    else:
        ops = layered_circuit(n, 4, 22, mcphase=True)
        ref = O.run_sv(n, ops, init_index=index)
        tile = (12, 8, 0, 4) if prec == q.C128 else (14, 10, 0, 5)
    reg = q.Register(env, n, kind, prec)
    reg.init_plus()  # overwritten without being read
    c = q.Circuit(ops)
    passes = c.run_compiled(reg, *tile, init_basis=index)
    got = reg.get_amps()
    log(f'from basis {index}: {kind_name} {prec_name} n={n}, {passes} passes')
    if prec == q.C128:
        assert max_abs(got, ref) <= 1e-12
    else:
        assert abs(fidelity_deficit(ref, got)) <= 1e-5
    # the same plan without the folded initialisation
    reg.init_basis(index)
    assert c.run_compiled(reg, *tile) == passes
    assert max_abs(reg.get_amps(), got) <= (1e-14 if prec == q.C128 else 1e-6)
    c.close()
    empty = q.Circuit([])
    reg.init_plus()
    empty.run_compiled(reg, *tile, init_basis=index)
    pos = index + (index << n) if kind == q.DENSITY else index
    amps = reg.get_amps()
    assert amps[pos] == 1.0 and np.count_nonzero(amps) == 1
    with pytest.raises(q.QStateError, match='QS_E_ARG'):
        empty.run_compiled(reg, *tile, init_basis=1 << n)
    empty.close()
    reg.close()


@pytest.mark.parametrize('prec_name', ['C64', 'C128'])
def test_deferred_global_factor_stays_in_range(q, env, prec_name):
    """800 Hadamards on one register (H H = I, so the state returns to
    |0..0>): each runs as a core whose deferred factor has magnitude 1/sqrt 2,
    so without multiplying the global factor in along the way the stored
    complex64 amplitudes would grow by 2^400 and overflow.  Both fused paths
    (compiled and generic) must return |0..0>."""
    from workloads import H, Op
    prec = getattr(q, prec_name)
    n = 14
    ops = [Op('u', target=k % n, u=H) for k in range(2 * n * 28)]
    tol = 1e-12 if prec == q.C128 else 1e-5
    for how in ('compiled', 'generic'):
        reg = q.Register(env, n, q.STATEVEC, prec)
        reg.init_zero()
        c = q.Circuit(ops)
        if how == 'compiled':
            c.run_compiled(reg, 12, 8, 0, 4)
        else:
            c.run(reg, 12)
        amps = reg.get_amps()
        c.close()
        reg.close()
        log(f'{len(ops)} Hadamards, {how} {prec_name}: |amp[0] - 1| = {abs(amps[0] - 1):.2e}')
        assert np.all(np.isfinite(amps))
        assert abs(amps[0] - 1.0) <= tol and np.max(np.abs(amps[1:])) <= tol
