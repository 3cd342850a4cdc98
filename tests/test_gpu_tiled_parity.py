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
