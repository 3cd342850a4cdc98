"""The paper-shaped random circuit (gate set {H, T, CZ, X^1/2, Y^1/2} on the
linear topology, Sec. II.C) through every execution path, against the
oracle: one kernel per gate, the generic fused interpreter and the run-time
compiled passes at the bench tile (at 26 qubits every workgroup loops over
tiles), and complex64 by fidelity deficit."""
import pytest

import oracle as O
from tests.gpu_util import fidelity_deficit, log, max_abs, run_gpu
from workloads import paper_random_circuit

pytestmark = pytest.mark.gpu

from bench import DEFAULT_TILE  # noqa: E402


@pytest.fixture(scope='module')
def q():
    import paper_1802_08032_amd as q
    return q


@pytest.fixture(scope='module')
def env(q):
    e = q.Env(0)
    yield e
    e.close()


def test_paper_circuit_20q_every_path(q, env):
    n = 20
    ops = paper_random_circuit(n, 60, 3)
    ref = O.run_sv(n, ops)
    for fusion in (None, 12):
        got = run_gpu(q, env, n, ops, fusion=fusion)
        log(f'paper circuit n={n} ({len(ops)} gates) fusion={fusion}: {max_abs(got, ref):.2e}')
        assert max_abs(got, ref) <= 1e-12
    K, TB, L = DEFAULT_TILE
    reg = q.Register(env, n)
    reg.init_zero()
    c = q.Circuit(ops)
    passes = c.run_compiled(reg, K, TB, 0, L)
    err = max_abs(reg.get_amps(), ref)
    log(f'  compiled: {passes} passes, {err:.2e}')
    assert err <= 1e-12
    c.close()
    reg.close()
    got64 = run_gpu(q, env, n, ops, prec=q.C64, fusion=12)
    assert abs(fidelity_deficit(ref, got64)) <= 1e-5


def test_paper_circuit_26q_compiled_whole_state(q, env):
    n = 26
    ops = paper_random_circuit(n, 30, 4)
    K, TB, L = DEFAULT_TILE
    reg = q.Register(env, n)
    reg.init_zero()
    c = q.Circuit(ops)
    passes = c.run_compiled(reg, K, TB, 0, L)
    got = reg.get_amps()
    c.close()
    reg.close()
    ref = O.run_sv(n, ops)
    err = max_abs(got, ref)
    log(f'paper circuit n={n} ({len(ops)} gates), compiled: {passes} passes, {err:.2e}')
    assert err <= 1e-12
