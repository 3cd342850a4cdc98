"""Full-size state vectors: 32 qubits complex128 (64 GiB) and 33 qubits
complex64 (64 GiB), through the run-time compiled passes in the bench's
launch configuration (bench.DEFAULT_TILE),
the generic fused interpreter and the per-gate kernels.  Outputs the oracle can produce one by one are sampled: a product
state (one Haar gate on every target) followed by CNOTs, phases and a few
controlled dense gates; and a random circuit followed by its inverse must
return to |0..0>."""
import gc

import numpy as np
import pytest

import oracle as O
from tests.gpu_util import log
from workloads import Op, haar_unitary, inverse, layered_circuit, product_layer

pytestmark = pytest.mark.gpu

# tile qubits, thread bits and contiguous qubits of the fused passes bench.py times
from bench import DEFAULT_TILE as BENCH_TILE  # noqa: E402


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


def tail_ops(n, seed):
    rng = np.random.default_rng(seed)
    ops = [Op('x', target=q + 1, controls=(q,)) for q in range(0, n - 1, 2)]
    ops.append(Op('phase', qubits=(1, 9, 20, n - 1), angle=1.234))
    # a few dense gates on low, middle and top targets, some controlled
    for t, ctrls in ((0, ()), (3, (n - 2,)), (7, ()), (n - 1, (2, 5)), (17, ()), (31 % n, (0,))):
        ops.append(Op('u', target=t, controls=ctrls, u=haar_unitary(rng)))
    ops.append(Op('x', target=4, controls=(n - 1, 12)))
    return ops


def sample_indices(n, count, seed):
    rng = np.random.default_rng(seed)
    idx = list(rng.integers(0, 1 << n, count, dtype=np.uint64))
    idx += [0, (1 << n) - 1, 1 << (n - 1), (1 << 6) - 1]
    return [int(i) for i in idx]


@pytest.mark.parametrize('n,prec_name,fusion,tol', [(32, 'C128', 13, 1e-12), (33, 'C64', 14, None)])
def test_product_state_and_tail_sampled(q, env, n, prec_name, fusion, tol):
    prec = getattr(q, prec_name)
    prod = product_layer(n, 40 + n)
    tail = tail_ops(n, n)
    vecs = np.array([op.u[:, 0] for op in prod])
    idx = sample_indices(n, 2048, n)
    ref = O.amps_after(n, vecs, tail, idx)
    for mode in ('compiled', fusion, None):
        log(f'large n={n} {prec_name} fusion={mode}')
        reg = q.Register(env, n, q.STATEVEC, prec)
        reg.init_zero()
        c = q.Circuit(prod + tail)
        if mode == 'compiled':  # the run-time compiled passes, in the bench's tile shape
            c.run_compiled(reg, *BENCH_TILE[:2], 0, BENCH_TILE[2])
        else:
            c.run(reg, mode or 0)
        c.close()
        got = np.array([reg.get_amps(i, 1)[0] for i in idx])
        scale = 2.0 ** (-n / 2)
        if tol is not None:
            assert np.max(np.abs(got - ref)) <= tol
        else:  # complex64: relative error of the sampled amplitudes
            assert np.sqrt(np.sum(np.abs(got - ref) ** 2) / np.sum(np.abs(ref) ** 2)) <= 1e-5
        p = reg.calc_total_prob()
        assert abs(p - 1.0) <= (1e-12 if tol else 1e-5)
        reg.close()
        del reg
        release()
        assert scale > 0


@pytest.mark.parametrize('mode', ['compiled', 'fused'])
def test_circuit_then_inverse_returns_to_zero_32q(q, env, mode):
    n = 32
    ops = layered_circuit(n, 2, 9, mcphase=True)
    ops = ops + inverse(ops)
    log(f'large inverse n=32 {mode}')
    reg = q.Register(env, n)
    reg.init_zero()
    c = q.Circuit(ops)
    if mode == 'compiled':
        passes = c.run_compiled(reg, *BENCH_TILE[:2], 0, BENCH_TILE[2])
    else:
        passes = c.run(reg, 13)
    c.close()
    assert passes < len(ops)
    a0 = reg.get_amps(0, 1)[0]
    assert abs(a0 - 1.0) <= 1e-12
    rest = reg.get_amps(1, 4095)
    assert np.max(np.abs(rest)) <= 1e-12
    assert abs(reg.calc_total_prob() - 1.0) <= 1e-12
    assert abs(reg.calc_prob_of_outcome(n - 1, 0) - 1.0) <= 1e-12
    reg.close()
    del reg
    release()


def test_c64_33q_fidelity_against_c128_reference(q, env):
    """The 33-qubit depth-10 circuit in complex64 (64 GiB) against the same
    circuit in complex128 (128 GiB), both through the compiled passes:
    fidelity deficit 1 - |<ref|psi>|^2 (psi not renormalised) <= 1e-5."""
    import torch
    from bench import C64_TILE, fidelity_deficit
    n = 33
    ops = layered_circuit(n, 10, 1, mcphase=True)
    c = q.Circuit(ops)
    log('33q c128 reference')
    ref = q.Register(env, n, q.STATEVEC, q.C128)
    ref.init_zero()
    c.run_compiled(ref, BENCH_TILE[0], BENCH_TILE[1], 0, BENCH_TILE[2])
    assert abs(ref.calc_total_prob() - 1.0) <= 1e-12
    log('33q c64')
    cur = q.Register(env, n, q.STATEVEC, q.C64)
    cur.init_zero()
    c.run_compiled(cur, C64_TILE[0], C64_TILE[1], 0, C64_TILE[2])
    torch.cuda.synchronize()
    deficit = fidelity_deficit(torch, ref.tensor, cur.tensor)
    log(f'33q fidelity deficit {deficit:.3e}')
    assert abs(deficit) <= 1e-5
    assert abs(cur.calc_total_prob() - 1.0) <= 1e-5
    cur.close()
    ref.close()
    c.close()
    del cur, ref
    release()


def test_bench_step_readouts_32q(q, env):
    """The bench step at full size: the bench circuit from |0..0> with the
    readouts summed by its last pass.  The circuit is unitary, so the total
    is 1; each qubit's P(q = 0) must equal what the reduction kernels sum
    from the stored state (an independent path over the same amplitudes);
    P(qubit q = 0) of the inverse-appended circuit is 1 for every q."""
    n = 32
    K, TB, L = BENCH_TILE
    ops = layered_circuit(n, 10, 1, mcphase=True)
    log('large readouts n=32 (bench circuit)')
    reg = q.Register(env, n)
    c = q.Circuit(ops)
    passes, probs = c.run_compiled_probs(reg, K, TB, 0, L, init_basis=0)
    c.close()
    assert passes >= 2
    assert abs(probs[0] - 1.0) <= 1e-12
    for k in (0, 1, 5, 11, 12, 20, 31):
        assert abs(probs[1 + k] - reg.calc_prob_of_outcome(k, 0)) <= 1e-13, k
    assert np.all((probs[1:] >= 0.0) & (probs[1:] <= probs[0] + 1e-12))
    ops2 = layered_circuit(n, 2, 9, mcphase=True)
    c = q.Circuit(ops2 + inverse(ops2))
    _, probs = c.run_compiled_probs(reg, K, TB, 0, L, init_basis=0)
    c.close()
    assert np.max(np.abs(probs - 1.0)) <= 1e-12
    reg.close()
    del reg
    release()
