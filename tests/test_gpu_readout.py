"""Readouts summed by the last compiled pass (qs_circuit_run_compiled_probs)
and the measurement that takes them (qs_measure_given_probs).

The last pass of a compiled circuit can add up, as it stores the final
state, the total probability and P(qubit q = 0) for every q (Sec. II.B.1's
calcTotalProb and calcProbOfOutcome).  Each is compared with the oracle's
value for the oracle's final state, at a size where every workgroup of the
persistent grid walks several tiles, from a basis state formed inside the
first pass and from a state read from the register, in both precisions; the
stored state must be the oracle's too.  A circuit planned as one pass runs
the form that both forms its tiles and sums the readouts.  The measurement
given those probabilities must leave the same outcome and state as qs_measure
on the same state.
"""
import gc

import numpy as np
import pytest

import oracle as O
from tests.gpu_util import log, max_abs
from workloads import layered_circuit, random_state

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


def oracle_probs(ref, n):
    return np.array([O.sv_total_prob(ref, n)] + [O.sv_prob_outcome(ref, n, k, 0) for k in range(n)])


@pytest.mark.parametrize('prec_name,n,from_basis', [('C128', 22, True), ('C128', 23, False), ('C64', 23, True)])
def test_readout_sums_match_oracle(q, env, prec_name, n, from_basis):
    prec = getattr(q, prec_name)
    K, TB, L = BENCH_TILE if prec == q.C128 else C64_TILE
    ops = layered_circuit(n, 4, 7, mcphase=True)
    log(f'readout parity: n={n} {prec_name} tile=({K},{TB},{L}) from_basis={from_basis}')
    reg = q.Register(env, n, q.STATEVEC, prec)
    if from_basis:
        start = np.zeros(1 << n, dtype=np.complex128)
        start[5] = 1.0
    else:
        start = random_state(n, 21)
        reg.set_amps(start.astype(np.complex128 if prec == q.C128 else np.complex64))
    c = q.Circuit(ops)
    passes, got = c.run_compiled_probs(reg, K, TB, 0, L, init_basis=5 if from_basis else None)
    amps = reg.get_amps()
    # the same state summed by the reduction kernels
    total = reg.calc_total_prob()
    p_top = reg.calc_prob_of_outcome(n - 1, 0)
    c.close()
    reg.close()
    release()
    ref = start.copy()
    for op in ops:
        O.apply_sv(ref, n, op)
    want = oracle_probs(ref, n)
    tol = 1e-12 if prec == q.C128 else 2e-5
    err = np.abs(got - want).max()
    log(f'  {passes} passes, readouts max abs error {err:.2e}, state {max_abs(amps, ref):.2e}')
    assert passes >= 2
    assert err <= tol
    assert max_abs(amps, ref) <= tol
    # both sum the same stored values in double precision
    assert abs(got[0] - total) <= 1e-13
    assert abs(got[n] - p_top) <= 1e-13


def test_one_pass_plan_forms_tiles_and_sums(q, env):
    """A circuit inside one tile: its single pass both forms |j> and sums."""
    n = 16
    K, TB, L = BENCH_TILE
    from workloads.circuits import Op, haar_unitary
    rng = np.random.default_rng(4)
    ops = [Op('u', target=t, u=haar_unitary(rng)) for t in range(K)] + [Op('x', target=1, controls=(0,))]
    reg = q.Register(env, n)
    c = q.Circuit(ops)
    passes, got = c.run_compiled_probs(reg, K, TB, 0, L, init_basis=3)
    amps = reg.get_amps()
    c.close()
    reg.close()
    release()
    ref = O.run_sv(n, ops, init_index=3)
    assert passes == 1
    assert np.abs(got - oracle_probs(ref, n)).max() <= 1e-12
    assert max_abs(amps, ref) <= 1e-12


def test_empty_circuit_readouts(q, env):
    n = 12
    reg = q.Register(env, n)
    psi = random_state(n, 2)
    reg.set_amps(psi)
    c = q.Circuit([])
    passes, got = c.run_compiled_probs(reg, 12, 8, 0, 4)
    c.close()
    reg.close()
    assert passes == 0
    assert np.abs(got - oracle_probs(psi, n)).max() <= 1e-12


def test_measure_given_probs_equals_measure(q, env):
    n = 20
    K, TB, L = BENCH_TILE
    ops = layered_circuit(n, 3, 2, mcphase=True)
    c = q.Circuit(ops)
    draws = (0.13, 0.71, 0.5)
    for k, u in enumerate(draws):
        qubit = (0, n - 1, 7)[k]
        a = q.Register(env, n)
        b = q.Register(env, n)
        _, pr = c.run_compiled_probs(a, K, TB, 0, L, init_basis=0)
        c.run_compiled(b, K, TB, 0, L, init_basis=0)
        p0 = pr[1 + qubit]
        oa, pa = a.measure_given_probs(qubit, p0, pr[0] - p0, u)
        ob, pb = b.measure(qubit, u)
        sa, sb = a.get_amps(), b.get_amps()
        a.close()
        b.close()
        assert oa == ob
        assert abs(pa - pb) <= 1e-13
        assert max_abs(sa, sb) <= 1e-12
    c.close()
    release()


def test_readouts_refuse_density_matrices_and_bad_probabilities(q, env):
    reg = q.Register(env, 5, q.DENSITY)
    c = q.Circuit(layered_circuit(5, 1, 1))
    with pytest.raises(q.QStateError, match='QS_E_KIND'):
        c.run_compiled_probs(reg, 10, 8, 0, 4)
    reg.close()
    sv = q.Register(env, 10)
    sv.init_zero()
    with pytest.raises(q.QStateError, match='QS_E_ARG'):
        sv.measure_given_probs(0, -0.1, 1.1, 0.5)
    with pytest.raises(q.QStateError, match='QS_E_ARG'):
        sv.measure_given_probs(0, float('nan'), 1.0, 0.5)
    sv.close()
    c.close()
