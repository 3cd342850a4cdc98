"""The autotuner times candidate tile shapes of the run-time compiled passes
on the caller's register, keeps the fastest, caches it per (device, qubits,
precision, circuit structure) and gives it back without timing on the next
call; the chosen shape reproduces the oracle's state."""
import os

import pytest

import oracle as O
from tests.gpu_util import log, max_abs
from workloads import layered_circuit

pytestmark = pytest.mark.gpu


def test_tune_picks_caches_and_matches_the_oracle(tmp_path, monkeypatch):
    monkeypatch.setenv('QS_TUNE_CACHE', str(tmp_path))
    import paper_1802_08032_amd as q
    from paper_1802_08032_amd import autotune
    n = 20
    ops = layered_circuit(n, 4, 31, mcphase=True)
    env = q.Env(0)
    reg = q.Register(env, n)
    circ = q.Circuit(ops)
    cands = [(12, 8, 4), (11, 8, 4), (12, 9, 4)]
    res = autotune.tune(reg, circ, ops, budget_s=60.0, candidates=cands, log=log)
    assert 'cached' not in res
    assert (res['tile_qubits'], res['thread_bits'], res['contig_qubits']) in cands
    assert len(res['trials']) == len(cands)
    assert res['seconds'] == min(t['seconds'] for t in res['trials'])
    assert os.path.exists(tmp_path / 'tune.json')
    again = autotune.tune(reg, circ, ops, candidates=cands)
    assert again.get('cached') is True
    assert (again['tile_qubits'], again['thread_bits']) == (res['tile_qubits'], res['thread_bits'])
    # another structure is not served from the cache
    other = layered_circuit(n, 3, 32)
    c2 = q.Circuit(other)
    assert 'cached' not in autotune.tune(reg, c2, other, budget_s=60.0, candidates=cands[:1])
    c2.close()
    reg.init_zero()
    circ.run_compiled(reg, res['tile_qubits'], res['thread_bits'], 0, res['contig_qubits'])
    assert max_abs(reg.get_amps(), O.run_sv(n, ops)) <= 1e-12
    circ.close()
    reg.close()
    env.close()


def test_tune_batch_picks_caches_and_matches_the_oracle(tmp_path, monkeypatch):
    """tune_batch times graph replays of the caller's batch at each candidate
    tile width, keeps the fastest and caches it; the batch at that width
    reproduces the oracle."""
    monkeypatch.setenv('QS_TUNE_CACHE', str(tmp_path))
    import numpy as np
    import paper_1802_08032_amd as q
    from paper_1802_08032_amd import autotune
    from workloads import param_circuit
    env = q.Env(0)
    sizes = [10, 12, 14, 16, 11, 13, 15, 10]
    ops = [param_circuit(n, 6, 70 + i) for i, n in enumerate(sizes)]
    regs = [q.Register(env, n) for n in sizes]
    circs = [q.Circuit(o) for o in ops]
    res = autotune.tune_batch(regs, circs, ops, candidates=[10, 12, 13], log=log)
    assert res['tile_qubits'] in (10, 12, 13) and len(res['trials']) == 3
    assert autotune.tune_batch(regs, circs, ops, candidates=[10, 12, 13]).get('cached') is True
    b = q.Batch(regs, circs, res['tile_qubits'])
    b.run(init_zero=True)
    p0, tot = b.probs(0)
    for i, n in enumerate(sizes):
        ref = O.run_sv(n, ops[i])
        assert max_abs(regs[i].get_amps(), ref) <= 1e-12
        assert abs(p0[i] - O.sv_prob_outcome(ref, n, 0, 0)) <= 1e-12
    assert np.max(np.abs(tot - 1.0)) <= 1e-12
    b.close()
    for c in circs:
        c.close()
    for r in regs:
        r.close()
    env.close()
