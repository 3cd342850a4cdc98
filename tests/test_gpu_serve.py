"""Serving loop on the GPU: requests overlapping on the device give the same
results as each request run alone, and those agree with the oracle."""
import numpy as np
import pytest

import oracle as O
from tests.gpu_util import log, max_abs
from workloads import serving_requests

pytestmark = pytest.mark.gpu


@pytest.fixture(scope='module')
def q():
    import paper_1802_08032_amd as q
    return q


def requests(count, rate, seed):
    from paper_1802_08032_amd.serve import Request
    specs = serving_requests(count, rate, seed, sv_range=(10, 16), dm_range=(4, 7), depth_range=(3, 10))
    return [Request(s['rid'], 1 if s['density'] else 0, s['n'], s['ops'], s['arrival'], s['draws'], s['family'])
            for s in specs]


@pytest.mark.parametrize('prec_name,batch', [('C128', True), ('C128', False), ('C64', True)])
def test_each_result_same_alone_and_in_the_mix(q, prec_name, batch):
    """With batching, the state vectors (10..16 qubits) run as batch jobs
    through qs_batch, alone as a batch of one; without, each on its own
    stream through the generic fused kernel."""
    from paper_1802_08032_amd.serve import GpuExecutor, Server
    prec = getattr(q, prec_name)
    env = q.Env(0)
    ex = GpuExecutor(env, prec, slots=6, fusion=12, min_fused=12, keep_amps=True,
                     batch_max_qubits=20 if batch else 0)
    reqs = requests(18, rate=400.0, seed=11)
    log(f'serve mix {prec_name} batch={batch}')
    srv = Server(ex, slots=6)
    mix = srv.serve(reqs)
    assert all(r.error is None for r in mix), [r.error for r in mix if r.error]
    # near-tie band of the measurement draws (8 x the path's error scale:
    # 1e-12 complex128, 1e-5 complex64) and the tolerance of P(outcome)
    band = 8e-12 if prec == q.C128 else 8e-5
    prob_tol = 1e-12 if prec == q.C128 else 1e-4
    near_ties = checked = 0
    for req, r_mix in zip(reqs, mix):
        alone = Server(ex, slots=1).serve([req])[0]
        assert alone.outcomes == r_mix.outcomes
        assert max_abs(alone.amps, r_mix.amps) == 0.0
        # against the oracle, qubit by qubit in measurement order
        if req.kind == 1:
            st = O.run_dm(req.n, req.ops)
            p0_of, measure = O.dm_prob_outcome, O.dm_measure
        else:
            st = O.run_sv(req.n, req.ops)
            p0_of, measure = O.sv_prob_outcome, O.sv_measure
        diverged = False
        for k in range(req.n):
            p0 = p0_of(st, req.n, k, 0)
            o, p = measure(st, req.n, k, req.draws[k])
            if r_mix.outcomes[k] != o:
                # only a draw within the near-tie band of the oracle's p0 may
                # pick the other outcome; later qubits are then measured on
                # another branch and are not comparable
                assert abs(req.draws[k] - p0) < band, (req.rid, k, req.draws[k], p0)
                near_ties += 1
                diverged = True
                break
            assert abs(r_mix.probs[k] - p) <= prob_tol, (req.rid, k, r_mix.probs[k], p)
        checked += 1
        if prec == q.C128 and not diverged:
            # the collapsed state is the measured basis entry scaled by
            # sqrt(g) (state vector) or g (density matrix), g = 1 / P(all
            # outcomes): an amplitude error eps before the collapse is
            # eps * sqrt(g) or eps * g after it
            g = 1.0 / float(np.prod(r_mix.probs))
            bound = 1e-12 * (g if req.kind == 1 else np.sqrt(g))
            assert max_abs(r_mix.amps, st) <= bound, (req.rid, max_abs(r_mix.amps, st), bound)
    log(f'  {checked} requests checked against the oracle, {near_ties} near-tie outcomes')
    assert near_ties <= 2
    s = srv.summary(mix)
    assert s['completed'] == len(reqs)
    env.close()
