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


@pytest.mark.parametrize('prec_name', ['C128', 'C64'])
def test_each_result_same_alone_and_in_the_mix(q, prec_name):
    from paper_1802_08032_amd.serve import GpuExecutor, Server
    prec = getattr(q, prec_name)
    env = q.Env(0)
    ex = GpuExecutor(env, prec, slots=6, fusion=12, min_fused=12, keep_amps=True)
    reqs = requests(18, rate=400.0, seed=11)
    log(f'serve mix {prec_name}')
    srv = Server(ex, slots=6)
    mix = srv.serve(reqs)
    assert all(r.error is None for r in mix), [r.error for r in mix if r.error]
    for req, r_mix in zip(reqs, mix):
        alone = Server(ex, slots=1).serve([req])[0]
        assert alone.outcomes == r_mix.outcomes
        assert max_abs(alone.amps, r_mix.amps) == 0.0
        # against the oracle (outcomes exact away from near-ties)
        if req.kind == 1:
            st = O.run_dm(req.n, req.ops)
            ref = [O.dm_measure(st, req.n, k, req.draws[k]) for k in range(req.n)]
        else:
            st = O.run_sv(req.n, req.ops)
            ref = [O.sv_measure(st, req.n, k, req.draws[k]) for k in range(req.n)]
        tol = 1e-12 if prec == q.C128 else 1e-4
        for k, (o, p) in enumerate(ref):
            if prec == q.C128:
                assert r_mix.outcomes[k] == o
            assert abs(r_mix.probs[k] - p) <= tol or r_mix.outcomes[k] != o
        if prec == q.C128:
            assert max_abs(r_mix.amps, st) <= 1e-11
    s = srv.summary(mix)
    assert s['completed'] == len(reqs)
    env.close()
