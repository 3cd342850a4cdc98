"""Scheduler logic of the serving loop on the CPU: an executor backed by the
oracle stands in for the GPU (this is not a second product path).  Checks
admission by bytes against the budget, arrival-order admission, the slot
limit, completion of every request and the measured outcomes."""
import threading
import time

import numpy as np
import pytest

import oracle as O
from workloads import serving_requests


class OracleExecutor:
    def __init__(self, delay=0.01):
        self.delay = delay
        self.lock = threading.Lock()
        self.in_use = 0
        self.peak = 0
        self.running = 0
        self.peak_running = 0
        self.order = []

    def nbytes(self, req):
        return 16 << (2 * req.n if req.kind == 1 else req.n)

    def run(self, req, slot):
        b = self.nbytes(req)
        with self.lock:
            self.in_use += b
            self.peak = max(self.peak, self.in_use)
            self.running += 1
            self.peak_running = max(self.peak_running, self.running)
            self.order.append(req.rid)
        try:
            time.sleep(self.delay)
            if req.kind == 1:
                st = O.run_dm(req.n, req.ops)
                res = [O.dm_measure(st, req.n, q, req.draws[q]) for q in range(req.n)]
            else:
                st = O.run_sv(req.n, req.ops)
                res = [O.sv_measure(st, req.n, q, req.draws[q]) for q in range(req.n)]
            return [o for o, _ in res], [p for _, p in res], None
        finally:
            with self.lock:
                self.in_use -= b
                self.running -= 1


def make_requests(count, rate, seed=3):
    from paper_1802_08032_amd.serve import Request
    specs = serving_requests(count, rate, seed, sv_range=(3, 9), dm_range=(2, 4), depth_range=(1, 4))
    return [Request(s['rid'], 1 if s['density'] else 0, s['n'], s['ops'], s['arrival'], s['draws'], s['family'])
            for s in specs]


def test_budget_slots_and_order():
    from paper_1802_08032_amd.serve import Server
    reqs = make_requests(40, rate=0.0)
    ex = OracleExecutor()
    budget = 16 << 9  # room for about two of the larger requests
    srv = Server(ex, budget_bytes=budget, slots=3)
    res = srv.serve(reqs)
    assert len(res) == 40 and all(r.error is None for r in res)
    assert ex.peak <= budget
    assert ex.peak_running <= 3
    assert ex.order == sorted(ex.order)  # admitted in arrival order
    s = srv.summary(res)
    assert s['completed'] == 40 and s['hbm_peak_bytes'] <= budget
    assert 0 < s['hbm_occupancy_mean'] <= 1


def test_outcomes_match_direct_oracle_runs():
    from paper_1802_08032_amd.serve import Server
    reqs = make_requests(12, rate=200.0)
    res = Server(OracleExecutor(0.0), slots=4).serve(reqs)
    for r, q in zip(res, reqs):
        st = O.run_dm(q.n, q.ops) if q.kind == 1 else O.run_sv(q.n, q.ops)
        for k in range(q.n):
            o, p = (O.dm_measure if q.kind == 1 else O.sv_measure)(st, q.n, k, q.draws[k])
            assert r.outcomes[k] == o and r.probs[k] == pytest.approx(p, abs=1e-15)
        assert r.latency >= 0 and r.finished >= r.admitted >= r.arrival - 1e-9


def test_oversized_request_is_rejected_not_hung():
    from paper_1802_08032_amd.serve import Request, Server
    reqs = make_requests(3, rate=0.0)
    big = Request(99, 0, 9, reqs[0].ops, 0.0, np.zeros(9))
    res = Server(OracleExecutor(0.0), budget_bytes=16 << 8, slots=2).serve(reqs + [big])
    errs = [r for r in res if r.error]
    assert any(r.rid == 99 for r in errs)


class BatchingOracleExecutor(OracleExecutor):
    """Also takes batch jobs: state vectors of 5..8 qubits."""

    def __init__(self, delay=0.01):
        super().__init__(delay)
        self.jobs = []

    def batchable(self, req):
        return req.kind == 0 and 5 <= req.n <= 8

    def run_batch(self, reqs, slot):
        assert all(self.batchable(r) for r in reqs)
        with self.lock:
            self.jobs.append([r.rid for r in reqs])
        return [self.run(r, slot) for r in reqs]


def test_small_state_vectors_run_as_batch_jobs():
    """Pending batchable requests are admitted together as one job per slot
    (up to batch_max, within the byte budget) once batch_min of them wait;
    the others run one by one; every request's outcomes are its own."""
    from paper_1802_08032_amd.serve import Server
    reqs = make_requests(40, rate=0.0, seed=5)
    ex = BatchingOracleExecutor(0.0)
    srv = Server(ex, slots=3, batch_min=2, batch_max=6)
    res = srv.serve(reqs)
    assert len(res) == 40 and all(r.error is None for r in res)
    small = {r.rid for r in reqs if ex.batchable(r)}
    assert small and any(len(j) > 1 for j in ex.jobs)
    assert all(2 <= len(j) <= 6 for j in ex.jobs)
    batched = sorted(rid for j in ex.jobs for rid in j)
    assert len(set(batched)) == len(batched) and set(batched) <= small
    for j in ex.jobs:
        assert j == sorted(j)  # a job takes its requests in arrival order
    for r, q in zip(res, reqs):
        st = O.run_dm(q.n, q.ops) if q.kind == 1 else O.run_sv(q.n, q.ops)
        for k in range(q.n):
            o, p = (O.dm_measure if q.kind == 1 else O.sv_measure)(st, q.n, k, q.draws[k])
            assert r.outcomes[k] == o and r.probs[k] == pytest.approx(p, abs=1e-15)
    # the byte budget holds with batch jobs too
    ex2 = BatchingOracleExecutor(0.0)
    budget = 16 << 9
    srv2 = Server(ex2, budget_bytes=budget, slots=3, batch_min=2, batch_max=64)
    res2 = srv2.serve(reqs)
    assert all(r.error is None for r in res2)
    assert srv2.summary(res2)['hbm_peak_bytes'] <= budget
    assert ex2.jobs and sum(ex2.nbytes(reqs[rid]) for rid in max(ex2.jobs, key=len)) <= budget
    # one request at a time (no queue): nothing is batched
    ex3 = BatchingOracleExecutor(0.0)
    res3 = Server(ex3, slots=3, batch_min=2).serve(make_requests(6, rate=5.0, seed=5))
    assert all(r.error is None for r in res3) and not ex3.jobs
