"""Continuous-batching request loop for circuits on one GPU.

Requests (state-vector or density-matrix circuits, each ending with the
measurement of every qubit under its own draws) arrive over time.  The loop
admits them in arrival order as soon as a slot and enough HBM are free:
admission counts the register's bytes (16 * 2^n, or 16 * 4^n for a density
matrix, halved in complex64) against a budget.  Every admitted request runs
on its own HIP stream in a worker thread, so requests that arrive while
others are on the GPU start right away and their kernels overlap on the
device.  With batching on (GpuExecutor batch_max_qubits > 0), small
state-vector requests are admitted together when a queue has formed: with
at least `batch_min` of them pending, every pending one (up to `batch_max`)
joins one batch job, which runs all their circuits through one qs_batch
launch per pass level and tile shape on one slot.  Below that each runs
alone, as a batch of one, so that its rounding is the same either way.
Batching raises throughput under a backlog (fewer launches, one plan
upload per job) and costs latency at light load (a job finishes with its
slowest member, and a batch of one carries the batch set-up), so it is off
by default.  Per request the loop records arrival, admission and completion
times; `summary` gives p50 / p99 latency, circuits/s and the time-averaged
HBM occupancy.

The scheduling logic is independent of the executor, which only needs
`nbytes(request)` and `run(request, slot)`; one that also has
`batchable(request)` and `run_batch(requests, slot)` gets batch jobs.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import time
from dataclasses import dataclass, field

import numpy as np

from . import qstate as Q


@dataclass
class Request:
    rid: int
    kind: int            # qstate.STATEVEC or qstate.DENSITY
    n: int               # qubits
    ops: list            # workloads.Op list
    arrival: float       # seconds after the start of serving
    draws: np.ndarray    # one uniform draw per qubit for the final measurements
    family: str = ''


@dataclass
class Result:
    rid: int
    outcomes: list
    probs: list
    arrival: float
    admitted: float
    finished: float
    nbytes: int
    amps: np.ndarray | None = None
    error: str | None = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


# thread bits of the generic fused kernel's tile for each tile width
# (complex128 takes 9 at 13 qubits: 16 registers per thread, not 32)
_TB_OF = {9: 6, 10: 7, 11: 8, 12: 8, 13: 8, 14: 9}


class GpuExecutor:
    """Runs one request: register on the slot's stream, |0..0>, the circuit
    (state vectors of 9..batch_max_qubits qubits through qs_batch; other
    state vectors of at least `min_fused` qubits fused through the generic
    pass kernel; density matrices whose 2N-qubit vector holds a tile of at
    least 9 qubits through the generic kernel's tiles; one kernel per op
    otherwise), then measures qubits 0..n-1 in order (one measure-all call:
    a histogram walk and a single collapse)."""

    def __init__(self, env: Q.Env, prec: int = Q.C128, slots: int = 8, fusion: int = 12,
                 min_fused: int = 12, keep_amps: bool = False, batch_max_qubits: int = 0,
                 batch_tile: int = 12):
        import torch
        self.torch = torch
        self.env, self.prec, self.fusion, self.min_fused = env, prec, fusion, min_fused
        self.keep_amps = keep_amps
        # state vectors of 9..batch_max_qubits qubits go through qs_batch
        # (0 turns batching off)
        self.batch_max_qubits, self.batch_tile = batch_max_qubits, batch_tile
        self.streams = [torch.cuda.Stream(device=env.device) for _ in range(slots)]

    def batchable(self, req: Request) -> bool:
        return req.kind == Q.STATEVEC and 9 <= req.n <= self.batch_max_qubits

    def run_batch(self, reqs, slot: int):
        """All `reqs` (batchable) on one slot: their registers, one qs_batch
        run from |0..0>, then each register's measure-all.  A register's
        arithmetic depends only on its own circuit and the batch tile width,
        so its result is the same in any batch."""
        torch = self.torch
        stream = self.streams[slot]
        regs, circs, out = [], [], []
        with torch.cuda.stream(stream):
            try:
                for r in reqs:
                    regs.append(Q.Register(self.env, r.n, Q.STATEVEC, self.prec, stream=stream))
                    circs.append(Q.Circuit(r.ops))
                b = Q.Batch(regs, circs, self.batch_tile)
                try:
                    b.run(init_zero=True)
                finally:
                    b.close()
                for r, reg in zip(reqs, regs):
                    outs, probs = reg.measure_all(r.draws[:r.n])
                    out.append((outs, probs, reg.get_amps() if self.keep_amps else None))
            finally:
                for c in circs:
                    c.close()
                for reg in regs:
                    reg.close()
        return out

    def nbytes(self, req: Request) -> int:
        return Q.reg_bytes(req.n, req.kind, self.prec)

    def run(self, req: Request, slot: int):
        if self.batchable(req):
            # a batch of one: the same kernels as in a batch job, so a
            # request's result does not depend on whether it was batched
            return self.run_batch([req], slot)[0]
        torch = self.torch
        stream = self.streams[slot]
        with torch.cuda.stream(stream):
            reg = Q.Register(self.env, req.n, req.kind, self.prec, stream=stream)
            try:
                reg.init_zero()
                circ = Q.Circuit(req.ops)
                if req.kind == Q.DENSITY and 2 * req.n >= 9:
                    k = min(self.fusion, 2 * req.n, 14 if self.prec == Q.C64 else 13)
                    tb = 9 if (k == 13 and self.prec == Q.C128) else _TB_OF[k]
                    circ.run_tiled(reg, k, tb)
                else:
                    fused = req.kind == Q.STATEVEC and req.n >= self.min_fused
                    circ.run(reg, self.fusion if fused else 0)
                circ.close()
                outs, probs = reg.measure_all(req.draws[:req.n])
                amps = reg.get_amps() if self.keep_amps else None
            finally:
                reg.close()
        return outs, probs, amps


@dataclass
class Server:
    executor: object
    budget_bytes: int = 256 << 30
    slots: int = 8
    batch_min: int = 4   # pending small requests that make a batch job
    batch_max: int = 64  # requests per batch job
    events: list = field(default_factory=list)  # (time, bytes in use)

    def serve(self, requests, clock=time.perf_counter) -> list:
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        pending = collections.deque()
        inflight = {}
        results = []
        used = 0
        free = list(range(self.slots))[::-1]
        nxt = 0
        t0 = clock()
        self.events = [(0.0, 0)]
        can_batch = hasattr(self.executor, 'run_batch') and hasattr(self.executor, 'batchable')
        with cf.ThreadPoolExecutor(max_workers=self.slots) as pool:
            while nxt < len(reqs) or pending or inflight:
                now = clock() - t0
                while nxt < len(reqs) and reqs[nxt].arrival <= now:
                    pending.append(reqs[nxt])
                    nxt += 1
                # admit in arrival order while a slot and the bytes are free
                while pending and free:
                    r = pending[0]
                    b = self.executor.nbytes(r)
                    if b == 0 or b > self.budget_bytes:
                        pending.popleft()
                        results.append(Result(r.rid, [], [], r.arrival, now, now, b,
                                              error='request exceeds the HBM budget'))
                        continue
                    if used + b > self.budget_bytes:
                        break
                    if (can_batch and self.executor.batchable(r)
                            and sum(1 for x in pending if self.executor.batchable(x)) >= self.batch_min):
                        # the head and every other pending batchable request
                        # that fits, in arrival order, as one job
                        group, gb, rest = [], 0, collections.deque()
                        while pending:
                            x = pending.popleft()
                            xb = self.executor.nbytes(x)
                            if (len(group) < self.batch_max and self.executor.batchable(x)
                                    and 0 < xb and used + gb + xb <= self.budget_bytes):
                                group.append(x)
                                gb += xb
                            else:
                                rest.append(x)
                        pending = rest
                        used += gb
                        slot = free.pop()
                        fut = pool.submit(self.executor.run_batch, group, slot)
                        inflight[fut] = (group, now, gb, slot)
                        self.events.append((now, used))
                        continue
                    pending.popleft()
                    used += b
                    slot = free.pop()
                    fut = pool.submit(self.executor.run, r, slot)
                    inflight[fut] = (r, now, b, slot)
                    self.events.append((now, used))
                if inflight:
                    timeout = None
                    if nxt < len(reqs):
                        timeout = max(0.0, reqs[nxt].arrival - (clock() - t0))
                    done, _ = cf.wait(list(inflight), timeout=timeout, return_when=cf.FIRST_COMPLETED)
                else:
                    done = set()
                    if nxt < len(reqs):
                        time.sleep(max(0.0, reqs[nxt].arrival - (clock() - t0)))
                for fut in done:
                    r, t_adm, b, slot = inflight.pop(fut)
                    t_end = clock() - t0
                    used -= b
                    free.append(slot)
                    self.events.append((t_end, used))
                    group = r if isinstance(r, list) else [r]
                    try:
                        outs = fut.result() if isinstance(r, list) else [fut.result()]
                        for x, (o, p, amps) in zip(group, outs):
                            results.append(Result(x.rid, o, p, x.arrival, t_adm, t_end, self.executor.nbytes(x), amps))
                    except Exception as e:  # reported per request; the loop keeps serving
                        for x in group:
                            results.append(Result(x.rid, [], [], x.arrival, t_adm, t_end, self.executor.nbytes(x),
                                                  error=str(e)))
        return sorted(results, key=lambda x: x.rid)

    def summary(self, results) -> dict:
        ok = [r for r in results if r.error is None]
        lat = np.array([r.latency for r in ok]) if ok else np.array([0.0])
        makespan = max((r.finished for r in results), default=0.0)
        ev = (self.events or [(0.0, 0)]) + [(makespan, 0)]
        area = sum((ev[i + 1][0] - ev[i][0]) * ev[i][1] for i in range(len(ev) - 1))
        return {
            'requests': len(results),
            'completed': len(ok),
            'failed': len(results) - len(ok),
            'makespan_s': makespan,
            'circuits_per_s': len(ok) / makespan if makespan > 0 else 0.0,
            'latency_p50_s': float(np.percentile(lat, 50)),
            'latency_p99_s': float(np.percentile(lat, 99)),
            'latency_mean_s': float(lat.mean()),
            'hbm_occupancy_mean': area / (self.budget_bytes * makespan) if makespan > 0 else 0.0,
            'hbm_peak_bytes': max((e[1] for e in self.events), default=0),
        }
