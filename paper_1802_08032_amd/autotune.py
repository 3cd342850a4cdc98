"""Autotuner for fused state-vector circuits.

`tune` chooses the tile shape of the run-time compiled passes -- tile qubits
K (fusion width), thread bits TB (workgroup size 2^TB, so 2^(K-TB)
amplitudes per thread) and the number of low qubits kept contiguous in HBM
-- by timing candidates on the caller's own register and circuit.
`tune_batch` chooses the tile width of a batch of registers (qs_batch) by
timing graph replays of the caller's own batch at each candidate width.  Results are cached in
a JSON file ($QS_TUNE_CACHE, else $QS_JIT_CACHE, else ~/.cache/qstate)
keyed by (device name, qubits, precision, circuit structure).
"""
from __future__ import annotations

import hashlib
import json
import os
import time

import torch

from . import qstate as Q

# (tile qubits, thread bits, contiguous qubits), most promising first
CANDIDATES = {
    Q.C128: [(12, 8, 4), (13, 9, 4), (12, 9, 4), (13, 10, 4), (12, 9, 6), (11, 8, 4)],
    Q.C64: [(14, 10, 5), (13, 9, 4), (14, 10, 4), (12, 8, 4), (13, 10, 4), (14, 10, 6)],
}


def _cache_path() -> str:
    d = (os.environ.get('QS_TUNE_CACHE') or os.environ.get('QS_JIT_CACHE')
         or os.path.join(os.path.expanduser('~'), '.cache', 'qstate'))
    os.makedirs(d, exist_ok=True)
    return os.path.join(d, 'tune.json')


def circuit_signature(ops) -> str:
    """Hash of the structure (kinds, targets, controls) -- not of the matrices."""
    h = hashlib.sha1()
    for o in ops:
        h.update(f'{o.kind}:{o.target}:{sorted(o.controls)}:{sorted(o.qubits)};'.encode())
    return h.hexdigest()[:16]


def _key(n, prec, sig) -> str:
    name = torch.cuda.get_device_name(0) if torch.cuda.is_available() else 'cpu'
    return f'{name}|n={n}|prec={prec}|{sig}'


def _load_cache(path):
    if os.path.exists(path):
        try:
            return json.load(open(path))
        except (OSError, ValueError):
            return {}
    return {}


def _store(path, cache, key, value):
    cache[key] = value
    tmp = path + f'.tmp{os.getpid()}'
    with open(tmp, 'w') as f:
        json.dump(cache, f)
    os.replace(tmp, path)


def tune(reg: Q.Register, circuit: Q.Circuit, ops, budget_s: float = 90.0, reps: int = 2,
         candidates=None, use_cache: bool = True, log=None) -> dict:
    """Time the candidate shapes on `reg` (its contents are overwritten) and
    return {'tile_qubits', 'thread_bits', 'contig_qubits', 'seconds', 'passes', 'trials'}."""
    n, prec = reg.n, reg.prec
    key = _key(n, prec, circuit_signature(ops))
    path = _cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            return dict(cache[key], cached=True)
    cands = [c for c in (candidates or CANDIDATES[prec]) if c[0] <= n]
    trials = []
    t_start = time.perf_counter()
    for K, TB, L in cands:
        if trials and time.perf_counter() - t_start > budget_s:
            break
        try:
            reg.init_zero()
            passes = circuit.run_compiled(reg, K, TB, 0, L)  # compiles (cached on disk) and warms up
            torch.cuda.synchronize()
            best = float('inf')
            for _ in range(reps):
                reg.init_zero()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                circuit.run_compiled(reg, K, TB, 0, L)
                torch.cuda.synchronize()
                best = min(best, time.perf_counter() - t0)
        except Q.QStateError as e:
            if log:
                log(f'autotune: {K},{TB},{L} failed: {e}')
            continue
        trials.append({'tile_qubits': K, 'thread_bits': TB, 'contig_qubits': L, 'seconds': best,
                       'passes': passes})
        if log:
            log(f'autotune: tile={K} tb={TB} contig={L} passes={passes} {best * 1e3:.1f} ms')
    if not trials:
        raise Q.QStateError(-1, 'no tile shape could run this circuit')
    win = min(trials, key=lambda t: t['seconds'])
    out = dict(win, trials=trials)
    if use_cache:
        cache[key] = out
        tmp = path + f'.tmp{os.getpid()}'
        with open(tmp, 'w') as f:
            json.dump(cache, f)
        os.replace(tmp, path)
    return out


# batch tile widths (qubits), most promising first
BATCH_CANDIDATES = {Q.C128: [12, 11, 13, 10], Q.C64: [12, 13, 14, 11, 10]}


def tune_batch(regs, circuits, ops_list, candidates=None, reps: int = 3, use_cache: bool = True,
               log=None) -> dict:
    """Time a batch of `regs` x `circuits` (captured into a HIP graph, then
    replayed) at each candidate tile width; return {'tile_qubits', 'seconds',
    'passes', 'trials'} for the fastest, cached per (device, precision,
    register sizes and circuit structures).  The registers are overwritten."""
    prec = regs[0].prec
    h = hashlib.sha1()
    for r, ops in zip(regs, ops_list):
        h.update(f'{r.n}:{circuit_signature(ops)};'.encode())
    key = _key(f'batch{len(regs)}', prec, h.hexdigest()[:16])
    path = _cache_path()
    cache = _load_cache(path) if use_cache else {}
    if use_cache and key in cache:
        return dict(cache[key], cached=True)
    trials = []
    for K in (candidates or BATCH_CANDIDATES[prec]):
        try:
            b = Q.Batch(regs, circuits, K)
        except Q.QStateError as e:
            if log:
                log(f'autotune batch: tile {K} failed: {e}')
            continue
        b.capture(init_zero=True)
        b.replay()  # warm
        torch.cuda.synchronize()
        best = float('inf')
        for _ in range(reps):
            t0 = time.perf_counter()
            b.replay()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        trials.append({'tile_qubits': K, 'seconds': best, 'passes': b.info()['passes']})
        b.close()
        if log:
            log(f'autotune batch: tile {K}: {best * 1e3:.2f} ms')
    if not trials:
        raise Q.QStateError(-1, 'no batch tile width could run these circuits')
    out = dict(min(trials, key=lambda t: t['seconds']), trials=trials)
    if use_cache:
        _store(path, cache, key, out)
    return out
