"""Throughput of the gate path on one MI355X.

Workload: one 32-qubit complex128 state vector (64 GiB) and a depth-10
layered random circuit (per layer: a Haar-random unitary on every qubit, a
CNOT brick, one phase gate with 3 controls + 1 target), 485 gates.  One step
= init |0..0> + the whole circuit (fused into HBM round trips of 2^K-
amplitude tiles by run-time compiled pass kernels, the first of which forms
|0..0> instead of reading the register; 12-qubit tiles of 256 threads by
default, or the autotuner's choice with --tile auto) + total probability +
probability of an outcome (both summed by the last pass as it stores the
final state) + one measurement of qubit 0 (its probabilities from the same
sums, then the collapse pass).  Inputs are seeded and synthetic; the register is resident
in HBM before the timed region starts.

Prints one JSON line (metric, value = gates/s, roofline of the dominant
kernel measured with HIP events around each of its launches, CPU oracle
baseline on a bounded sample).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
# fused-pass tile shapes: tile qubits, thread bits, contiguous qubits (complex128
# default, and the complex64 run of the 33-qubit leg)
DEFAULT_TILE = (12, 8, 4)
C64_TILE = (14, 10, 5)


def log(msg):
    print(f'[bench] {msg}', file=sys.stderr, flush=True)


def algorithmic_bytes(ops, n, elem):
    """One-pass-per-gate byte model: a gate reads and writes every amplitude
    it may change (2 E per amplitude)."""
    total = 0
    for o in ops:
        if o.kind == 'u':
            total += 2 * elem * (1 << (n - len(o.controls)))
        elif o.kind == 'x':
            total += 2 * elem * (1 << (n - len(o.controls)))
        elif o.kind == 'phase':
            total += 2 * elem * (1 << (n - len(o.qubits)))
    return total


FP64_PEAK_TFLOPS = 78.6


def algorithmic_flops(ops, n):
    """Real floating-point operations of the gates: a dense 2x2 gate costs
    14 per amplitude it may change (two complex products and a complex
    sum), a phase 6 per amplitude it multiplies, a NOT none."""
    total = 0
    for o in ops:
        if o.kind == 'u':
            total += 14 * (1 << (n - len(o.controls)))
        elif o.kind == 'phase':
            total += 6 * (1 << (n - len(o.qubits)))
    return total


def recorded_traffic(n, K, TB, L):
    """HBM bytes per fused pass from the committed rocprofv3 counter summary,
    or None when that summary was taken for another shape or an older version
    of the pass generator."""
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(root, 'profiles', f'qs_pass_{n}q_c128_hbm_traffic.md')
    if not os.path.exists(path):
        return None
    src = b''.join(open(os.path.join(root, 'paper_1802_08032_amd', 'csrc', f), 'rb').read()
                   for f in ('qs_jit.hip', 'qs_plan.hip'))
    sha = hashlib.sha1(src).hexdigest()[:12]
    for line in open(path):
        line = line.strip()
        if line.startswith('{') and '"traffic_bytes"' in line:
            rec = json.loads(line)
            if rec.get('tile') == [K, TB, L] and rec.get('generator_sha1') == sha and rec.get('qubits') == n:
                return rec['traffic_bytes']
    return None


def cpu_model():
    try:
        for line in open('/proc/cpuinfo'):
            if line.startswith('model name'):
                return line.split(':', 1)[1].strip()
    except OSError:
        pass
    return 'unknown'


def cpu_baseline(ops_full, n_full, sample_qubits=28, budget_s=12.0, single_qubits=26, single_budget_s=6.0):
    """Oracle (plain CPU code) applying the same circuit's gates to a
    sample_qubits register until ~budget_s elapses; scaled to n_full by the
    2^(n_full - sample_qubits) amplitude ratio (the cost per gate is linear
    in the number of amplitudes).  Timed with the process's OpenMP threads,
    then on one thread over a smaller sample."""
    import oracle as O

    def sample(n, budget):
        amp = O.zero_state(n)
        ops = [o for o in ops_full if max(o.touched()) < n][:200]
        t0 = time.perf_counter()
        done = 0
        for op in ops:
            O.apply_sv(amp, n, op)
            done += 1
            if time.perf_counter() - t0 > budget:
                break
        dt = time.perf_counter() - t0
        return 1.0 / (dt / done * (1 << (n_full - n))), (f'first {done} gates of the same circuit on a {n}-qubit '
                                                        f'complex128 register ({dt:.1f} s), scaled by '
                                                        f'2^{n_full - n} to {n_full} qubits')

    threads = int(os.environ.get('OMP_NUM_THREADS', os.cpu_count() or 1))
    value, text = sample(sample_qubits, budget_s)
    prev = O.set_threads(1)
    try:
        value1, text1 = sample(single_qubits, single_budget_s)
    finally:
        O.set_threads(prev)
    return {
        'value': value,
        'unit': 'gates/s',
        'cores': threads,
        'kind': 'oracle',
        'sample': text,
        'cpu_model': cpu_model(),
        'logical_cpus': os.cpu_count(),
        'single_thread': {'value': value1, 'unit': 'gates/s', 'cores': 1, 'sample': text1},
    }


def fidelity_deficit(torch, ref, cur, chunk=1 << 28):
    """1 - |<ref|cur>|^2 of two registers' tensors (cur not renormalised),
    accumulated in complex128 over chunks."""
    acc = 0j
    for s in range(0, ref.numel(), chunk):
        a = ref[s:s + chunk]
        b = cur[s:s + chunk].to(torch.complex128)
        acc += complex(torch.vdot(a, b).item())
    return 1.0 - abs(acc) ** 2


def paper_leg(q, torch, log, n=32, depth=100, seed=7, tiles=((12, 8, 4), (13, 9, 4))):
    """The paper's own benchmark shape (Sec. II.C): gate set {H, T, CZ,
    X^1/2, Y^1/2} on the linear topology, 32 qubits complex128, depth 100,
    through the compiled passes; gates/s of the circuit alone (init
    excluded), at each of `tiles` (the bench tile and 13-qubit tiles, which
    hold this circuit in fewer passes) and at the faster of them."""
    from workloads import paper_random_circuit
    ops = paper_random_circuit(n, depth, seed)
    single = sum(1 for o in ops if not (o.kind == 'phase' and len(o.qubits) == 2))
    env = q.Env(0)
    reg = q.Register(env, n, q.STATEVEC, q.C128)
    c = q.Circuit(ops)
    by_tile = {}
    for K, TB, L in tiles:
        reg.init_zero()
        passes = c.run_compiled(reg, K, TB, 0, L)  # compile + warm
        times = []
        for _ in range(3):
            reg.init_zero()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            c.run_compiled(reg, K, TB, 0, L)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        by_tile[f'{K},{TB},{L}'] = {'fused_passes': passes, 'fused_s': min(times),
                                    'fused_gates_per_s': len(ops) / min(times),
                                    'total_prob_error': abs(reg.calc_total_prob() - 1.0)}
        log(f"paper circuit {n}q depth {depth}, tile {K},{TB},{L}: {len(ops)} gates in {passes} passes, "
            f"{len(ops) / min(times):.0f} gates/s")
    best = min(by_tile, key=lambda k: by_tile[k]['fused_s'])
    out = {'qubits': n, 'depth': depth, 'gates': len(ops), 'single_qubit_gates': single,
           'cz_gates': len(ops) - single, 'tile': [int(x) for x in best.split(',')], **by_tile[best],
           'by_tile': by_tile}
    c.close()
    reg.close()
    env.close()
    torch.cuda.empty_cache()
    return out


def cpu_configs_leg(log, budget_s=5.0):
    """The oracle on the host cores for the other workloads, with all OpenMP
    threads and with one:
    * 16-qubit depth-20 layered circuit (Haar layer + CNOT brick, 470 gates), whole;
    * the 512 registers of 10..20 qubits with depth-16 RY/RZ + CZ circuits:
      one register of every size present, each circuit whole, weighted by the
      number of registers of that size (one thread: sizes above 16 scaled from
      size 16 by the amplitude ratio, labelled);
    * the 14-qubit noisy density matrix (1015 ops): the first ops until the
      budget runs out, scaled to the whole list (labelled)."""
    import oracle as O
    from workloads import layered_circuit, noisy_circuit, param_circuit
    threads = int(os.environ.get('OMP_NUM_THREADS', os.cpu_count() or 1))
    out = {'cpu_model': cpu_model(), 'kind': 'oracle'}
    c0 = layered_circuit(16, 20, seed=0)
    rng = np.random.Generator(np.random.PCG64(3))
    sizes = [int(v) for v in rng.integers(10, 21, 512)]
    counts = {n: sizes.count(n) for n in sorted(set(sizes))}
    dm_ops = noisy_circuit(14, 10, 2)
    for label, nthr in (('all_threads', threads), ('one_thread', 1)):
        prev = O.set_threads(nthr)
        try:
            t0 = time.perf_counter()
            O.run_sv(16, c0)
            t_c0 = time.perf_counter() - t0
            per_size, scaled = {}, []
            for n in counts:
                if nthr == 1 and n > 16:
                    per_size[n] = per_size[16] * (1 << (n - 16))
                    scaled.append(n)
                    continue
                ops = param_circuit(n, 16, 1000 + sizes.index(n))
                t0 = time.perf_counter()
                O.run_sv(n, ops)
                per_size[n] = time.perf_counter() - t0
            t_batch = sum(counts[n] * per_size[n] for n in counts)
            rho = O.dm_zero(14)
            t0 = time.perf_counter()
            done = 0
            for op in dm_ops:
                O.apply_dm(rho, 14, op)
                done += 1
                if time.perf_counter() - t0 > budget_s:
                    break
            t_dm = (time.perf_counter() - t0) / done * len(dm_ops)
        finally:
            O.set_threads(prev)
        out[label] = {
            'cores': nthr,
            'c0_16q_layered_circuits_per_s': 1.0 / t_c0, 'c0_gates_per_s': len(c0) / t_c0,
            'c3_512_registers_circuits_per_s': 512 / t_batch,
            'c3_sample': ('one whole circuit per register size, weighted by the size counts'
                          + (f'; sizes {scaled} scaled from 16 qubits' if scaled else '')),
            'c2_14q_noisy_dm_s': t_dm, 'c2_ops_per_s': len(dm_ops) / t_dm,
            'c2_sample': f'first {done} of {len(dm_ops)} ops timed, scaled to all',
        }
        log(f"cpu {label}: c0 {1.0 / t_c0:.2f} circuits/s, c3 {512 / t_batch:.1f} circuits/s, "
            f"c2 {t_dm:.0f} s per circuit")
    return out


def c64_33q_leg(q, torch, log, depth=10):
    """33-qubit depth-10 layered circuit (the 32-qubit workload's generator)
    in complex64 (64 GiB), scored against a complex128 run of the same
    circuit (128 GiB) by fidelity; both through the compiled passes."""
    from workloads import layered_circuit
    n = 33
    ops = layered_circuit(n, depth, seed=1, mcphase=True)
    env = q.Env(0)
    c = q.Circuit(ops)
    out = {'qubits': n, 'gates': len(ops)}
    ref = q.Register(env, n, q.STATEVEC, q.C128)
    ref.init_zero()
    c.run_compiled(ref, DEFAULT_TILE[0], DEFAULT_TILE[1], 0, DEFAULT_TILE[2])
    cur = q.Register(env, n, q.STATEVEC, q.C64)
    cur.init_zero()
    c.run_compiled(cur, C64_TILE[0], C64_TILE[1], 0, C64_TILE[2])  # compile + warm
    times = []
    for _ in range(2):
        cur.init_zero()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c.run_compiled(cur, C64_TILE[0], C64_TILE[1], 0, C64_TILE[2])
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    out['c64_gates_per_s'] = len(ops) / min(times)
    out['c64_tile'] = list(C64_TILE)
    out['c64_vs_c128_fidelity_deficit'] = fidelity_deficit(torch, ref.tensor, cur.tensor)
    out['c128_total_prob_error'] = abs(ref.calc_total_prob() - 1.0)
    log(f"33q c64: {out['c64_gates_per_s']:.1f} gates/s, fidelity deficit vs c128 "
        f"{out['c64_vs_c128_fidelity_deficit']:.2e}")
    cur.close()
    ref.close()
    c.close()
    env.close()
    torch.cuda.empty_cache()
    return out


def batched_leg(q, torch, log, reps=5):
    """512 registers of 10..20 qubits (uniform, seed 3), depth-16 RY/RZ + CZ
    ladder circuits (register i: seed 1000 + i): one persistent launch per
    batch replayed from a HIP graph, in complex128 and complex64, against the
    plain path that runs one circuit at a time with one kernel per gate."""
    from workloads import param_circuit
    rng = np.random.Generator(np.random.PCG64(3))
    sizes = [int(v) for v in rng.integers(10, 21, 512)]
    ops = [param_circuit(n, 16, 1000 + i) for i, n in enumerate(sizes)]
    from paper_1802_08032_amd import autotune
    env = q.Env(0)
    out = {'registers': len(sizes), 'depth': 16, 'gates': int(sum(len(o) for o in ops))}
    amps = {}
    for name, prec in (('c128', q.C128), ('c64', q.C64)):
        regs = [q.Register(env, n, q.STATEVEC, prec) for n in sizes]
        circs = [q.Circuit(o) for o in ops]
        # tile width chosen by the autotuner (graph replays of this batch)
        tuned = autotune.tune_batch(regs, circs, ops, log=log)
        out[f'batched_{name}_tile_qubits'] = tuned['tile_qubits']
        out[f'batched_{name}_autotune'] = [{k: t[k] for k in ('tile_qubits', 'seconds', 'passes')}
                                           for t in tuned.get('trials', [])]
        b = q.Batch(regs, circs, tuned['tile_qubits'])
        b.capture(init_zero=True)
        b.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            b.replay()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        p0, tot = b.probs(0)
        out[f'batched_{name}_circuits_per_s'] = len(sizes) / dt
        out[f'batched_{name}_ms_per_batch'] = dt * 1e3
        out[f'batched_{name}_max_total_prob_error'] = float(np.max(np.abs(tot - 1.0)))
        out[f'batched_{name}_mean_z0'] = float(np.mean(2 * p0 - 1))
        amps[name] = [r.get_amps() for r in regs]
        log(f'batched {name}: {dt * 1e3:.2f} ms per 512 circuits')
        b.close()
        for c in circs:
            c.close()
        for r in regs:
            r.close()
    fids = [1.0 - abs(np.vdot(a, b)) ** 2 for a, b in zip(amps['c128'], amps['c64'])]
    out['c64_vs_c128_max_fidelity_deficit'] = float(np.max(fids))
    # plain path: one circuit at a time, one kernel per gate, complex128
    regs = [q.Register(env, n, q.STATEVEC, q.C128) for n in sizes]
    circs = [q.Circuit(o) for o in ops]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r, c in zip(regs, circs):
        r.init_zero()
        c.run(r, 0)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out['plain_c128_circuits_per_s'] = len(sizes) / dt
    log(f'plain c128: {dt:.2f} s per 512 circuits')
    for c in circs:
        c.close()
    for r in regs:
        r.close()
    env.close()
    return out


def dm_leg(q, torch, log, N=14, depth=10, seed=2):
    """14-qubit density matrix (its Eq. 2 vector has 2^28 entries, 4 GiB
    complex128): the depth-10 layered circuit with depolarising, dephasing
    and damping after every gate on each touched qubit, run one kernel per
    op and as fused passes of the 28-qubit vector; trace, per-qubit outcome
    probabilities, Hermiticity on sampled entry pairs, and fused vs per-op
    agreement."""
    from workloads import noisy_circuit
    ops = noisy_circuit(N, depth, seed)
    elem = 16
    chans = sum(1 for o in ops if o.kind in ('dephasing', 'depolarising', 'damping'))
    # one-pass-per-op byte model: a gate (Eq. 2 fused into one pass) or a
    # channel reads and writes the whole vector, dephasing only its
    # off-diagonal half of each 2x2 block
    dm_bytes = sum(elem * (1 << (2 * N)) * (1 if o.kind == 'dephasing' else 2) for o in ops)
    env = q.Env(0)
    reg = q.Register(env, N, q.DENSITY, q.C128)
    c = q.Circuit(ops)
    out = {'qubits': N, 'vector_entries': 1 << (2 * N), 'ops': len(ops), 'gates': len(ops) - chans,
           'channels': chans, 'tile': list(DEFAULT_TILE)}
    times = []
    for _ in range(2):
        reg.init_zero()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c.run(reg, 0)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    per_op = reg.tensor.clone()
    out['per_op_s'] = min(times)
    out['per_op_effective_gbps'] = dm_bytes / min(times) / 1e9
    K, TB, L = DEFAULT_TILE
    reg.init_zero()
    c.run_compiled(reg, K, TB, 0, L)  # compile + warm
    times = []
    for _ in range(3):
        reg.init_zero()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        passes = c.run_compiled(reg, K, TB, 0, L)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    out['fused_s'] = min(times)
    out['fused_passes'] = passes
    out['fused_speedup'] = out['per_op_s'] / out['fused_s']
    out['fused_ops_per_s'] = len(ops) / out['fused_s']
    out['fused_vs_per_op_max_abs'] = float((reg.tensor - per_op).abs().max())
    del per_op
    out['trace_error'] = abs(reg.calc_total_prob() - 1.0)
    out['prob0_per_qubit'] = [reg.calc_prob_of_outcome(k, 0) for k in range(N)]
    g = torch.Generator().manual_seed(seed)
    j = torch.randint(0, 1 << N, (1 << 16,), generator=g).to(reg.tensor.device)
    k = torch.randint(0, 1 << N, (1 << 16,), generator=g).to(reg.tensor.device)
    a = reg.tensor[j + (k << N)]
    b = reg.tensor[k + (j << N)]
    out['max_hermiticity_error'] = float((a - b.conj()).abs().max())
    log(f"density matrix {N} q: per-op {out['per_op_s']:.3f} s, fused {out['fused_s'] * 1e3:.1f} ms "
        f"({passes} passes), trace error {out['trace_error']:.1e}")
    c.close()
    reg.close()
    env.close()
    torch.cuda.empty_cache()
    return out


EXTRAS = ('unfused', 'pertarget', 'measure', 'cpu', 'cpuconfigs', 'paper', 'c64', 'batched', 'serving', 'dm')


def serving_leg(q, torch, log, count=200):
    """Mixed request stream (80 % state vectors of 12..30 qubits, 20 % noisy
    density matrices of 8..13 qubits, log-uniform sizes, depth 5..40, every
    qubit measured at the end), admitted by HBM bytes against 256 GiB with 8
    concurrent slots: a closed-loop run (all requests at t = 0) gives the
    capacity, then Poisson arrivals at 0.8 x that rate give the latencies.
    Each precision runs twice: every request on its own stream, and with
    state vectors of up to 20 qubits batched through qs_batch
    ('batched': batch jobs once 4 such requests wait)."""
    from paper_1802_08032_amd.serve import GpuExecutor, Request, Server
    from workloads import serving_requests

    def reqs(rate):
        return [Request(s['rid'], q.DENSITY if s['density'] else q.STATEVEC, s['n'], s['ops'], s['arrival'],
                        s['draws'], s['family']) for s in serving_requests(count, rate, 7)]

    out = {'requests': count, 'budget_gib': 256, 'slots': 8}
    for name, prec in (('c128', q.C128), ('c64', q.C64)):
        for batched in (False, True):
            env = q.Env(0)
            ex = GpuExecutor(env, prec, slots=8, batch_max_qubits=20 if batched else 0)
            srv = Server(ex, budget_bytes=256 << 30, slots=8, batch_min=4, batch_max=64)
            closed = srv.summary(srv.serve(reqs(0.0)))
            rate = 0.8 * closed['circuits_per_s']
            res = srv.serve(reqs(rate))
            opened = dict(srv.summary(res), arrival_rate=rate)
            key = name + ('_batched' if batched else '')
            out[key] = {'closed_loop': closed, 'open_loop': opened}
            log(f"serving {key}: {closed['circuits_per_s']:.2f} circuits/s closed loop; open loop at "
                f"{rate:.2f}/s: p50 {opened['latency_p50_s']:.3f} s, p99 {opened['latency_p99_s']:.3f} s")
            del ex, srv
            env.close()
            torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=5)
    ap.add_argument('--warmup', type=int, default=1)
    ap.add_argument('--qubits', type=int, default=32)
    ap.add_argument('--depth', type=int, default=10)
    ap.add_argument('--tile', default=','.join(map(str, DEFAULT_TILE)),
                    help="K,TB,contig of the fused passes, or 'auto' (autotuner)")
    ap.add_argument('--no-extras', action='store_true', help='skip every leg beyond the timed steps')
    ap.add_argument('--extras', default='all',
                    help='comma-separated legs to run after the timed steps: ' + ','.join(EXTRAS) + ' (default all)')
    ap.add_argument('--copy-calibration', action='store_true',
                    help='only run a device copy of 16 GiB (HBM counter calibration)')
    args = ap.parse_args()
    legs = set() if args.no_extras else (set(EXTRAS) if args.extras == 'all' else set(args.extras.split(',')))
    if legs - set(EXTRAS):
        sys.exit(f'unknown legs {sorted(legs - set(EXTRAS))}; choose from {",".join(EXTRAS)}')
    if args.gpus != 1:
        sys.exit('bench.py measures one GPU only: the method runs on one MI355X with the whole '
                 'state resident; --gpus above 1 is not supported.')

    import torch
    if args.copy_calibration:
        a = torch.zeros(1 << 30, dtype=torch.complex128, device='cuda')
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({'copy_bytes_read': a.numel() * 16, 'copy_bytes_written': b.numel() * 16, 'launches': 3}))
        return
    import paper_1802_08032_amd as q
    from paper_1802_08032_amd import autotune
    from workloads import layered_circuit, measurement_draws

    n, depth = args.qubits, args.depth
    elem = 16
    ops = layered_circuit(n, depth, seed=1, mcphase=True)
    gates = len(ops)
    log(f'{n} qubits c128, depth {depth}, {gates} gates')
    env = q.Env(0)
    reg = q.Register(env, n, q.STATEVEC, q.C128)
    circ = q.Circuit(ops)
    draws = measurement_draws(1, 0, args.warmup + args.steps)
    if args.tile == 'auto':
        tuned = autotune.tune(reg, circ, ops, budget_s=60.0, log=log)
        K, TB, L = tuned['tile_qubits'], tuned['thread_bits'], tuned['contig_qubits']
    else:
        K, TB, L = (int(v) for v in args.tile.split(','))
        tuned = None
    log(f'tile: {K} qubits, {1 << TB} threads, {L} contiguous qubits')

    readouts = []

    def step(i):
        # |0..0> is formed inside the first fused pass (no separate init
        # pass), and the last pass sums the total probability and P(q = 0)
        # of every qubit as it stores the final state (no separate reduction
        # passes); the measurement of qubit 0 takes its probabilities from
        # there and runs the collapse pass
        passes, probs = circ.run_compiled_probs(reg, K, TB, 0, L, init_basis=0)
        total, p_top0, p0 = probs[0], probs[n], probs[1]
        reg.measure_given_probs(0, p0, total - p0, float(draws[i]))
        readouts.append((total, p_top0))
        return passes

    passes = 0
    for i in range(args.warmup):
        passes = step(i)
        log(f'warmup {i} done ({passes} fused passes)')
    torch.cuda.synchronize()
    env.profile(True)
    env.profile_reset()
    t0 = time.perf_counter()
    for i in range(args.steps):
        passes = step(args.warmup + i)
        log(f'step {i} done')
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    launches, fused_ms = env.profile_read(q.qstate.K_FUSED)
    env.profile(False)
    ms_per_step = dt / args.steps * 1e3

    # dominant kernel: the fused tile pass, one HBM read + write of the state
    # (the first pass forms |0..0> and only writes)
    bytes_per_launch = (2 * passes - 1) * elem * (1 << n) / max(1, passes)
    avg_ms = fused_ms / max(1, launches)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9

    step_bytes = (algorithmic_bytes(ops, n, elem) + elem * (1 << n) * (1 + 1 + 0.5 + 2.5))
    eff_gbs = step_bytes * args.steps / dt / 1e9

    # Roofline of the dominant kernel (the fused pass).  Per launch it must
    # move 2 E 2^n bytes and carry the circuit's algorithmic FP64 work
    # divided over the passes; the bound is the larger of the two floors.
    flops_per_launch = algorithmic_flops(ops, n) / max(1, passes)
    hbm_floor_ms = bytes_per_launch / (HBM_PEAK_GBS * 1e9) * 1e3
    alu_floor_ms = flops_per_launch / (FP64_PEAK_TFLOPS * 1e12) * 1e3
    achieved_tf = flops_per_launch / (avg_ms * 1e-3) / 1e12
    hbm_part = {'achieved': achieved, 'peak': HBM_PEAK_GBS, 'unit': 'GB/s', 'frac': achieved / HBM_PEAK_GBS,
                'floor_ms': hbm_floor_ms}
    alu_part = {'achieved': achieved_tf, 'peak': FP64_PEAK_TFLOPS, 'unit': 'TFLOP/s',
                'frac': achieved_tf / FP64_PEAK_TFLOPS, 'floor_ms': alu_floor_ms}
    main_part, companion = (alu_part, ('hbm', hbm_part)) if alu_floor_ms > hbm_floor_ms else \
        (hbm_part, ('alu', alu_part))
    roofline = {
        'bound': 'alu' if alu_floor_ms > hbm_floor_ms else 'hbm',
        'achieved': main_part['achieved'], 'peak': main_part['peak'], 'unit': main_part['unit'],
        'frac': main_part['frac'], 'traffic': recorded_traffic(n, K, TB, L),
        'kernel': f'qs_pass (run-time compiled fused pass, {K}-qubit tile)', 'launches': launches,
        'avg_ms': avg_ms, 'bytes_per_launch': bytes_per_launch, 'flops_per_launch': flops_per_launch,
        companion[0]: companion[1],
    }

    out = {
        'metric': 'gates/s & effective HBM GB/s (% peak), 32q SV; circuits/s + p99 latency',
        'value': gates * args.steps / dt,
        'unit': 'gates/s',
        'n_gpus': 1,
        'steps': args.steps,
        'warmup': args.warmup,
        'ms_per_step': ms_per_step,
        'higher_is_better': True,
        'scaling': 'weak',
        'vs_baseline': None,
        'dtype': 'f64',
        'data': 'synthetic',
        'config': {
            'workload': f'{n}-qubit complex128 state vector, depth-{depth} layered random circuit '
                        f'(Haar 1q layer + CNOT brick + 3-control phase per layer), fused tiles of {K} qubits',
            'qubits': n, 'depth': depth, 'gates_per_step': gates, 'tile_qubits': K,
            'workgroup_threads': 1 << TB, 'contig_qubits': L, 'autotuned': tuned is not None,
            'fused_passes_per_step': passes, 'parallelism': 'single GPU',
        },
        'circuits_per_s': args.steps / dt,
        # readouts the last pass summed in the timed steps
        'step_total_prob_max_error': max(abs(t - 1.0) for t, _ in readouts[args.warmup:]),
        'step_prob_top_qubit_0': readouts[-1][1],
        # the paper's one-pass-per-gate bytes over the fused step time: what
        # an unfused engine would need to sustain; above the HBM peak, so it
        # is not a roofline fraction
        'one_pass_per_gate_equiv_gbps': eff_gbs,
        'one_pass_per_gate_equiv_pct_of_hbm_peak': 100.0 * eff_gbs / HBM_PEAK_GBS,
        'roofline': roofline,
    }
    if 'unfused' in legs:
        # unfused circuit (one kernel per gate, the paper's one pass per gate)
        log('unfused circuit')
        reg.init_zero()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        circ.run(reg, 0)
        torch.cuda.synchronize()
        t_unf = time.perf_counter() - t1
        out['unfused_gates_per_s'] = gates / t_unf
        out['unfused_effective_gbps'] = algorithmic_bytes(ops, n, elem) / t_unf / 1e9
        out['unfused_pct_of_hbm_peak'] = 100.0 * out['unfused_effective_gbps'] / HBM_PEAK_GBS
        out['fused_pass_speedup'] = t_unf / (fused_ms / max(1, launches) * passes * 1e-3)
    if tuned is not None:
        out['autotune_trials'] = [{k: t[k] for k in ('tile_qubits', 'thread_bits', 'contig_qubits', 'passes',
                                                      'seconds')} for t in tuned.get('trials', [])]
    if 'pertarget' in legs:
        # per-target effective bandwidth of one dense gate (median of 5)
        log('per-target sweep')
        u = ops[0].u
        per_t = []
        for t in range(n):
            times = []
            for _ in range(5):
                s = torch.cuda.Event(enable_timing=True)
                e = torch.cuda.Event(enable_timing=True)
                s.record()
                reg.unitary(t, u)
                e.record()
                e.synchronize()
                times.append(s.elapsed_time(e))
            per_t.append(round(2 * elem * (1 << n) / (sorted(times)[2] * 1e-3) / 1e9, 1))
        out['per_target_gbps'] = per_t
    if 'measure' in legs:
        # measurement of every qubit on the circuit's output: qs_measure_all
        # (histogram walk, one write-only collapse) against n successive
        # qs_measure calls with the same draws, from the same snapshot
        log('measure all qubits')
        reg.init_zero()
        circ.run_compiled(reg, K, TB, 0, L)
        snap = reg.tensor.clone()
        mdraws = measurement_draws(2, 0, n)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        outs_all, probs_all = reg.measure_all(mdraws)
        torch.cuda.synchronize()  # the collapse is queued after the outcomes return
        t_all = time.perf_counter() - t1
        reg.tensor.copy_(snap)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        seq = [reg.measure(k, float(mdraws[k])) for k in range(n)]
        torch.cuda.synchronize()
        t_seq = time.perf_counter() - t1
        del snap
        torch.cuda.empty_cache()
        out['measure_all'] = {
            'qubits': n, 'measure_all_ms': t_all * 1e3, 'sequential_ms': t_seq * 1e3,
            'speedup': t_seq / t_all,
            'outcomes_equal': [o for o, _ in seq] == outs_all,
            'max_prob_rel_diff': max(abs(p - ps) / ps for (_, ps), p in zip(seq, probs_all)),
        }
        log(f"measure all {n} qubits: {t_all * 1e3:.1f} ms vs {t_seq * 1e3:.1f} ms sequential")
    if 'cpu' in legs:
        log('cpu baseline')
        out['cpu_baseline'] = cpu_baseline(ops, n)
    circ.close()
    reg.close()
    env.close()
    del reg
    torch.cuda.empty_cache()
    if 'cpuconfigs' in legs:
        log('cpu baselines of the other workloads')
        out['cpu_baseline_other_workloads'] = cpu_configs_leg(log)
    if 'paper' in legs:
        log('paper-shaped random circuit')
        out['paper_circuit'] = paper_leg(q, torch, log)
    if 'c64' in legs:
        log('33-qubit complex64 vs complex128')
        out['c64_33q'] = c64_33q_leg(q, torch, log)
    if 'dm' in legs:
        log('14-qubit noisy density matrix')
        out['density_matrix'] = dm_leg(q, torch, log)
    if 'batched' in legs:
        log('batched registers')
        out['batched'] = batched_leg(q, torch, log)
    if 'serving' in legs:
        log('serving')
        out['serving'] = serving_leg(q, torch, log)
    print(json.dumps(out), flush=True)


if __name__ == '__main__':
    main()
