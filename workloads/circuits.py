"""Seeded random circuits shaped like the paper's random-circuit benchmark.

The paper (Sec. II.C) benchmarks random circuits whose gate count grows as
O(n d), alternating single-qubit gates and controlled two-qubit gates on a
linear topology.  The exact generator it cites is not reproduced here; the
workloads below keep that shape with rules of their own:

* ``layered_circuit``  -- per layer a Haar-random 2x2 unitary on every qubit
  (ascending), then CNOT(q, q+1) on pairs starting at offset (layer mod 2);
  optionally one multi-controlled phase per layer on 4 distinct random qubits.
* ``noisy_circuit``    -- the same gates on an N-qubit density matrix; after
  every gate each touched qubit (ascending) receives depolarising, dephasing
  and amplitude damping, in that order.
* ``param_circuit``    -- per layer RY(theta) then RZ(phi) on every qubit with
  angles uniform in [0, 2 pi), then a CZ ladder on (q, q+1).
* ``paper_random_circuit`` -- the paper's gate set {H, T, CZ, X^1/2, Y^1/2}
  on a fixed linear topology (see its docstring); its gate count for 30
  qubits at depth 100 is the one the paper prints.

Everything is drawn from ``numpy.random.Generator(PCG64(seed))`` so that the
oracle and the GPU path receive identical gate lists.  Measurement draws use
a Philox4x64-10 stream keyed by (seed, request id).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Fixed 2x2 matrices (row-major, element [r][c] multiplies the bit=c amplitude
# into the bit=r amplitude, as in Eq. 1).
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / math.sqrt(2.0)


# square roots of X and Y (their squares are X and Y)
SQRT_X = np.array([[1 + 1j, 1 - 1j], [1 - 1j, 1 + 1j]], dtype=np.complex128) / 2.0
SQRT_Y = np.array([[1 + 1j, -1 - 1j], [1 + 1j, 1 + 1j]], dtype=np.complex128) / 2.0


def ry(theta: float) -> np.ndarray:
    """exp(-i theta Y / 2)."""
    c, s = math.cos(theta / 2.0), math.sin(theta / 2.0)
    return np.array([[c, -s], [s, c]], dtype=np.complex128)


def rz(phi: float) -> np.ndarray:
    """exp(-i phi Z / 2)."""
    return np.array([[np.exp(-0.5j * phi), 0], [0, np.exp(0.5j * phi)]],
                    dtype=np.complex128)


@dataclass
class Op:
    """One circuit operation.

    kind:
      'u'            dense 2x2 ``u`` on ``target`` where every qubit in
                     ``controls`` is 1
      'x'            NOT on ``target`` where every control is 1 (CNOT, Toffoli)
      'phase'        multiply by exp(i*angle) every amplitude whose bits in
                     ``qubits`` are all 1 (CZ is angle = pi on two qubits)
      'dephasing' / 'depolarising' / 'damping'
                     single-qubit channel of strength ``p`` on ``target``
      'unitary'      dense 2^k x 2^k ``u`` on ``targets`` (matrix index bit j
                     is qubit targets[j]) where every control is 1
      'kraus'        Kraus map with operators ``kraus`` (each 2^k x 2^k) on
                     ``targets`` (density matrices only)
    """
    kind: str
    target: int = -1
    controls: tuple = ()
    u: np.ndarray | None = None
    qubits: tuple = ()
    angle: float = 0.0
    p: float = 0.0
    targets: tuple = ()
    kraus: tuple = ()

    def touched(self) -> tuple:
        if self.kind == 'phase':
            return tuple(sorted(self.qubits))
        if self.kind in ('unitary', 'kraus'):
            return tuple(sorted(set(self.controls) | set(self.targets)))
        return tuple(sorted(set(self.controls) | {self.target}))


def haar_unitary(rng: np.random.Generator) -> np.ndarray:
    """Haar-random U(2): QR of a complex Gaussian matrix with the phases of
    R's diagonal moved into Q (Mezzadri, Notices AMS 54 (2007) 592)."""
    z = (rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r)
    lam = d / np.abs(d)
    return np.ascontiguousarray(q * lam[None, :], dtype=np.complex128)


def layered_circuit(n: int, depth: int, seed: int, mcphase: bool = False) -> list[Op]:
    """Haar layer + CNOT brick (+ one 4-qubit multi-controlled phase)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ops: list[Op] = []
    for layer in range(depth):
        for q in range(n):
            ops.append(Op('u', target=q, u=haar_unitary(rng)))
        q = layer % 2
        while q + 1 < n:
            ops.append(Op('x', target=q + 1, controls=(q,)))
            q += 2
        if mcphase:
            picks = [int(v) for v in rng.choice(n, size=4, replace=False)]
            phi = float(rng.uniform(0.0, 2.0 * math.pi))
            ops.append(Op('phase', qubits=tuple(picks), angle=phi,
                          controls=tuple(picks[:3]), target=picks[3]))
    return ops


def noisy_circuit(N: int, depth: int, seed: int, p_depol: float = 1e-3,
                  p_deph: float = 1e-3, gamma: float = 2e-3) -> list[Op]:
    """Layered circuit on an N-qubit density matrix with per-gate noise."""
    ops: list[Op] = []
    for g in layered_circuit(N, depth, seed):
        ops.append(g)
        for q in g.touched():
            ops.append(Op('depolarising', target=q, p=p_depol))
            ops.append(Op('dephasing', target=q, p=p_deph))
            ops.append(Op('damping', target=q, p=gamma))
    return ops


def param_circuit(n: int, depth: int, seed: int) -> list[Op]:
    """RY/RZ rotations on every qubit then a CZ ladder, per layer."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ops: list[Op] = []
    for _ in range(depth):
        for q in range(n):
            theta, phi = rng.uniform(0.0, 2.0 * math.pi, size=2)
            ops.append(Op('u', target=q, u=ry(float(theta))))
            ops.append(Op('u', target=q, u=rz(float(phi))))
        for q in range(n - 1):
            ops.append(Op('phase', qubits=(q, q + 1), angle=math.pi,
                          controls=(q,), target=q + 1))
    return ops


def product_layer(n: int, seed: int) -> list[Op]:
    """One Haar unitary per qubit (a product state when applied to |0..0>)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [Op('u', target=q, u=haar_unitary(rng)) for q in range(n)]


def measurement_draws(seed: int, request_id: int, count: int) -> np.ndarray:
    """Uniform [0, 1) doubles from Philox4x64-10 keyed by (seed, request id).

    numpy forms each double as (x >> 11) * 2**-53 from one 64-bit output."""
    gen = np.random.Generator(np.random.Philox(key=[seed & (2**64 - 1), request_id & (2**64 - 1)]))
    return gen.random(count)


def gate_counts(ops: list[Op]) -> dict:
    out: dict = {}
    for o in ops:
        key = o.kind
        if o.kind == 'u' and o.controls:
            key = 'cu'
        out[key] = out.get(key, 0) + 1
    return out


def inverse(ops: list[Op]) -> list[Op]:
    """The adjoint gate list: reversed order, U -> U^dagger, phase -> -phase."""
    out: list[Op] = []
    for o in reversed(ops):
        if o.kind == 'u':
            out.append(Op('u', target=o.target, controls=o.controls,
                          u=np.ascontiguousarray(o.u.conj().T)))
        elif o.kind == 'x':
            out.append(Op('x', target=o.target, controls=o.controls))
        elif o.kind == 'phase':
            out.append(Op('phase', qubits=o.qubits, angle=-o.angle,
                          controls=o.controls, target=o.target))
        else:
            raise ValueError(f'{o.kind} has no inverse')
    return out


def haar_unitary_dim(rng: np.random.Generator, d: int) -> np.ndarray:
    """Haar-random U(d), by the same QR recipe as haar_unitary."""
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    dg = np.diagonal(r)
    return np.ascontiguousarray(q * (dg / np.abs(dg))[None, :], dtype=np.complex128)


def haar_unitary_k(rng: np.random.Generator, k: int) -> np.ndarray:
    """Haar-random unitary on k qubits (2^k x 2^k)."""
    return haar_unitary_dim(rng, 1 << k)


def random_kraus(rng: np.random.Generator, k: int, count: int) -> tuple:
    """`count` Kraus operators on k qubits with sum K^dagger K = I: the
    blocks of the first 2^k columns of a Haar unitary of size count * 2^k
    (a Stinespring isometry)."""
    d = 1 << k
    w = haar_unitary_dim(rng, count * d)[:, :d]
    return tuple(np.ascontiguousarray(w[m * d:(m + 1) * d, :]) for m in range(count))


def random_multi_ops(n: int, count: int, seed: int, max_targets: int = 3, max_controls: int = 2,
                     kraus: bool = False) -> list[Op]:
    """Dense k-qubit unitaries (k = 1..max_targets, Haar) on random distinct
    targets with 0..max_controls random controls; with `kraus`, every third op
    is instead a random 1- or 2-qubit Kraus map of 1..4 operators."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ops: list[Op] = []
    for i in range(count):
        if kraus and i % 3 == 2:
            k = int(rng.integers(1, min(2, n) + 1))
            ts = tuple(int(v) for v in rng.choice(n, size=k, replace=False))
            ops.append(Op('kraus', targets=ts, kraus=random_kraus(rng, k, int(rng.integers(1, 5)))))
            continue
        k = int(rng.integers(1, min(max_targets, n) + 1))
        c = int(rng.integers(0, min(max_controls, n - k) + 1))
        qs = [int(v) for v in rng.choice(n, size=k + c, replace=False)]
        ops.append(Op('unitary', targets=tuple(qs[:k]), controls=tuple(qs[k:]), u=haar_unitary_k(rng, k)))
    return ops


def random_state(nbits: int, seed: int) -> np.ndarray:
    """A normalised complex Gaussian vector of 2^nbits amplitudes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    psi = rng.standard_normal(1 << nbits) + 1j * rng.standard_normal(1 << nbits)
    return np.ascontiguousarray(psi / np.linalg.norm(psi))


def random_gate_ops(n: int, count: int, seed: int, max_controls: int = 3) -> list[Op]:
    """Mixed single-target gates: dense (Haar), NOT and multi-qubit phases on
    random targets with 0..max_controls random controls."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ops: list[Op] = []
    for _ in range(count):
        k = int(rng.integers(0, min(max_controls, n - 1) + 1))
        qs = [int(v) for v in rng.choice(n, size=k + 1, replace=False)]
        kind = ('u', 'u', 'x', 'phase')[int(rng.integers(0, 4))]
        if kind == 'u':
            ops.append(Op('u', target=qs[k], controls=tuple(qs[:k]), u=haar_unitary(rng)))
        elif kind == 'x':
            ops.append(Op('x', target=qs[k], controls=tuple(qs[:k])))
        else:
            ops.append(Op('phase', qubits=tuple(qs), angle=float(rng.uniform(0, 2 * math.pi)),
                          controls=tuple(qs[:k]), target=qs[k]))
    return ops


def serving_requests(count: int, rate: float, seed: int = 7, sv_range=(12, 30), dm_range=(8, 13),
                     depth_range=(5, 40), dm_fraction: float = 0.2) -> list[dict]:
    """A stream of circuit requests with Poisson arrivals at `rate` per second
    (rate <= 0: all arrive at t = 0).  A request is a density-matrix noisy
    circuit with probability dm_fraction, else a state-vector circuit that is
    layered or parameterised with probability 1/2 each.  Qubit counts are
    log-uniform in the inclusive ranges, depths uniform; request rid draws
    its circuit from seed (seed * 1000003 + rid) and its final measurement
    draws from the Philox stream (seed, rid)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    t = 0.0
    for rid in range(count):
        if rate > 0:
            t += float(rng.exponential(1.0 / rate))
        dm = bool(rng.random() < dm_fraction)
        lo, hi = dm_range if dm else sv_range
        n = min(hi, int(math.floor(math.exp(rng.uniform(math.log(lo), math.log(hi + 1))))))
        depth = int(rng.integers(depth_range[0], depth_range[1] + 1))
        family = 'noisy' if dm else ('layered' if rng.random() < 0.5 else 'param')
        cseed = seed * 1000003 + rid
        if family == 'noisy':
            ops = noisy_circuit(n, depth, cseed)
        elif family == 'layered':
            ops = layered_circuit(n, depth, cseed)
        else:
            ops = param_circuit(n, depth, cseed)
        out.append({'rid': rid, 'density': dm, 'n': n, 'depth': depth, 'family': family, 'ops': ops,
                    'arrival': t, 'draws': measurement_draws(seed, rid, n)})
    return out


def paper_random_circuit(n: int, depth: int, seed: int) -> list[Op]:
    """Random circuit over the paper's gate set {H, T, CZ, X^1/2, Y^1/2}
    (Sec. II.C): a fixed topology for given (n, depth) and a random sequence
    of single-qubit gates.

    * Cycle 0 puts H on every qubit.
    * Cycle c = 1..depth applies CZ on the nearest-neighbour pairs (q, q+1)
      with q = (c - 1) mod 3, (c - 1) mod 3 + 3, ... (three pair classes in
      turn, so each qubit meets both neighbours).
    * In the same cycle every qubit that was in a CZ in the previous cycle
      and is not in one now gets a single-qubit gate: T if its only earlier
      single-qubit gate is the initial H, else one of {T, X^1/2, Y^1/2}
      drawn uniformly among those differing from its previous gate.

    At 30 qubits and depth 100 this gives 1020 single-qubit and 967 CZ gates,
    the counts the paper states for that size.  T is diag(1, e^(i pi/4)) and
    CZ a phase of pi on |11>, both written as phase ops."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ops: list[Op] = [Op('u', target=q, u=H) for q in range(n)]
    last = ['h'] * n
    busy_prev: set = set()
    for c in range(depth):
        pairs = [(q, q + 1) for q in range(c % 3, n - 1, 3)]
        busy = {q for p in pairs for q in p}
        for q in range(n):
            if q not in busy_prev or q in busy:
                continue
            if last[q] == 'h':
                g = 't'
            else:
                choices = [k for k in ('t', 'sx', 'sy') if k != last[q]]
                g = choices[int(rng.integers(0, len(choices)))]
            if g == 't':
                ops.append(Op('phase', qubits=(q,), angle=math.pi / 4.0, target=q))
            else:
                ops.append(Op('u', target=q, u=SQRT_X if g == 'sx' else SQRT_Y))
            last[q] = g
        for a, b in pairs:
            ops.append(Op('phase', qubits=(a, b), angle=math.pi, controls=(a,), target=b))
        busy_prev = busy
    return ops
