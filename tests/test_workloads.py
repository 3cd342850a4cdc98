"""CPU checks of the seeded input generators (no GPU).

The paper-shaped random circuit (Sec. II.C) is pinned to the gate counts the
paper prints for 30 qubits at depth 100 (tests/golden/paper_random_circuit.txt)
and checked against the rules its docstring states."""
import math
import os

import numpy as np

from workloads import H, SQRT_X, SQRT_Y, X, paper_random_circuit

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def split(ops):
    single = [o for o in ops if not (o.kind == 'phase' and len(o.qubits) == 2)]
    cz = [o for o in ops if o.kind == 'phase' and len(o.qubits) == 2]
    return single, cz


def test_paper_gate_counts():
    rows = [l.split() for l in open(os.path.join(ROOT, 'tests', 'golden', 'paper_random_circuit.txt'))
            if l.strip() and not l.startswith('#')]
    assert rows
    for n, depth, n1, n2 in ([int(v) for v in r] for r in rows):
        for seed in (0, 1, 2):  # the topology (and so the counts) does not depend on the seed
            single, cz = split(paper_random_circuit(n, depth, seed))
            assert (len(single), len(cz)) == (n1, n2)
        assert 1.0 <= n1 / n2 <= 1.4


def test_square_roots():
    assert np.allclose(SQRT_X @ SQRT_X, X)
    assert np.allclose(SQRT_Y @ SQRT_Y, np.array([[0, -1j], [1j, 0]]))


def test_paper_circuit_rules():
    n, depth = 17, 40
    ops = paper_random_circuit(n, depth, 5)
    # cycle 0: H on every qubit
    for q in range(n):
        assert ops[q].kind == 'u' and ops[q].target == q and np.array_equal(ops[q].u, H)
    last = {q: 'h' for q in range(n)}
    kinds = set()
    for o in ops[n:]:
        if o.kind == 'phase' and len(o.qubits) == 2:
            a, b = o.qubits
            assert b == a + 1 and o.angle == math.pi
            continue
        if o.kind == 'phase':
            (q,) = o.qubits
            assert o.angle == math.pi / 4
            g = 't'
        else:
            q = o.target
            assert not o.controls
            g = 'sx' if np.array_equal(o.u, SQRT_X) else 'sy'
            assert np.array_equal(o.u, SQRT_X) or np.array_equal(o.u, SQRT_Y)
        # the first gate after H is T; later ones differ from the previous one
        assert (g == 't') if last[q] == 'h' else (g != last[q])
        last[q] = g
        kinds.add(g)
    assert kinds == {'t', 'sx', 'sy'}
    # the CZs of one cycle act on disjoint qubits
    cyc = []
    for o in ops[n:]:
        if o.kind == 'phase' and len(o.qubits) == 2:
            cyc.append(o.qubits)
    assert len(cyc) == sum(len(range(c % 3, n - 1, 3)) for c in range(depth))
    # same seed, same list; another seed, another sequence of single-qubit gates
    again = paper_random_circuit(n, depth, 5)
    assert [(o.kind, o.qubits, o.target) for o in again] == [(o.kind, o.qubits, o.target) for o in ops]
    other = paper_random_circuit(n, depth, 6)
    assert [(o.kind, o.qubits) for o in other] != [(o.kind, o.qubits) for o in ops]
