"""Brute-force reference: full 2^n x 2^n operators built from Kronecker products.

Independent of the oracle's pair-update loops: a gate is materialised as a
dense matrix (qubit 0 is the rightmost Kronecker factor, so qubit q is bit q
of the index) and applied by a matrix-vector product.  Only for n <= 10.
"""
from __future__ import annotations

from functools import reduce

import numpy as np

I2 = np.eye(2, dtype=np.complex128)
P1 = np.array([[0, 0], [0, 1]], dtype=np.complex128)
PX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
PY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
PZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)


def kron_factors(n: int, factors: dict) -> np.ndarray:
    """kron(f_{n-1}, ..., f_0) with f_q = factors.get(q, I)."""
    return reduce(np.kron, [factors.get(q, I2) for q in reversed(range(n))])


def gate_matrix(n: int, controls, target: int, u) -> np.ndarray:
    """|1..1><1..1|_C (x) U_t + (I - |1..1><1..1|_C) (x) I_t."""
    u = np.asarray(u, dtype=np.complex128)
    proj = {c: P1 for c in controls}
    with_u = dict(proj)
    with_u[target] = u
    dim = 1 << n
    return np.eye(dim, dtype=np.complex128) - kron_factors(n, proj) + kron_factors(n, with_u)


def phase_matrix(n: int, qubits, angle: float) -> np.ndarray:
    proj = kron_factors(n, {q: P1 for q in qubits})
    dim = 1 << n
    return np.eye(dim, dtype=np.complex128) + (np.exp(1j * angle) - 1.0) * proj


def op_matrix(n: int, op) -> np.ndarray:
    if op.kind == 'u':
        return gate_matrix(n, op.controls, op.target, op.u)
    if op.kind == 'x':
        return gate_matrix(n, op.controls, op.target, PX)
    if op.kind == 'phase':
        return phase_matrix(n, op.qubits, op.angle)
    raise ValueError(op.kind)


def kraus_ops(kind: str, p: float):
    if kind == 'dephasing':
        return [np.sqrt(1 - p) * I2, np.sqrt(p) * PZ]
    if kind == 'depolarising':
        return [np.sqrt(1 - p) * I2] + [np.sqrt(p / 3) * P for P in (PX, PY, PZ)]
    if kind == 'damping':
        return [np.array([[1, 0], [0, np.sqrt(1 - p)]], dtype=np.complex128),
                np.array([[0, np.sqrt(p)], [0, 0]], dtype=np.complex128)]
    raise ValueError(kind)


def run_sv(n: int, ops, init_index: int = 0) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[init_index] = 1
    for op in ops:
        psi = op_matrix(n, op) @ psi
    return psi


def run_dm(N: int, ops, init_index: int = 0) -> np.ndarray:
    """Returns the 2^N x 2^N matrix rho (not the Eq. 2 vector)."""
    dim = 1 << N
    rho = np.zeros((dim, dim), dtype=np.complex128)
    rho[init_index, init_index] = 1
    for op in ops:
        if op.kind in ('u', 'x', 'phase'):
            G = op_matrix(N, op)
            rho = G @ rho @ G.conj().T
        else:
            Ks = [kron_factors(N, {op.target: K}) for K in kraus_ops(op.kind, op.p)]
            rho = sum(K @ rho @ K.conj().T for K in Ks)
    return rho


def dm_to_vector(rho: np.ndarray) -> np.ndarray:
    """Eq. 2 layout: rho[j][k] at j + 2^N k (column stacking)."""
    return np.ascontiguousarray(rho.T).reshape(-1)
