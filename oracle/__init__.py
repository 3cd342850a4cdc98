"""Python shim over the plain CPU oracle (oracle.c) -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It never imports the HIP library and
the HIP library never imports it.

Conventions (shared with the paper, Sec. II.B.1): qubit q is bit q of the
index; a density matrix on N qubits is the 2N-qubit vector of Eq. 2 with
rho[j][k] stored at j + 2^N k.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, 'oracle.c')
_LIB = os.path.join(_HERE, 'liboracle.so')

OR_U, OR_X, OR_PHASE = 0, 1, 2


class OrGate(C.Structure):
    _fields_ = [('kind', C.c_int), ('target', C.c_int), ('mask', C.c_uint64),
                ('u', C.c_double * 8), ('angle', C.c_double)]


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB):
        cmd = ['gcc', '-std=c99', '-O2', '-fno-fast-math', '-fopenmp', '-fPIC',
               '-shared', _SRC, '-o', _LIB + '.tmp', '-lm']
        subprocess.check_call(cmd, cwd=_HERE)
        os.replace(_LIB + '.tmp', _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        vp, i, d, u64 = C.c_void_p, C.c_int, C.c_double, C.c_uint64
        sig = {
            'or_init_basis': (None, [vp, u64, u64]),
            'or_sv_unitary': (None, [vp, i, vp, i, i, vp]),
            'or_sv_x': (None, [vp, i, vp, i, i]),
            'or_sv_phase': (None, [vp, i, vp, i, d]),
            'or_sv_total_prob': (d, [vp, i]),
            'or_sv_prob_outcome': (d, [vp, i, i, i]),
            'or_sv_measure': (i, [vp, i, i, d, C.POINTER(d)]),
            'or_dm_unitary': (None, [vp, i, vp, i, i, vp]),
            'or_dm_x': (None, [vp, i, vp, i, i]),
            'or_dm_phase': (None, [vp, i, vp, i, d]),
            'or_dm_kraus': (None, [vp, i, i, vp, i]),
            'or_dm_dephasing': (None, [vp, i, i, d]),
            'or_dm_depolarising': (None, [vp, i, i, d]),
            'or_dm_damping': (None, [vp, i, i, d]),
            'or_dm_total_prob': (d, [vp, i]),
            'or_dm_prob_outcome': (d, [vp, i, i, i]),
            'or_dm_measure': (i, [vp, i, i, d, C.POINTER(d)]),
            'or_neumaier_sum': (d, [vp, u64]),
            'or_set_threads': (i, [i]),
            'or_sv_multi_unitary': (None, [vp, i, vp, i, vp, i, vp]),
            'or_dm_multi_unitary': (None, [vp, i, vp, i, vp, i, vp]),
            'or_dm_kraus_multi': (None, [vp, i, vp, i, vp, i]),
            'or_init_uniform': (None, [vp, u64, d]),
            'or_dm_init_pure': (None, [vp, i, vp]),
            'or_dm_purity': (d, [vp, i]),
            'or_dm_fidelity_pure': (d, [vp, i, vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        # returns double complex: read back through a 2-double struct
        class _C2(C.Structure):
            _fields_ = [('re', C.c_double), ('im', C.c_double)]
        L.or_sv_inner_product.restype = _C2
        L.or_sv_inner_product.argtypes = [vp, vp, i]
        L.or_sv_amp_after.restype = _C2
        L.or_sv_amp_after.argtypes = [i, vp, vp, i, u64]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags.c_contiguous
    return a.ctypes.data_as(C.c_void_p)


def _ints(xs) -> np.ndarray:
    return np.ascontiguousarray(np.array(list(xs), dtype=np.int32).reshape(-1))


def _mat(u) -> np.ndarray:
    m = np.ascontiguousarray(np.asarray(u, dtype=np.complex128).reshape(4))
    return m


# ---- state vectors ------------------------------------------------------

def zero_state(n: int, index: int = 0) -> np.ndarray:
    a = np.empty(1 << n, dtype=np.complex128)
    lib().or_init_basis(_p(a), a.size, index)
    return a


def sv_unitary(amp, n, controls, target, u):
    c = _ints(controls)
    m = _mat(u)
    lib().or_sv_unitary(_p(amp), n, _p(c), len(c), target, _p(m))


def sv_x(amp, n, controls, target):
    c = _ints(controls)
    lib().or_sv_x(_p(amp), n, _p(c), len(c), target)


def sv_phase(amp, n, qubits, angle):
    q = _ints(qubits)
    lib().or_sv_phase(_p(amp), n, _p(q), len(q), float(angle))


def sv_total_prob(amp, n) -> float:
    return lib().or_sv_total_prob(_p(amp), n)


def sv_prob_outcome(amp, n, q, o) -> float:
    return lib().or_sv_prob_outcome(_p(amp), n, q, o)


def sv_measure(amp, n, q, r):
    p = C.c_double()
    o = lib().or_sv_measure(_p(amp), n, q, float(r), C.byref(p))
    return o, p.value


# ---- density matrices ---------------------------------------------------

def dm_zero(N: int, index: int = 0) -> np.ndarray:
    """|index><index| as the 2N-qubit vector."""
    dim = 1 << N
    return zero_state(2 * N, index + dim * index)


def dm_unitary(rho, N, controls, target, u):
    c = _ints(controls)
    m = _mat(u)
    lib().or_dm_unitary(_p(rho), N, _p(c), len(c), target, _p(m))


def dm_x(rho, N, controls, target):
    c = _ints(controls)
    lib().or_dm_x(_p(rho), N, _p(c), len(c), target)


def dm_phase(rho, N, qubits, angle):
    q = _ints(qubits)
    lib().or_dm_phase(_p(rho), N, _p(q), len(q), float(angle))


def dm_kraus(rho, N, target, kraus_ops):
    k = np.ascontiguousarray(np.asarray(kraus_ops, dtype=np.complex128).reshape(-1))
    lib().or_dm_kraus(_p(rho), N, target, _p(k), k.size // 4)


def dm_dephasing(rho, N, t, p):
    lib().or_dm_dephasing(_p(rho), N, t, float(p))


def dm_depolarising(rho, N, t, p):
    lib().or_dm_depolarising(_p(rho), N, t, float(p))


def dm_damping(rho, N, t, g):
    lib().or_dm_damping(_p(rho), N, t, float(g))


def _matk(u, k) -> np.ndarray:
    d = 1 << k
    m = np.ascontiguousarray(np.asarray(u, dtype=np.complex128).reshape(d * d))
    return m


def sv_multi_unitary(amp, n, controls, targets, u):
    c, t = _ints(controls), _ints(targets)
    m = _matk(u, len(t))
    lib().or_sv_multi_unitary(_p(amp), n, _p(c), len(c), _p(t), len(t), _p(m))


def dm_multi_unitary(rho, N, controls, targets, u):
    c, t = _ints(controls), _ints(targets)
    m = _matk(u, len(t))
    lib().or_dm_multi_unitary(_p(rho), N, _p(c), len(c), _p(t), len(t), _p(m))


def dm_kraus_multi(rho, N, targets, kraus_ops):
    t = _ints(targets)
    d = 1 << len(t)
    k = np.ascontiguousarray(np.asarray(kraus_ops, dtype=np.complex128).reshape(-1))
    lib().or_dm_kraus_multi(_p(rho), N, _p(t), len(t), _p(k), k.size // (d * d))


def uniform_state(nbits: int, value: float) -> np.ndarray:
    a = np.empty(1 << nbits, dtype=np.complex128)
    lib().or_init_uniform(_p(a), a.size, float(value))
    return a


def dm_pure(N, psi) -> np.ndarray:
    psi = np.ascontiguousarray(np.asarray(psi, dtype=np.complex128))
    rho = np.empty(1 << (2 * N), dtype=np.complex128)
    lib().or_dm_init_pure(_p(rho), N, _p(psi))
    return rho


def sv_inner_product(bra, ket, n) -> complex:
    z = lib().or_sv_inner_product(_p(bra), _p(ket), n)
    return complex(z.re, z.im)


def dm_purity(rho, N) -> float:
    return lib().or_dm_purity(_p(rho), N)


def dm_fidelity_pure(rho, N, psi) -> float:
    psi = np.ascontiguousarray(np.asarray(psi, dtype=np.complex128))
    return lib().or_dm_fidelity_pure(_p(rho), N, _p(psi))


def dm_total_prob(rho, N) -> float:
    return lib().or_dm_total_prob(_p(rho), N)


def dm_prob_outcome(rho, N, q, o) -> float:
    return lib().or_dm_prob_outcome(_p(rho), N, q, o)


def dm_measure(rho, N, q, r):
    p = C.c_double()
    o = lib().or_dm_measure(_p(rho), N, q, float(r), C.byref(p))
    return o, p.value


def dm_matrix(rho, N) -> np.ndarray:
    """View the 2N-qubit vector as the 2^N x 2^N matrix rho[j][k]."""
    dim = 1 << N
    return rho.reshape(dim, dim).T  # vector index j + dim*k -> [k][j] in C order


# ---- circuits -----------------------------------------------------------

def apply_sv(amp, n, op):
    if op.kind == 'u':
        sv_unitary(amp, n, op.controls, op.target, op.u)
    elif op.kind == 'x':
        sv_x(amp, n, op.controls, op.target)
    elif op.kind == 'phase':
        sv_phase(amp, n, op.qubits, op.angle)
    elif op.kind == 'unitary':
        sv_multi_unitary(amp, n, op.controls, op.targets, op.u)
    else:
        raise ValueError(f'{op.kind} is not defined on a state vector')


def apply_dm(rho, N, op):
    if op.kind == 'u':
        dm_unitary(rho, N, op.controls, op.target, op.u)
    elif op.kind == 'x':
        dm_x(rho, N, op.controls, op.target)
    elif op.kind == 'phase':
        dm_phase(rho, N, op.qubits, op.angle)
    elif op.kind == 'dephasing':
        dm_dephasing(rho, N, op.target, op.p)
    elif op.kind == 'depolarising':
        dm_depolarising(rho, N, op.target, op.p)
    elif op.kind == 'damping':
        dm_damping(rho, N, op.target, op.p)
    elif op.kind == 'unitary':
        dm_multi_unitary(rho, N, op.controls, op.targets, op.u)
    elif op.kind == 'kraus':
        dm_kraus_multi(rho, N, op.targets, op.kraus)
    else:
        raise ValueError(op.kind)


def run_sv(n, ops, init_index: int = 0) -> np.ndarray:
    amp = zero_state(n, init_index)
    for op in ops:
        apply_sv(amp, n, op)
    return amp


def run_dm(N, ops, init_index: int = 0) -> np.ndarray:
    rho = dm_zero(N, init_index)
    for op in ops:
        apply_dm(rho, N, op)
    return rho


def _gate_records(ops):
    recs = (OrGate * max(1, len(ops)))()
    for k, op in enumerate(ops):
        g = recs[k]
        if op.kind == 'u':
            g.kind = OR_U
            m = np.asarray(op.u, dtype=np.complex128).reshape(4)
            for e in range(4):
                g.u[2 * e] = m[e].real
                g.u[2 * e + 1] = m[e].imag
        elif op.kind == 'x':
            g.kind = OR_X
        elif op.kind == 'phase':
            g.kind = OR_PHASE
            g.angle = op.angle
        else:
            raise ValueError(op.kind)
        g.target = op.target if op.kind != 'phase' else -1
        qs = op.qubits if op.kind == 'phase' else op.controls
        m = 0
        for q in qs:
            m |= 1 << q
        g.mask = m
    return recs


def amps_after(n, product_vectors, ops, indices) -> np.ndarray:
    """Output amplitudes at ``indices`` of (x)_q v_q followed by ``ops``.

    ``product_vectors`` is (n, 2): row q is the single-qubit state of qubit q.
    Each output element is evaluated on its own from Eq. 1."""
    v = np.ascontiguousarray(np.asarray(product_vectors, dtype=np.complex128).reshape(-1))
    recs = _gate_records(ops)
    out = np.empty(len(indices), dtype=np.complex128)
    L = lib()
    for k, i in enumerate(indices):
        r = L.or_sv_amp_after(n, _p(v), C.cast(recs, C.c_void_p), len(ops), int(i))
        out[k] = complex(r.re, r.im)
    return out


def neumaier_sum(x) -> float:
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    return lib().or_neumaier_sum(_p(a), a.size)


def set_threads(n: int) -> int:
    """Thread count of the oracle's OpenMP loops (timing only); returns the
    previous count."""
    return lib().or_set_threads(int(n))
