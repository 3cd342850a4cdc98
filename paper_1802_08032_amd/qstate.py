"""Thin Python binding over the qstate C ABI (include/qstate.h).

Argument marshalling only: every operation runs in the HIP kernels of
libqstate.so.  PyTorch provides device memory (registers wrap a torch
tensor) and the HIP stream (the current torch stream); it is imported
before the library so that both share one HIP runtime.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library binds to)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, 'libqstate.so')

STATEVEC, DENSITY = 0, 1
C64, C128 = 1, 2
DEPHASING, DEPOLARISING, DAMPING = 0, 1, 2
K_INIT, K_GATE, K_GATE_LOW, K_NOT, K_PHASE, K_DM_GATE, K_DM_CHANNEL, K_REDUCE, K_COLLAPSE, K_FUSED = range(10)
KERNEL_CLASSES = ['init', 'gate', 'gate_low', 'not', 'phase', 'dm_gate', 'dm_channel', 'reduce',
                  'collapse', 'fused']

_STATUS = {0: 'QS_OK', -1: 'QS_E_ARG', -2: 'QS_E_KIND', -3: 'QS_E_OOM', -4: 'QS_E_DEVICE',
           -5: 'QS_E_HANDLE', -6: 'QS_E_NOT_UNITARY', -7: 'QS_E_NOT_CPTP'}


class QStateError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f'{_STATUS.get(status, status)}: {message}')
        self.status = status
        self.name = _STATUS.get(status, str(status))


class Cplx(C.Structure):
    _fields_ = [('re', C.c_double), ('im', C.c_double)]


_lib = None

# name -> (restype, argtypes); every qs_status function returns c_int
_vp, _i, _d, _u64, _sz = C.c_void_p, C.c_int, C.c_double, C.c_uint64, C.c_size_t
_PI, _PD, _PU64 = C.POINTER(C.c_int), C.POINTER(C.c_double), C.POINTER(C.c_uint64)
SIGNATURES = {
    'qs_env_create': (_i, [_i, C.POINTER(_vp)]),
    'qs_env_destroy': (_i, [_vp]),
    'qs_env_sync': (_i, [_vp]),
    'qs_last_error': (C.c_char_p, []),
    'qs_profile_enable': (_i, [_vp, _i]),
    'qs_profile_read': (_i, [_vp, _i, _PU64, _PD]),
    'qs_profile_reset': (_i, [_vp]),
    'qs_reg_bytes': (_sz, [_i, _i, _i]),
    'qs_reg_create': (_i, [_vp, _i, _i, _i, _vp, C.POINTER(_vp)]),
    'qs_reg_wrap': (_i, [_vp, _i, _i, _i, _vp, _sz, _vp, C.POINTER(_vp)]),
    'qs_reg_destroy': (_i, [_vp]),
    'qs_reg_info': (_i, [_vp, _PI, _PI, _PI, C.POINTER(_vp), C.POINTER(_vp)]),
    'qs_init_zero': (_i, [_vp]),
    'qs_init_basis': (_i, [_vp, _u64]),
    'qs_get_amps': (_i, [_vp, _u64, _u64, _vp]),
    'qs_set_amps': (_i, [_vp, _u64, _u64, _vp]),
    'qs_unitary': (_i, [_vp, _i, _vp]),
    'qs_controlled_unitary': (_i, [_vp, _i, _i, _vp]),
    'qs_multi_controlled_unitary': (_i, [_vp, _vp, _i, _i, _vp]),
    'qs_multi_controlled_not': (_i, [_vp, _vp, _i, _i]),
    'qs_multi_controlled_phase': (_i, [_vp, _vp, _i, _d]),
    'qs_mix_dephasing': (_i, [_vp, _i, _d]),
    'qs_mix_depolarising': (_i, [_vp, _i, _d]),
    'qs_mix_damping': (_i, [_vp, _i, _d]),
    'qs_calc_total_prob': (_i, [_vp, _PD]),
    'qs_calc_prob_of_outcome': (_i, [_vp, _i, _i, _PD]),
    'qs_measure': (_i, [_vp, _i, _d, _PI, _PD]),
    'qs_measure_given_probs': (_i, [_vp, _i, _d, _d, _d, _PI, _PD]),
    'qs_measure_all': (_i, [_vp, _PD, _PI, _PD]),
    'qs_circuit_set_unitary': (_i, [_vp, _i, _vp]),
    'qs_circuit_set_phase': (_i, [_vp, _i, _d]),
    'qs_batch_update': (_i, [_vp]),
    'qs_hadamard': (_i, [_vp, _i]),
    'qs_cnot': (_i, [_vp, _i, _i]),
    'qs_cz': (_i, [_vp, _i, _i]),
    'qs_rotate_x': (_i, [_vp, _i, _d]),
    'qs_rotate_y': (_i, [_vp, _i, _d]),
    'qs_rotate_z': (_i, [_vp, _i, _d]),
    'qs_t_gate': (_i, [_vp, _i]),
    'qs_sqrt_x': (_i, [_vp, _i]),
    'qs_sqrt_y': (_i, [_vp, _i]),
    'qs_philox_draws': (_i, [_u64, _u64, _u64, _i, _PD]),
    'qs_env_seed': (_i, [_vp, _u64, _u64]),
    'qs_measure_seeded': (_i, [_vp, _i, _PI, _PD]),
    'qs_measure_all_seeded': (_i, [_vp, _PI, _PD]),
    'qs_circuit_create': (_i, [C.POINTER(_vp)]),
    'qs_circuit_destroy': (_i, [_vp]),
    'qs_circuit_add_unitary': (_i, [_vp, _vp, _i, _i, _vp]),
    'qs_circuit_add_not': (_i, [_vp, _vp, _i, _i]),
    'qs_circuit_add_two_qubit_unitary': (_i, [_vp, _i, _i, _vp]),
    'qs_circuit_add_phase': (_i, [_vp, _vp, _i, _d]),
    'qs_circuit_add_channel': (_i, [_vp, _i, _i, _d]),
    'qs_circuit_size': (_i, [_vp, _PI]),
    'qs_circuit_run': (_i, [_vp, _vp, _i, _PI]),
    'qs_circuit_run_tiled': (_i, [_vp, _vp, _i, _i, _i, _PI]),
    'qs_circuit_run_compiled': (_i, [_vp, _vp, _i, _i, _i, _i, _PI]),
    'qs_circuit_run_compiled_from_basis': (_i, [_vp, _vp, _i, _i, _i, _i, _u64, _PI]),
    'qs_circuit_run_compiled_probs': (_i, [_vp, _vp, _i, _i, _i, _i, _vp, _PD, _PI]),
    'qs_circuit_source': (_i, [_vp, _i, _i, _i, _i, _i, _i, _i, _i, C.c_char_p, _sz, C.POINTER(_sz), _PI]),
    'qs_circuit_pass_data': (_i, [_vp, _i, _i, _i, _i, _i, _i, _i, _i, _PD, _sz, C.POINTER(_sz), _PI]),
    'qs_batch_create': (_i, [_vp, _vp, _i, _i, C.POINTER(_vp)]),
    'qs_batch_destroy': (_i, [_vp]),
    'qs_batch_run': (_i, [_vp, _i]),
    'qs_batch_capture': (_i, [_vp, _i]),
    'qs_batch_replay': (_i, [_vp]),
    'qs_batch_probs': (_i, [_vp, _i, _vp, _vp]),
    'qs_batch_info': (_i, [_vp, _PI, _PI, _PI]),
    'qs_multi_qubit_unitary': (_i, [_vp, _vp, _i, _vp, _i, _vp]),
    'qs_two_qubit_unitary': (_i, [_vp, _i, _i, _vp]),
    'qs_mix_multi_kraus': (_i, [_vp, _vp, _i, _vp, _i]),
    'qs_mix_kraus': (_i, [_vp, _i, _vp, _i]),
    'qs_mix_two_qubit_kraus': (_i, [_vp, _i, _i, _vp, _i]),
    'qs_init_plus': (_i, [_vp]),
    'qs_init_pure_state': (_i, [_vp, _vp]),
    'qs_clone': (_i, [_vp, _vp]),
    'qs_calc_inner_product': (_i, [_vp, _vp, _vp]),
    'qs_calc_purity': (_i, [_vp, _PD]),
    'qs_calc_fidelity': (_i, [_vp, _vp, _PD]),
    'qs_save_state': (_i, [_vp, C.c_char_p]),
    'qs_load_state': (_i, [_vp, C.c_char_p]),
    'qs_prob_noalloc': (_i, [_i, _vp, _i, _i, _i, _i, _vp, _vp]),
}


def lib():
    """Load libqstate.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f'{LIB_PATH} is missing: build it with '
                              f'`python -m paper_1802_08032_amd.build`')
        L = C.CDLL(LIB_PATH, mode=C.RTLD_GLOBAL)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != 0:
        raise QStateError(status, lib().qs_last_error().decode())


def _ints(xs):
    xs = [int(x) for x in xs]
    arr = (C.c_int * max(1, len(xs)))(*xs)
    return arr, len(xs)


def _mat(u):
    m = np.asarray(u, dtype=np.complex128).reshape(4)
    return (Cplx * 4)(*[Cplx(float(z.real), float(z.imag)) for z in m])


def _cplx_array(a):
    """Contiguous complex128 copy of `a` (passed as qs_cplx[]) and its size."""
    m = np.ascontiguousarray(np.asarray(a, dtype=np.complex128).reshape(-1))
    return m, m.size


def philox_draws(seed: int, stream: int, first: int, count: int) -> np.ndarray:
    """Draws first .. first + count - 1 of the library's Philox4x64-10 stream
    (seed, stream), as doubles in [0, 1)."""
    out = np.empty(max(count, 0), dtype=np.float64)  # the library rejects a negative count
    _check(lib().qs_philox_draws(seed & (2**64 - 1), stream & (2**64 - 1), first, count, out.ctypes.data_as(_PD)))
    return out


def prob_noalloc(device: int, dev_amps: int, n: int, kind: int, prec: int, qubit: int, dev_out: int,
                 stream: int = 0):
    """qs_prob_noalloc: the probability reduction over caller-owned device
    amplitudes, two doubles written to the device address dev_out; allocates
    nothing (include/qstate_noalloc.h)."""
    _check(lib().qs_prob_noalloc(device, C.c_void_p(dev_amps), n, kind, prec, qubit, C.c_void_p(dev_out),
                                 C.c_void_p(stream)))


def reg_bytes(n: int, kind: int = STATEVEC, prec: int = C128) -> int:
    return lib().qs_reg_bytes(n, kind, prec)


class Env:
    """A device (createQuESTEnv)."""

    def __init__(self, device: int = 0):
        h = C.c_void_p()
        _check(lib().qs_env_create(device, C.byref(h)))
        self.h = h
        self.device = device

    def sync(self):
        _check(lib().qs_env_sync(self.h))

    def seed(self, seed: int, stream: int = 0):
        """Measurement draw stream (seed, stream) for the *_seeded calls,
        rewound to its first draw."""
        _check(lib().qs_env_seed(self.h, seed & (2**64 - 1), stream & (2**64 - 1)))

    def profile(self, enable: bool = True):
        _check(lib().qs_profile_enable(self.h, int(enable)))

    def profile_read(self, klass: int):
        n, ms = C.c_uint64(), C.c_double()
        _check(lib().qs_profile_read(self.h, klass, C.byref(n), C.byref(ms)))
        return n.value, ms.value

    def profile_reset(self):
        _check(lib().qs_profile_reset(self.h))

    def close(self):
        if self.h:
            _check(lib().qs_env_destroy(self.h))
            self.h = None


class Register:
    """A register of n qubits (state vector or density matrix).

    By default the amplitudes live in a torch tensor on this device (wrapped
    through qs_reg_wrap) and work is issued on the current torch stream;
    ``owned=True`` lets the library allocate instead."""

    def __init__(self, env: Env, n: int, kind: int = STATEVEC, prec: int = C128,
                 owned: bool = False, stream=None):
        self.env, self.n, self.kind, self.prec = env, n, kind, prec
        nbits = 2 * n if kind == DENSITY else n
        self.nbits = nbits
        if stream is None:
            stream = torch.cuda.current_stream(env.device)
        self.stream = stream
        sptr = C.c_void_p(stream.cuda_stream)
        h = C.c_void_p()
        self.tensor = None
        if owned:
            _check(lib().qs_reg_create(env.h, n, kind, prec, sptr, C.byref(h)))
        else:
            nbytes = reg_bytes(n, kind, prec)
            if nbytes == 0:
                raise QStateError(-1, 'invalid qubit count, kind or precision')
            dt = torch.complex128 if prec == C128 else torch.complex64
            self.tensor = torch.empty(1 << nbits, dtype=dt, device=f'cuda:{env.device}')
            _check(lib().qs_reg_wrap(env.h, n, kind, prec, C.c_void_p(self.tensor.data_ptr()),
                                     nbytes, sptr, C.byref(h)))
        self.h = h

    # -- lifecycle --------------------------------------------------------
    def close(self):
        if self.h:
            _check(lib().qs_reg_destroy(self.h))
            self.h = None
            self.tensor = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- state --------------------------------------------------------------
    def init_zero(self):
        _check(lib().qs_init_zero(self.h))

    def init_basis(self, index: int):
        _check(lib().qs_init_basis(self.h, index))

    def get_amps(self, start: int = 0, count: int | None = None) -> np.ndarray:
        if count is None:
            count = (1 << self.nbits) - start
        out = np.empty(count, dtype=np.complex128)
        _check(lib().qs_get_amps(self.h, start, count, out.ctypes.data_as(C.c_void_p)))
        return out

    def set_amps(self, amps, start: int = 0):
        a = np.ascontiguousarray(np.asarray(amps, dtype=np.complex128))
        _check(lib().qs_set_amps(self.h, start, a.size, a.ctypes.data_as(C.c_void_p)))

    # -- gates --------------------------------------------------------------
    def unitary(self, target: int, u):
        _check(lib().qs_unitary(self.h, target, _mat(u)))

    def controlled_unitary(self, control: int, target: int, u):
        _check(lib().qs_controlled_unitary(self.h, control, target, _mat(u)))

    def multi_controlled_unitary(self, controls, target: int, u):
        arr, k = _ints(controls)
        _check(lib().qs_multi_controlled_unitary(self.h, arr, k, target, _mat(u)))

    def multi_controlled_not(self, controls, target: int):
        arr, k = _ints(controls)
        _check(lib().qs_multi_controlled_not(self.h, arr, k, target))

    def multi_controlled_phase(self, qubits, angle: float):
        arr, k = _ints(qubits)
        _check(lib().qs_multi_controlled_phase(self.h, arr, k, float(angle)))

    def hadamard(self, target: int):
        _check(lib().qs_hadamard(self.h, target))

    def cnot(self, control: int, target: int):
        _check(lib().qs_cnot(self.h, control, target))

    def cz(self, q1: int, q2: int):
        _check(lib().qs_cz(self.h, q1, q2))

    def rotate_x(self, target: int, theta: float):
        _check(lib().qs_rotate_x(self.h, target, float(theta)))

    def rotate_y(self, target: int, theta: float):
        _check(lib().qs_rotate_y(self.h, target, float(theta)))

    def rotate_z(self, target: int, theta: float):
        _check(lib().qs_rotate_z(self.h, target, float(theta)))

    def t_gate(self, target: int):
        _check(lib().qs_t_gate(self.h, target))

    def sqrt_x(self, target: int):
        _check(lib().qs_sqrt_x(self.h, target))

    def sqrt_y(self, target: int):
        _check(lib().qs_sqrt_y(self.h, target))

    def mix_dephasing(self, target: int, p: float):
        _check(lib().qs_mix_dephasing(self.h, target, float(p)))

    def mix_depolarising(self, target: int, p: float):
        _check(lib().qs_mix_depolarising(self.h, target, float(p)))

    def mix_damping(self, target: int, gamma: float):
        _check(lib().qs_mix_damping(self.h, target, float(gamma)))

    def multi_qubit_unitary(self, targets, u, controls=()):
        """Dense 2^k x 2^k unitary on targets (matrix index bit j <->
        targets[j]), where every control is 1."""
        t, k = _ints(targets)
        c, nc = _ints(controls)
        m, _ = _cplx_array(u)
        _check(lib().qs_multi_qubit_unitary(self.h, c, nc, t, k, m.ctypes.data_as(C.c_void_p)))

    def two_qubit_unitary(self, target1: int, target2: int, u):
        m, _ = _cplx_array(u)
        _check(lib().qs_two_qubit_unitary(self.h, target1, target2, m.ctypes.data_as(C.c_void_p)))

    def mix_multi_kraus(self, targets, ops):
        """Kraus map sum_m K rho K^dagger on 1 or 2 targets; ops: (m, d, d)."""
        t, k = _ints(targets)
        m, size = _cplx_array(ops)
        d = 1 << k
        _check(lib().qs_mix_multi_kraus(self.h, t, k, m.ctypes.data_as(C.c_void_p), size // (d * d)))

    def mix_kraus(self, target: int, ops):
        m, size = _cplx_array(ops)
        _check(lib().qs_mix_kraus(self.h, target, m.ctypes.data_as(C.c_void_p), size // 4))

    def mix_two_qubit_kraus(self, target1: int, target2: int, ops):
        m, size = _cplx_array(ops)
        _check(lib().qs_mix_two_qubit_kraus(self.h, target1, target2, m.ctypes.data_as(C.c_void_p), size // 16))

    def init_plus(self):
        _check(lib().qs_init_plus(self.h))

    def init_pure_state(self, pure: 'Register'):
        _check(lib().qs_init_pure_state(self.h, pure.h))

    def clone_from(self, src: 'Register'):
        _check(lib().qs_clone(self.h, src.h))

    def calc_inner_product(self, ket: 'Register') -> complex:
        """<self|ket>."""
        out = (Cplx * 1)()
        _check(lib().qs_calc_inner_product(self.h, ket.h, out))
        return complex(out[0].re, out[0].im)

    def calc_purity(self) -> float:
        v = C.c_double()
        _check(lib().qs_calc_purity(self.h, C.byref(v)))
        return v.value

    def calc_fidelity(self, pure: 'Register') -> float:
        v = C.c_double()
        _check(lib().qs_calc_fidelity(self.h, pure.h, C.byref(v)))
        return v.value

    def save_state(self, path: str):
        _check(lib().qs_save_state(self.h, os.fsencode(path)))

    def load_state(self, path: str):
        _check(lib().qs_load_state(self.h, os.fsencode(path)))

    def apply(self, op):
        """Apply one workloads.Op."""
        if op.kind == 'u':
            self.multi_controlled_unitary(op.controls, op.target, op.u)
        elif op.kind == 'x':
            self.multi_controlled_not(op.controls, op.target)
        elif op.kind == 'phase':
            self.multi_controlled_phase(op.qubits, op.angle)
        elif op.kind == 'dephasing':
            self.mix_dephasing(op.target, op.p)
        elif op.kind == 'depolarising':
            self.mix_depolarising(op.target, op.p)
        elif op.kind == 'damping':
            self.mix_damping(op.target, op.p)
        elif op.kind == 'unitary':
            self.multi_qubit_unitary(op.targets, op.u, op.controls)
        elif op.kind == 'kraus':
            self.mix_multi_kraus(op.targets, np.stack(op.kraus))
        else:
            raise ValueError(op.kind)

    # -- probabilities --------------------------------------------------------
    def calc_total_prob(self) -> float:
        v = C.c_double()
        _check(lib().qs_calc_total_prob(self.h, C.byref(v)))
        return v.value

    def calc_prob_of_outcome(self, qubit: int, outcome: int) -> float:
        v = C.c_double()
        _check(lib().qs_calc_prob_of_outcome(self.h, qubit, outcome, C.byref(v)))
        return v.value

    def measure(self, qubit: int, u01: float):
        o, p = C.c_int(), C.c_double()
        _check(lib().qs_measure(self.h, qubit, float(u01), C.byref(o), C.byref(p)))
        return o.value, p.value

    def measure_given_probs(self, qubit: int, p0: float, p1: float, u01: float):
        """measure() with P(0) and P(1) supplied (e.g. from
        Circuit.run_compiled_probs) instead of summed from the state."""
        o, p = C.c_int(), C.c_double()
        _check(lib().qs_measure_given_probs(self.h, qubit, float(p0), float(p1), float(u01), C.byref(o),
                                            C.byref(p)))
        return o.value, p.value

    def measure_all(self, draws):
        """Measure qubits 0..n-1 in order with one draw each; returns
        (outcomes, probabilities) as lists."""
        d = np.ascontiguousarray(np.asarray(draws, dtype=np.float64)[:self.n])
        if d.size != self.n:
            raise ValueError(f'need {self.n} draws, got {d.size}')
        o = (C.c_int * self.n)()
        p = (C.c_double * self.n)()
        _check(lib().qs_measure_all(self.h, d.ctypes.data_as(_PD), o, p))
        return list(o), list(p)

    def measure_seeded(self, qubit: int):
        """qs_measure with the next draw of the environment's stream."""
        o, p = C.c_int(), C.c_double()
        _check(lib().qs_measure_seeded(self.h, qubit, C.byref(o), C.byref(p)))
        return o.value, p.value

    def measure_all_seeded(self):
        """qs_measure_all with the environment stream's next n draws."""
        o = (C.c_int * self.n)()
        p = (C.c_double * self.n)()
        _check(lib().qs_measure_all_seeded(self.h, o, p))
        return list(o), list(p)


class Circuit:
    """A recorded operation list, run with or without gate fusion."""

    def __init__(self, ops=None):
        h = C.c_void_p()
        _check(lib().qs_circuit_create(C.byref(h)))
        self.h = h
        for op in ops or []:
            self.add(op)

    def set_unitary(self, index: int, u):
        """New matrix for recorded unitary op `index` (kind and qubits kept)."""
        _check(lib().qs_circuit_set_unitary(self.h, index, _mat(u)))

    def set_phase(self, index: int, angle: float):
        """New angle for recorded phase op `index`."""
        _check(lib().qs_circuit_set_phase(self.h, index, float(angle)))

    def add(self, op):
        L = lib()
        if op.kind == 'u':
            arr, k = _ints(op.controls)
            _check(L.qs_circuit_add_unitary(self.h, arr, k, op.target, _mat(op.u)))
        elif op.kind == 'x':
            arr, k = _ints(op.controls)
            _check(L.qs_circuit_add_not(self.h, arr, k, op.target))
        elif op.kind == 'phase':
            arr, k = _ints(op.qubits)
            _check(L.qs_circuit_add_phase(self.h, arr, k, float(op.angle)))
        elif op.kind == 'unitary' and len(op.targets) == 1:
            arr, k = _ints(op.controls)
            _check(L.qs_circuit_add_unitary(self.h, arr, k, op.targets[0], _mat(op.u)))
        elif op.kind == 'unitary' and len(op.targets) == 2 and not op.controls:
            m, _ = _cplx_array(op.u)
            if m.size != 16:
                raise ValueError('a two-qubit unitary is 4x4')
            _check(L.qs_circuit_add_two_qubit_unitary(self.h, op.targets[0], op.targets[1],
                                                      C.c_void_p(m.ctypes.data)))
        elif op.kind == 'unitary':
            raise ValueError('circuits hold unitaries on one qubit (any controls) or on two qubits '
                             '(no controls); apply wider ones to a register directly')
        else:
            ch = {'dephasing': DEPHASING, 'depolarising': DEPOLARISING, 'damping': DAMPING}[op.kind]
            _check(L.qs_circuit_add_channel(self.h, ch, op.target, float(op.p)))

    def __len__(self):
        n = C.c_int()
        _check(lib().qs_circuit_size(self.h, C.byref(n)))
        return n.value

    def run(self, reg: Register, fusion_qubits: int = 0) -> int:
        passes = C.c_int()
        _check(lib().qs_circuit_run(reg.h, self.h, fusion_qubits, C.byref(passes)))
        return passes.value

    def run_tiled(self, reg: Register, tile_qubits: int, thread_bits: int, max_phases: int = 0) -> int:
        passes = C.c_int()
        _check(lib().qs_circuit_run_tiled(reg.h, self.h, tile_qubits, thread_bits, max_phases,
                                          C.byref(passes)))
        return passes.value

    def run_compiled(self, reg: Register, tile_qubits: int, thread_bits: int, max_phases: int = 0,
                     contig_qubits: int = 0, init_basis: int | None = None) -> int:
        """Run-time compiled fused passes; with init_basis, the register
        first becomes |init_basis> inside the first pass."""
        passes = C.c_int()
        if init_basis is None:
            _check(lib().qs_circuit_run_compiled(reg.h, self.h, tile_qubits, thread_bits, max_phases,
                                                 contig_qubits, C.byref(passes)))
        else:
            _check(lib().qs_circuit_run_compiled_from_basis(reg.h, self.h, tile_qubits, thread_bits, max_phases,
                                                            contig_qubits, init_basis, C.byref(passes)))
        return passes.value

    def run_compiled_probs(self, reg: Register, tile_qubits: int, thread_bits: int, max_phases: int = 0,
                           contig_qubits: int = 0, init_basis: int | None = None):
        """run_compiled whose last pass also sums the readouts: returns
        (passes, probs) with probs[0] the total probability and probs[1 + q]
        = P(qubit q = 0), as a float64 array of n + 1."""
        passes = C.c_int()
        out = np.zeros(reg.n + 1, dtype=np.float64)
        idx = C.c_uint64(init_basis) if init_basis is not None else None
        _check(lib().qs_circuit_run_compiled_probs(reg.h, self.h, tile_qubits, thread_bits, max_phases,
                                                   contig_qubits, C.byref(idx) if idx is not None else None,
                                                   out.ctypes.data_as(_PD), C.byref(passes)))
        return passes.value, out

    def source(self, n: int, prec: int, tile_qubits: int, thread_bits: int, pass_index: int = 0,
               max_phases: int = 0, contig_qubits: int = 0, kind: int = STATEVEC):
        """(generated HIP source of one pass, number of passes); host only."""
        ln, npass = C.c_size_t(), C.c_int()
        _check(lib().qs_circuit_source(self.h, n, kind, prec, tile_qubits, thread_bits, max_phases,
                                       contig_qubits, pass_index, None, 0, C.byref(ln), C.byref(npass)))
        buf = C.create_string_buffer(ln.value + 1)
        _check(lib().qs_circuit_source(self.h, n, kind, prec, tile_qubits, thread_bits, max_phases,
                                       contig_qubits, pass_index, buf, ln.value + 1, C.byref(ln), C.byref(npass)))
        return buf.value.decode(), npass.value

    def pass_data(self, n: int, prec: int, tile_qubits: int, thread_bits: int, pass_index: int = 0,
                  max_phases: int = 0, contig_qubits: int = 0, kind: int = STATEVEC):
        """Kernel data (float64 numpy array) that `source(...)`'s pass reads
        through its `mats` argument; host only."""
        import numpy as np
        ln, npass = C.c_size_t(), C.c_int()
        _check(lib().qs_circuit_pass_data(self.h, n, kind, prec, tile_qubits, thread_bits, max_phases,
                                          contig_qubits, pass_index, None, 0, C.byref(ln), C.byref(npass)))
        out = np.zeros(max(1, ln.value), dtype=np.float64)
        _check(lib().qs_circuit_pass_data(self.h, n, kind, prec, tile_qubits, thread_bits, max_phases,
                                          contig_qubits, pass_index,
                                          out.ctypes.data_as(C.POINTER(C.c_double)), ln.value,
                                          C.byref(ln), C.byref(npass)))
        return out[:ln.value]

    def close(self):
        if self.h:
            _check(lib().qs_circuit_destroy(self.h))
            self.h = None


class Batch:
    """Many state-vector registers, each with its own circuit, run by one
    persistent launch (optionally replayed from a captured HIP graph)."""

    def __init__(self, regs, circuits, tile_qubits: int = 10):
        if len(regs) != len(circuits) or not regs:
            raise ValueError('one circuit per register')
        rh = (C.c_void_p * len(regs))(*[r.h.value for r in regs])
        ch = (C.c_void_p * len(circuits))(*[c.h.value for c in circuits])
        h = C.c_void_p()
        _check(lib().qs_batch_create(rh, ch, len(regs), tile_qubits, C.byref(h)))
        self.h = h
        self.regs = list(regs)
        self.circuits = list(circuits)

    def run(self, init_zero: bool = True):
        _check(lib().qs_batch_run(self.h, int(init_zero)))

    def capture(self, init_zero: bool = True):
        _check(lib().qs_batch_capture(self.h, int(init_zero)))

    def replay(self):
        _check(lib().qs_batch_replay(self.h))

    def update(self):
        """Take the circuits' current parameters into the batch (and into a
        captured graph's next replay)."""
        _check(lib().qs_batch_update(self.h))

    def probs(self, qubit: int = 0):
        """(P(qubit = 0), total probability) per register, as numpy arrays."""
        n = len(self.regs)
        p0 = np.empty(n)
        tot = np.empty(n)
        _check(lib().qs_batch_probs(self.h, qubit, p0.ctypes.data_as(C.c_void_p), tot.ctypes.data_as(C.c_void_p)))
        return p0, tot

    def info(self):
        a, b, c = C.c_int(), C.c_int(), C.c_int()
        _check(lib().qs_batch_info(self.h, C.byref(a), C.byref(b), C.byref(c)))
        return {'registers': a.value, 'tile_qubits': b.value, 'passes': c.value}

    def close(self):
        if self.h:
            _check(lib().qs_batch_destroy(self.h))
            self.h = None
