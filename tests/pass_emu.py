"""Runs generated fused-pass kernels on the CPU (test infrastructure).

A generated pass is plain HIP C++ apart from a few device constructs.  This
module compiles its source with the host clang++ under a small shim (one OS
thread per GPU thread, a pthread barrier for the workgroup barrier, the LDS
array shared by the threads of the one workgroup that runs at a time, a
barrier per 64 threads for the wave-level ordering) and
runs the workgroups one after another.  That executes exactly the
arithmetic, register renames, LDS re-layouts and HBM addressing the
generator wrote, so a pass set can be checked against the oracle without a
GPU.  Timing, occupancy and memory ordering across workgroups are not
modelled (workgroups of one pass touch disjoint amplitudes).
"""
from __future__ import annotations

import ctypes as C
import hashlib
import os
import re
import subprocess
import tempfile

import numpy as np

CLANG = os.environ.get('QS_EMU_CXX', '/opt/rocm/llvm/bin/clang++')

_HEAD = r'''
#include <pthread.h>
#include <thread>
#include <vector>
struct double2 { double x, y; };
struct float2 { float x, y; };
struct QsEmuDim { unsigned x; };
static thread_local QsEmuDim threadIdx, blockIdx;
static QsEmuDim gridDim;
static pthread_barrier_t qs_emu_bar;
static inline void qs_emu_barrier() { pthread_barrier_wait(&qs_emu_bar); }
// wave-level ordering: the 64 threads of one wave wait for each other only
static pthread_barrier_t qs_emu_wbar[16];
static inline void qs_emu_wave_barrier() { pthread_barrier_wait(&qs_emu_wbar[threadIdx.x / 64]); }
#define __global__
#define __device__
#define __forceinline__ inline
#define __launch_bounds__(x)
#define __shared__ static
#define __builtin_amdgcn_s_waitcnt(x) ((void)0)
#define __builtin_amdgcn_readfirstlane(x) (x)
'''

_TAIL = r'''
extern "C" int qs_emu_run(V* amp, const R* mats, unsigned long long ntiles, unsigned grid, unsigned nthreads,
                          double* part)
{
    if (grid == 0 || grid > ntiles) return 1;
    gridDim.x = grid;
    pthread_barrier_init(&qs_emu_bar, nullptr, nthreads);
    for (unsigned w = 0; w * 64 < nthreads; ++w) pthread_barrier_init(&qs_emu_wbar[w], nullptr, nthreads < 64 ? nthreads : 64);
    for (unsigned b = 0; b < grid; ++b) {
        std::vector<std::thread> th;
        for (unsigned t = 0; t < nthreads; ++t)
            th.emplace_back([=] {
                threadIdx.x = t;
                blockIdx.x = b;
                qs_pass(amp, mats, ntiles QS_EMU_PART);
            });
        for (std::thread& x : th) x.join();
    }
    pthread_barrier_destroy(&qs_emu_bar);
    for (unsigned w = 0; w * 64 < nthreads; ++w) pthread_barrier_destroy(&qs_emu_wbar[w]);
    return 0;
}
'''

_CACHE = os.path.join(tempfile.gettempdir(), 'qs_pass_emu')


def available() -> bool:
    return os.path.exists(CLANG)


def compile_pass(src: str):
    """Build one generated pass as a host shared library (cached by source)."""
    body = re.sub(r'^#define QS_BAR\(\).*$', '#define QS_BAR() qs_emu_barrier()', src, flags=re.M)
    body = re.sub(r'^#define QS_WBAR\(\).*$', '#define QS_WBAR() qs_emu_wave_barrier()', body, flags=re.M)
    if 'qs_emu_barrier()' not in body and 'QS_BAR' in src:
        raise RuntimeError('pass source has no QS_BAR definition to replace')
    # register-class hints (an empty asm pinning a value to scalar registers)
    body = re.sub(r'asm\(""\s*:\s*"\+s"\((\w+)\)\);', '', body)
    if re.search(r'\basm\b', body):
        raise RuntimeError('pass source holds inline asm the emulator does not model')
    # the last pass in its readout form takes the per-workgroup sums buffer
    part = 'double* __restrict__ part)' in body
    full = _HEAD + ('#define QS_EMU_PART , part\n' if part else '#define QS_EMU_PART\n') + body + _TAIL
    key = hashlib.sha1(full.encode()).hexdigest()[:20]
    os.makedirs(_CACHE, exist_ok=True)
    so = os.path.join(_CACHE, key + '.so')
    if not os.path.exists(so):
        cpp = os.path.join(_CACHE, key + '.cpp')
        with open(cpp, 'w') as f:
            f.write(full)
        tmp = so + f'.tmp{os.getpid()}'
        r = subprocess.run([CLANG, '-O1', '-std=c++17', '-shared', '-fPIC', '-pthread', '-w', cpp, '-o', tmp],
                           capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f'emulator compile failed:\n{r.stderr[-4000:]}')
        os.replace(tmp, so)
    lib = C.CDLL(so)
    lib.qs_emu_run.restype = C.c_int
    lib.qs_emu_run.argtypes = [C.c_void_p, C.c_void_p, C.c_ulonglong, C.c_uint, C.c_uint, C.c_void_p]
    return lib


def run_passes(circuit, amp: np.ndarray, nbits: int, prec: int, tile_qubits: int, thread_bits: int,
               contig: int, kind: int, grid_div: int = 1, readout: bool = False):
    """Apply every generated pass of `circuit` to `amp` (complex128 for
    QS_C128, complex64 for QS_C64; 2^nbits entries) in place.  Each pass runs
    on ntiles / grid_div workgroups, so grid_div > 1 exercises the tile loop
    and its prefetch.  For a density matrix pass nbits = 2N and kind =
    DENSITY; `circuit.source` / `pass_data` take N.  Returns the pass count;
    with readout (state vectors) the last pass runs in its readout form and
    (pass count, per-workgroup sums of shape (grid, nbits + 1)) is returned."""
    from paper_1802_08032_amd import qstate as Q
    n_arg = nbits // 2 if kind == Q.DENSITY else nbits
    _, npass = circuit.source(n_arg, prec, tile_qubits, thread_bits, 0, 0, contig, kind=kind)
    ntiles = 1 << (nbits - tile_qubits)
    grid = max(1, ntiles // grid_div)
    assert amp.flags.c_contiguous and amp.size == 1 << nbits
    assert amp.dtype == (np.complex128 if prec == Q.C128 else np.complex64)
    part = np.full((grid, nbits + 1), np.nan)
    for p in range(npass):
        ro = readout and p == npass - 1
        src, _ = circuit.source(n_arg, prec, tile_qubits, thread_bits, -1 if ro else p, 0, contig, kind=kind)
        mats = circuit.pass_data(n_arg, prec, tile_qubits, thread_bits, p, 0, contig, kind=kind)
        m = np.ascontiguousarray(mats if prec == Q.C128 else mats.astype(np.float32))
        if m.size == 0:
            m = np.zeros(1, dtype=m.dtype)
        lib = compile_pass(src)
        rc = lib.qs_emu_run(amp.ctypes.data, m.ctypes.data, ntiles, grid, 1 << thread_bits,
                            part.ctypes.data if ro else None)
        if rc:
            raise RuntimeError('emulated launch rejected its grid')
    return (npass, part) if readout else npass
