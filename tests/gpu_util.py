"""Helpers for the GPU parity tests: run workloads through the C ABI (via the
thin binding) and measure errors against the oracle."""
from __future__ import annotations

import sys

import numpy as np


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def run_gpu(q, env, nq, ops, kind=None, prec=None, fusion=None, init=0, state=None, keep=False):
    """Apply ``ops`` on a fresh register; returns the amplitudes (and the
    register when ``keep``).  fusion=None: one C-ABI call per op; else
    qs_circuit_run with that fusion width."""
    kind = q.STATEVEC if kind is None else kind
    prec = q.C128 if prec is None else prec
    reg = q.Register(env, nq, kind, prec)
    if state is not None:
        reg.set_amps(state)
    else:
        reg.init_basis(init)
    if fusion is None:
        for op in ops:
            reg.apply(op)
    else:
        c = q.Circuit(ops)
        c.run(reg, fusion)
        c.close()
    amps = reg.get_amps()
    if keep:
        return amps, reg
    reg.close()
    return amps


def max_abs(a, b) -> float:
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b)))) if len(a) else 0.0


def fidelity_deficit(ref, got) -> float:
    """1 - |<ref|got>|^2 with neither vector renormalised."""
    ref = np.asarray(ref, dtype=np.complex128)
    got = np.asarray(got, dtype=np.complex128)
    ov = np.vdot(ref, got)
    return float(1.0 - abs(ov) ** 2)
