"""qs_prob_noalloc (include/qstate_noalloc.h) against the register calls it
mirrors: two calls in a row on one GPU, the second on a smaller input, for
state vectors and density matrices in both precisions.  The static partials
array keeps the first call's contents; the second call must not see them."""
import numpy as np
import pytest
import torch

import oracle as O
from tests.gpu_util import log
from workloads import random_multi_ops, random_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope='module')
def q():
    import paper_1802_08032_amd as q
    return q


def noalloc(q, reg, qubit):
    out = torch.full((2,), float('nan'), dtype=torch.float64, device='cuda:0')
    stream = torch.cuda.current_stream(0).cuda_stream
    q.prob_noalloc(0, reg.tensor.data_ptr(), reg.n, reg.kind, reg.prec, qubit, out.data_ptr(), stream)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def check_register(q, reg, ref_p0):
    total = reg.calc_total_prob()
    got = noalloc(q, reg, -1)
    assert got[0] == total and got[1] == 0.0, (got, total)
    tol = 1e-12 if reg.prec == q.C128 else 1e-5
    for k in range(reg.n):
        p0, p1 = reg.calc_prob_of_outcome(k, 0), reg.calc_prob_of_outcome(k, 1)
        got = noalloc(q, reg, k)
        assert abs(got[0] - p0) <= 1e-12 and abs(got[1] - p1) <= 1e-12, (k, got, p0, p1)
        assert abs(got[0] - ref_p0[k]) <= tol, (k, got[0], ref_p0[k])


@pytest.mark.parametrize('prec_name', ['C128', 'C64'])
def test_noalloc_matches_register_calls_sv(q, prec_name):
    prec = getattr(q, prec_name)
    env = q.Env(0)
    for n in (20, 12):  # second call on a smaller input
        psi = random_state(n, 70 + n)
        reg = q.Register(env, n, q.STATEVEC, prec)
        reg.set_amps(psi)
        log(f'no-alloc probabilities: state vector n={n} {prec_name}')
        check_register(q, reg, [O.sv_prob_outcome(psi, n, k, 0) for k in range(n)])
        reg.close()
    env.close()


@pytest.mark.parametrize('prec_name', ['C128', 'C64'])
def test_noalloc_matches_register_calls_dm(q, prec_name):
    prec = getattr(q, prec_name)
    env = q.Env(0)
    for N in (9, 5):
        rho = O.run_dm(N, random_multi_ops(N, 10, 80 + N, max_targets=2, max_controls=1, kraus=True))
        reg = q.Register(env, N, q.DENSITY, prec)
        reg.set_amps(rho)
        log(f'no-alloc probabilities: density matrix N={N} {prec_name}')
        check_register(q, reg, [O.dm_prob_outcome(rho, N, k, 0) for k in range(N)])
        reg.close()
    env.close()


def test_noalloc_rejects_bad_arguments(q):
    buf = torch.zeros(4, dtype=torch.complex128, device='cuda:0')
    out = torch.zeros(2, dtype=torch.float64, device='cuda:0')
    for args in ((0, 0, 2, q.STATEVEC, q.C128, 0, out.data_ptr()),           # NULL amplitudes
                 (0, buf.data_ptr(), 0, q.STATEVEC, q.C128, -1, out.data_ptr()),  # n = 0
                 (0, buf.data_ptr(), 41, q.STATEVEC, q.C128, -1, out.data_ptr()),
                 (0, buf.data_ptr(), 21, q.DENSITY, q.C128, -1, out.data_ptr()),
                 (0, buf.data_ptr(), 2, q.STATEVEC, q.C128, 2, out.data_ptr()),   # qubit >= n
                 (0, buf.data_ptr(), 2, 7, q.C128, 0, out.data_ptr()),
                 (0, buf.data_ptr(), 2, q.STATEVEC, 3, 0, out.data_ptr()),
                 (-1, buf.data_ptr(), 2, q.STATEVEC, q.C128, 0, out.data_ptr()),
                 (0, buf.data_ptr(), 2, q.STATEVEC, q.C128, 0, 0)):
        with pytest.raises(q.QStateError, match='QS_E_ARG'):
            q.prob_noalloc(*args)
