"""CPU checks of the C-ABI library: it loads, exports every symbol that
include/*.h declare, and its byte accounting follows the paper's
16 x 2^n B per double-precision state vector (Sec. II.B.1).  No kernels run."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INCLUDE = os.path.join(ROOT, 'include')


def declared_functions():
    text = ''.join(open(os.path.join(INCLUDE, f)).read() for f in sorted(os.listdir(INCLUDE)) if f.endswith('.h'))
    text = re.sub(r'/\*.*?\*/', '', text, flags=re.S)
    return sorted(set(re.findall(r'\b(qs_[a-z0-9_]+)\s*\(', text)))


def test_library_exports_every_declared_symbol():
    import paper_1802_08032_amd as q
    L = q.lib()
    names = declared_functions()
    assert len(names) >= 30
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # the binding declares a signature for every exported call
    from paper_1802_08032_amd.qstate import SIGNATURES
    assert sorted(SIGNATURES) == names


def test_reg_bytes_formula():
    import paper_1802_08032_amd as q
    for n in (1, 5, 16, 32, 40):
        assert q.reg_bytes(n, q.STATEVEC, q.C128) == 16 << n
        assert q.reg_bytes(n, q.STATEVEC, q.C64) == 8 << n
    for n in (1, 8, 14, 20):
        assert q.reg_bytes(n, q.DENSITY, q.C128) == 16 << (2 * n)
    for bad in ((0, 0, 2), (41, 0, 2), (21, 1, 2), (5, 2, 2), (5, 0, 3), (-1, 0, 1)):
        assert q.reg_bytes(*bad) == 0


def test_paper_memory_figures():
    import paper_1802_08032_amd as q
    rows = [l.split() for l in open(os.path.join(ROOT, 'tests', 'golden', 'paper_memory.txt'))
            if l.strip() and not l.startswith('#')]
    assert len(rows) == 8
    for r in rows:
        n, rel, limit, copies = int(r[0]), r[1], int(r[2]), int(r[3])
        need = copies * q.reg_bytes(n, q.STATEVEC, q.C128)
        if rel == 'fits':
            assert need <= limit, r
        elif rel == 'exceeds':
            assert need > limit, r
        else:
            assert need == limit, r


def test_philox_draws_are_numpy_philox4x64_stream():
    """qs_philox_draws (host only) is the Philox4x64-10 stream of Salmon et
    al. (SC'11) as numpy implements it: the same doubles, bit for bit, from
    the start and from an offset inside a 4-word block, for small keys and
    keys near 2^64."""
    import numpy as np
    import paper_1802_08032_amd as q
    for seed, stream in ((0, 0), (7, 3), (2**64 - 1, 2**63 + 5)):
        ref = np.random.Generator(np.random.Philox(key=[seed, stream])).random(40)
        assert np.array_equal(q.philox_draws(seed, stream, 0, 40), ref)
        assert np.array_equal(q.philox_draws(seed, stream, 5, 30), ref[5:35])
    assert q.philox_draws(1, 2, 0, 0).size == 0
    with pytest.raises(q.QStateError):
        q.philox_draws(1, 2, 0, -1)


def test_circuit_parameter_setters_validate_on_the_host():
    """qs_circuit_set_unitary / qs_circuit_set_phase (host only, no device):
    they accept new values for ops of their own kind and reject another
    kind, an index out of range, a non-unitary matrix and a non-finite
    angle, leaving the circuit usable."""
    import numpy as np
    import paper_1802_08032_amd as q
    from workloads import H, Op
    c = q.Circuit([Op('u', target=0, u=H), Op('x', target=1, controls=(0,)),
                   Op('phase', qubits=(0, 1), angle=0.5)])
    c.set_unitary(0, np.eye(2))
    c.set_phase(2, 1.0)
    for bad, code in ((lambda: c.set_unitary(1, H), 'QS_E_ARG'), (lambda: c.set_phase(0, 0.1), 'QS_E_ARG'),
                      (lambda: c.set_unitary(3, H), 'QS_E_ARG'), (lambda: c.set_unitary(-1, H), 'QS_E_ARG'),
                      (lambda: c.set_unitary(0, 2 * H), 'QS_E_NOT_UNITARY'),
                      (lambda: c.set_phase(2, float('nan')), 'QS_E_ARG')):
        with pytest.raises(q.QStateError, match=code):
            bad()
    c.set_unitary(0, H)  # still usable
    c.close()


def test_readout_source_is_the_last_pass_with_sums():
    """qs_circuit_source with pass -1 (host only): the last pass in the form
    qs_circuit_run_compiled_probs runs, with the per-workgroup sums buffer;
    the ordinary form of the same pass has none, and a density matrix has
    no readout form."""
    import paper_1802_08032_amd as q
    from workloads import layered_circuit
    c = q.Circuit(layered_circuit(16, 3, seed=1, mcphase=True))
    ro, npass = c.source(16, q.C128, 12, 8, -1, 0, 4)
    last, _ = c.source(16, q.C128, 12, 8, npass - 1, 0, 4)
    assert npass >= 2
    assert 'double* __restrict__ part' in ro and 'ro_t += t' in ro
    assert 'double* __restrict__ part' not in last and 'ro_t' not in last
    d = q.Circuit(layered_circuit(7, 1, seed=1))
    with pytest.raises(q.QStateError, match='QS_E_KIND'):
        d.source(7, q.C128, 12, 8, -1, 0, 4, kind=q.DENSITY)
    d.close()
    with pytest.raises(q.QStateError, match='QS_E_ARG'):
        c.source(16, q.C128, 12, 8, -2, 0, 4)
    c.close()
