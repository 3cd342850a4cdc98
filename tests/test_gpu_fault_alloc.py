"""Host-forced out-of-memory: QS_FAULT_ALLOC=k makes the library's k-th
device allocation fail.  A fresh child process (the variable is set before
the library makes any GPU call) checks that each failing call returns
QS_E_OOM, frees what it had taken and leaves existing registers as they
were, and that the next allocation succeeds."""
import os
import subprocess
import sys
import textwrap

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = textwrap.dedent('''
    import sys
    import numpy as np
    import paper_1802_08032_amd as q

    env = q.Env(0)
    # allocation 1: the reduction scratch of a register over torch memory
    a = q.Register(env, 10)
    a.init_zero()
    a.hadamard(3)
    a.cnot(3, 7)
    before = a.get_amps()
    fault = int(sys.argv[1])
    try:
        # allocation 2: amplitudes of an owned register; 3: its scratch
        # (fault 3 also checks that the amplitudes taken first are freed)
        q.Register(env, 12, owned=True)
    except q.QStateError as e:
        assert e.name == 'QS_E_OOM', e
        print('oom raised', e, flush=True)
    else:
        raise AssertionError('no QS_E_OOM for the faulted allocation')
    after = a.get_amps()
    assert np.array_equal(before, after)
    assert abs(a.calc_total_prob() - 1.0) <= 1e-12
    b = q.Register(env, 12, owned=True)
    b.init_zero()
    b.hadamard(0)
    assert abs(b.calc_total_prob() - 1.0) <= 1e-12
    b.close()
    a.close()
    env.close()
    print('FAULT_ALLOC_OK', flush=True)
''')


@pytest.mark.parametrize('fault', [2, 3])
def test_forced_allocation_failure_returns_oom(fault):
    envv = dict(os.environ, QS_FAULT_ALLOC=str(fault))
    envv['PYTHONPATH'] = ROOT + os.pathsep + envv.get('PYTHONPATH', '')
    print(f'child with QS_FAULT_ALLOC={fault}', flush=True)
    r = subprocess.run([sys.executable, '-c', CHILD, str(fault)], cwd=ROOT, env=envv, capture_output=True,
                       text=True, timeout=300)
    print(r.stdout[-2000:], r.stderr[-2000:], flush=True)
    assert r.returncode == 0
    assert 'FAULT_ALLOC_OK' in r.stdout
