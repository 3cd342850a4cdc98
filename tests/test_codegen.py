"""CPU checks of the run-time specialised pass kernels: the generated HIP
source of each pass compiles for gfx950 with hipRTC (no GPU needed), and
the generated code uses the literal layout the planner chose."""
import ctypes as C
import os

import pytest

from workloads import layered_circuit, random_gate_ops


def hiprtc():
    for name in ('libhiprtc.so', '/opt/rocm/lib/libhiprtc.so'):
        try:
            return C.CDLL(name)
        except OSError:
            continue
    pytest.skip('hipRTC not available')


def compile_src(src: str):
    L = hiprtc()
    prog = C.c_void_p()
    assert L.hiprtcCreateProgram(C.byref(prog), src.encode(), b'qs_pass.hip', 0, None, None) == 0
    opts = [b'--offload-arch=gfx950', b'-O3', b'-Xclang', b'-target-feature', b'-Xclang', b'-packed-fp32-ops']
    arr = (C.c_char_p * len(opts))(*opts)
    rc = L.hiprtcCompileProgram(prog, len(opts), arr)
    size = C.c_size_t()
    L.hiprtcGetProgramLogSize(prog, C.byref(size))
    log = C.create_string_buffer(size.value + 1)
    L.hiprtcGetProgramLog(prog, log)
    code = C.c_size_t()
    L.hiprtcGetCodeSize(prog, C.byref(code))
    L.hiprtcDestroyProgram(C.byref(prog))
    return rc, log.value.decode(errors='replace'), code.value


@pytest.mark.parametrize('prec_name,tile,tb', [('C128', 12, 9), ('C64', 14, 10)])
def test_generated_pass_compiles(prec_name, tile, tb):
    import paper_1802_08032_amd as q
    prec = getattr(q, prec_name)
    ops = layered_circuit(20, 3, 1, mcphase=True) + random_gate_ops(20, 40, 3, max_controls=3)
    c = q.Circuit(ops)
    src, npass = c.source(20, prec, tile, tb, 0)
    assert npass >= 1 and 'qs_pass' in src
    rc, log, size = compile_src(src)
    assert rc == 0, log
    assert size > 1000
    c.close()


def test_source_rejects_bad_shapes():
    import paper_1802_08032_amd as q
    c = q.Circuit(layered_circuit(12, 1, 0))
    for args in ((12, q.C128, 14, 9), (12, q.C128, 12, 5), (12, q.C128, 12, 11), (10, q.C128, 12, 8)):
        with pytest.raises(q.QStateError):
            c.source(*args)
    c.close()


def test_generated_density_matrix_pass_compiles():
    """Density matrices: gates on (q, q+N) and 4x4 channel superoperators."""
    import paper_1802_08032_amd as q
    from workloads import noisy_circuit
    c = q.Circuit(noisy_circuit(7, 2, 1) + random_gate_ops(7, 10, 2, max_controls=2))
    src, npass = c.source(7, q.C128, 12, 8, 0, 0, 4, kind=q.DENSITY)
    assert 'qs_ap4(' in src
    rc, log, size = compile_src(src)
    assert rc == 0, log
    c.close()


def test_pass_merges_and_deferred_flips_in_source():
    """On the layered brick circuit the generated passes merge runs of
    register-only gates into 4x4 ops (applied as unit-diagonal 4x4 cores) and
    keep thread-controlled NOTs as per-lane flips instead of register swaps;
    the passes still compile."""
    import re
    import paper_1802_08032_amd as q
    c = q.Circuit(layered_circuit(32, 10, seed=1, mcphase=True))
    _, npass = c.source(32, q.C128, 12, 8, 0, 0, 4)
    srcs = [c.source(32, q.C128, 12, 8, p, 0, 4)[0] for p in range(npass)]
    assert any('qs_core4(c, ' in s for s in srcs)
    flips = sum(len(re.findall(r'const bool f[0-9]+ = ', s)) for s in srcs)
    swaps = sum(s.count('const V ta =') for s in srcs)
    # a materialised flip swaps the 8 register pairs of a 16-register thread;
    # most thread-controlled NOTs stay flips
    assert flips > 30 and swaps / 8 < flips
    pick = max(range(npass), key=lambda p: srcs[p].count('twf') + srcs[p].count(' ^ sf)'))
    rc, log, _ = compile_src(srcs[pick])
    assert rc == 0, log
    c.close()


def test_library_kernels_use_no_scratch():
    """Every kernel of the streaming and fused sources compiles for gfx950
    without a private (scratch) segment: spills or arrays the compiler
    could not keep in registers would turn into per-lane memory traffic."""
    import re
    import subprocess
    import tempfile
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    csrc = os.path.join(root, 'paper_1802_08032_amd', 'csrc')
    for src in ('qs_kernels.hip', 'qs_fused.hip'):
        with tempfile.TemporaryDirectory() as d:
            out = os.path.join(d, 'k.s')
            cmd = ['/opt/rocm/bin/hipcc', '--offload-arch=gfx950', '-O3', '-std=c++17', '--cuda-device-only', '-S',
                   '-Xclang', '-target-feature', '-Xclang', '-packed-fp32-ops',
                   '-I', os.path.join(root, 'include'), os.path.join(csrc, src), '-o', out]
            r = subprocess.run(cmd, capture_output=True, text=True)
            if r.returncode != 0 and 'not found' in r.stderr and 'hipcc' in r.stderr:
                pytest.skip('hipcc not available')
            assert r.returncode == 0, r.stderr[-2000:]
            asm = open(out).read()
        kernels = re.findall(r'\.amdhsa_kernel (\S+)(.*?)\.end_amdhsa_kernel', asm, re.S)
        assert kernels
        for name, body in kernels:
            size = int(re.search(r'\.amdhsa_private_segment_fixed_size (\d+)', body).group(1))
            assert size == 0, f'{src}: {name} uses {size} bytes of scratch'


def test_planner_pass_counts():
    """The compiled path's partition (candidate tile sets with a one-pass
    lookahead) fits the 32-qubit depth-10 layered circuit (485 gates) into
    at most 12 HBM round trips with 12- or 13-qubit tiles, the same circuit
    at 33 qubits in complex64 into at most 11 with 14-qubit tiles, and the
    14-qubit noisy density matrix (1015 ops on its 28-qubit vector) into at
    most 10.  Guards against planner changes that add passes."""
    import paper_1802_08032_amd as q
    from workloads import noisy_circuit
    c = q.Circuit(layered_circuit(32, 10, seed=1, mcphase=True))
    for tile, tb in ((12, 8), (13, 9)):
        assert c.source(32, q.C128, tile, tb, 0, 0, 4)[1] <= 12, tile
    c.close()
    c = q.Circuit(layered_circuit(33, 10, seed=1, mcphase=True))
    assert c.source(33, q.C64, 14, 10, 0, 0, 5)[1] <= 11
    c.close()
    c = q.Circuit(noisy_circuit(14, 10, 2))
    assert c.source(14, q.C128, 12, 8, 0, 0, 4, kind=q.DENSITY)[1] <= 10
    c.close()
