"""The host side of the library under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only).

Every library source and a host-only driver (tests/sanitize/host_driver.cpp)
are built with the sanitizers on the host pass only (device code is built
as usual and never launched).  The driver plans and generates every pass of
seeded random circuits (state vectors in both precisions at three tile
shapes, noisy density matrices) through the C ABI, so the planner, the op
merger, the deferred-factor algebra and the source generator run under the
sanitizers; any report aborts the driver."""
import concurrent.futures as cf
import hashlib
import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get('HIPCC', '/opt/rocm/bin/hipcc')
CSRC = os.path.join(ROOT, 'paper_1802_08032_amd', 'csrc')
SOURCES = [os.path.join(CSRC, f) for f in
           ('qs_api.hip', 'qs_kernels.hip', 'qs_fused.hip', 'qs_plan.hip', 'qs_jit.hip', 'qs_noalloc.hip')]
DRIVER = os.path.join(ROOT, 'tests', 'sanitize', 'host_driver.cpp')
# sanitizers on the host compilation only
SAN = ('-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined '
       '-Xarch_host -fno-sanitize-recover=all -Xarch_host -fno-omit-frame-pointer').split()
FLAGS = ['--offload-arch=gfx950', '-O1', '-g', '-std=c++17', '-Xclang', '-target-feature', '-Xclang',
         '-packed-fp32-ops', '-I' + os.path.join(ROOT, 'include'), '-I' + CSRC] + SAN


def _build():
    h = hashlib.sha1()
    for f in SOURCES + [DRIVER] + [os.path.join(CSRC, x) for x in os.listdir(CSRC) if x.endswith('.h')]:
        h.update(open(f, 'rb').read())
    h.update(' '.join(FLAGS).encode())
    out = os.path.join(tempfile.gettempdir(), 'qs_sanitize', h.hexdigest()[:16])
    exe = os.path.join(out, 'driver')
    if os.path.exists(exe):
        return exe
    os.makedirs(out, exist_ok=True)

    def compile_one(src):
        obj = os.path.join(out, os.path.basename(src) + '.o')
        lang = ['-x', 'hip'] if src.endswith('.cpp') else []
        r = subprocess.run([HIPCC, *FLAGS, *lang, '-c', src, '-o', obj], capture_output=True, text=True)
        if r.returncode:
            raise RuntimeError(f'compile {src}:\n{r.stderr[-3000:]}')
        return obj

    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(compile_one, SOURCES + [DRIVER]))
    tmp = exe + f'.tmp{os.getpid()}'
    r = subprocess.run([HIPCC, '--offload-arch=gfx950', *SAN, *objs, '-o', tmp, '-lhiprtc'],
                       capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError(f'link:\n{r.stderr[-3000:]}')
    os.replace(tmp, exe)
    return exe


@pytest.mark.skipif(not os.path.exists(HIPCC), reason='hipcc not found')
def test_planner_and_generator_under_sanitizers():
    exe = _build()
    env = dict(os.environ, ASAN_OPTIONS='detect_leaks=0:abort_on_error=1',
               UBSAN_OPTIONS='print_stacktrace=1:halt_on_error=1')
    r = subprocess.run([exe], capture_output=True, text=True, timeout=900, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
    assert r.stdout.strip().endswith('ok')
