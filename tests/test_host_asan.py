"""The host runtime under AddressSanitizer: libpm_asan.so (host sources
instrumented, device objects of the normal build) runs every host-only path
of the C ABI (tests/host_asan_driver.py) in a child process with the
sanitizer runtime preloaded; any invalid access aborts it."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_host_runtime_under_asan():
    sys.path.insert(0, ROOT)
    from paper_2209_01290_amd import asan_host
    try:
        lib = asan_host.build()
        rt = asan_host.runtime()
    except RuntimeError as e:
        pytest.fail(str(e))
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1")
    p = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "host_asan_driver.py"), lib],
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, env=env, timeout=600)
    assert p.returncode == 0 and "AddressSanitizer" not in p.stdout, p.stdout[-4000:]
    assert "host paths ok" in p.stdout
