"""The serving queue under concurrent clients with AddressSanitizer on the
library's host code: tests/native/serve_threads (built with the library by
tests/native/build_asan.py, which __graft_entry__.build() runs) submits and
polls from three threads while a fourth reads the counters; every request
must finish with MLMC_OK and AddressSanitizer must report nothing."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
DRIVER = os.path.join(HERE, "native", "build", "serve_threads")


def test_serving_threads_under_address_sanitizer():
    assert os.path.exists(DRIVER), "build it first: python tests/native/build_asan.py"
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    r = subprocess.run([DRIVER], capture_output=True, text=True, timeout=240, env=env)
    out = r.stdout + r.stderr
    print(out[-2000:])
    assert "AddressSanitizer" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert "requests 36 done 36 bad 0 completed 36" in r.stdout
