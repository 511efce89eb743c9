"""liblt's host code under AddressSanitizer and UndefinedBehaviorSanitizer (host side
only; the device code is the regular build) on a GPU machine: the executable that
tests/test_host_sanitizers.py builds runs its "device" mode, which calls every
entry-point family on small inputs.  Skipped when that executable was not built."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sanitize", "_build", "lib_san")


def test_library_paths_with_host_sanitizers():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(EXE):
        pytest.skip("sanitized driver not built (run tests/test_host_sanitizers.py on the CPU first)")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([EXE, "device"], capture_output=True, text=True, env=env, timeout=240)
    print(r.stdout[-2000:], r.stderr[-2000:], flush=True)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "lib sanitizer run ok (device)" in r.stdout
