"""Host-code sanitizer runs (AddressSanitizer + UndefinedBehaviorSanitizer), CPU only.

* The CPU oracle (oracle/lt_oracle.c) built with gcc and both sanitizers, driven
  on random label images with and without spacing weights
  (tests/sanitize/oracle_main.c).
* liblt's host code: every .hip source compiled with the sanitizers on the host side
  only (-Xarch_host before each -fsanitize=; the device code is built as usual),
  linked with tests/sanitize/lib_driver.cpp and run in its "host" mode (status
  strings, argument checks, mesh cell tables, scratch sizing, injected allocation
  failure).  The executable stays in tests/sanitize/_build; its "device" mode is
  run on a GPU machine by tests/test_gpu_host_sanitized.py."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(HERE, "sanitize", "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _host_flags():
    out = []
    for f in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"):
        out += ["-Xarch_host", f]
    return out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_ubsan():
    os.makedirs(BUILD, exist_ok=True)
    exe = os.path.join(BUILD, "oracle_san")
    cmd = ["gcc", "-std=c99", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-o", exe, os.path.join(ROOT, "oracle", "lt_oracle.c"), os.path.join(HERE, "sanitize", "oracle_main.c")]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    r = subprocess.run([exe], capture_output=True, text=True, env=SAN_ENV, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "oracle sanitizer run ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_library_host_code_under_asan_ubsan():
    os.makedirs(BUILD, exist_ok=True)
    csrc = os.path.join(ROOT, "paper_2504_05808_amd", "csrc")
    srcs = sorted(os.path.join(csrc, f) for f in os.listdir(csrc) if f.endswith(".hip"))
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops"] + _host_flags()

    def compile_one(src):
        obj = os.path.join(BUILD, os.path.basename(src) + ".o")
        r = subprocess.run([HIPCC, *flags, "-c", src, "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        return obj

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, srcs))
    drv = os.path.join(BUILD, "lib_driver.o")
    r = subprocess.run([HIPCC, *flags, "-c", os.path.join(HERE, "sanitize", "lib_driver.cpp"), "-o", drv],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    exe = os.path.join(BUILD, "lib_san")
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", *_host_flags(), "-o", exe, drv, *objs],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    for o in objs + [drv]:                       # only the executable is kept
        os.remove(o)
    r = subprocess.run([exe, "host"], capture_output=True, text=True, env=SAN_ENV, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "lib sanitizer run ok (host)" in r.stdout
