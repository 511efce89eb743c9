"""LT_LOG: the library's stderr log (host side, no GPU needed).  Level 1 prints one
line per error status, naming the call it came from; level 2 also prints each call
that takes a volume with its shape, label type and label bound; unset prints
nothing.  Each case runs in a fresh process so that the library reads its own
environment."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import ctypes, sys
sys.path.insert(0, %r)
from paper_2504_05808_amd import lt
lib = lt.load()
shape = (ctypes.c_int64 * 3)(4, 5, 6)
# NULL context: an argument error before any device call
st = lib.lt_pipeline(None, None, 1, 3, shape, 7, None, None, None, None)
assert st == 1, st
# int32 labels and a shape the call would reject (the NULL context is checked first)
bad = (ctypes.c_int64 * 3)(4, -5, 6)
lib.lt_edt.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                       ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p, ctypes.c_void_p]
st = lib.lt_edt(None, None, 2, 3, bad, None, None)
assert st == 1, st
# a call without a volume: logged only when it fails
st = lib.lt_remap_roundness(None, None, 0, ctypes.c_float(0.0), None, None)
print("done", flush=True)
""" % ROOT


def _run(level):
    env = dict(os.environ)
    env.pop("LT_LOG", None)
    if level is not None:
        env["LT_LOG"] = str(level)
    r = subprocess.run([sys.executable, "-c", SCRIPT], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr
    assert "done" in r.stdout
    return [ln for ln in r.stderr.splitlines() if ln.startswith("[lt]")]


def test_unset_is_silent():
    assert _run(None) == []
    assert _run(0) == []


def test_level_1_names_the_failing_call():
    lines = _run(1)
    assert lines[0] == "[lt] lt_pipeline: invalid argument: ctx is NULL"
    assert lines[1] == "[lt] lt_edt: invalid argument: ctx is NULL"
    assert all(": " in ln for ln in lines) and not any("shape=" in ln for ln in lines)


def test_level_2_adds_the_volume_calls():
    lines = _run(2)
    assert lines[0] == "[lt] lt_pipeline shape=4x5x6 dtype=u16 max_label=7"
    assert lines[1] == "[lt] lt_pipeline: invalid argument: ctx is NULL"
    assert lines[2] == "[lt] lt_edt shape=4x-5x6 dtype=i32"
    assert lines[3] == "[lt] lt_edt: invalid argument: ctx is NULL"
    # the call without a volume prints only its error line, if any
    assert all(ln.startswith("[lt] lt_remap_roundness:") for ln in lines[4:])
