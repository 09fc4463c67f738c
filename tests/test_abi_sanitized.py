"""The CPU tests of the C ABI (tests/test_abi.py) once more, against a build
whose host code (argument validation, workspace planning, the batch planner
and the server's entry points) runs under AddressSanitizer and
UndefinedBehaviorSanitizer; any report aborts the child process."""
import os
import subprocess
import sys

import pytest

from tests.helpers import ROOT, ensure_built

CHILD = r"""
import sys
sys.path.insert(0, {root!r})
import paper_1310_7202_amd as m
m.LIB_PATH = {lib!r}
import pytest
sys.exit(pytest.main(["-q", "-x", "-s", "-p", "no:cacheprovider",
                      {test!r}]))
"""


def test_abi_under_address_and_undefined_behaviour_sanitizers():
    ensure_built()
    from paper_1310_7202_amd import build
    try:
        lib = build.build_sanitized()
        runtime = build.sanitizer_runtime()
    except RuntimeError as e:
        pytest.skip(f"no sanitizer build: {e}")
    env = dict(os.environ)
    env["LD_PRELOAD"] = runtime
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    code = CHILD.format(root=ROOT, lib=lib, test=os.path.join(ROOT, "tests", "test_abi.py"))
    res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                         timeout=600)
    out = res.stdout + res.stderr
    assert "runtime error" not in out, out[-4000:]
    assert "AddressSanitizer" not in out, out[-4000:]
    assert res.returncode == 0, out[-4000:]
    assert " passed" in out
