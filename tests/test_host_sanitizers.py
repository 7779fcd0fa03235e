"""The host code of the library (C ABI validation, plan set-up, tile -> frame
lists, strip records, workspace layout, batch bookkeeping) under
AddressSanitizer and UndefinedBehaviorSanitizer: the ABI tests of
test_abi.py run again in a child process against a build whose host objects
are instrumented (device code unchanged; no device work is done)."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_tests_pass_under_host_sanitizers(tmp_path):
    from paper_1602_01448_amd import build_sanitized
    from paper_1602_01448_amd.build import BUILD
    if not os.path.isdir(BUILD):
        pytest.skip("library not built in-tree (no kernel objects to link)")
    if shutil.which("nm") is None:
        pytest.skip("nm not available")
    lib = build_sanitized.build(str(tmp_path))
    syms = subprocess.run(["nm", "-D", lib], capture_output=True, text=True).stdout
    assert "__asan_report" in syms and "__ubsan_handle" in syms   # the host code is instrumented
    env = dict(os.environ, LD_PRELOAD=build_sanitized.runtime(), SHARP_LIBRARY=lib,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-m", "not gpu", os.path.join(ROOT, "tests", "test_abi.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out
