"""Host logic of the batched and serving forms (no GPU).

serve.hip is built with the host compiler against a host-only stand-in for the
HIP runtime and for the single-graph entry points (tests/host_mock), under
ThreadSanitizer, and driven by tests/host_mock/executor_driver.cpp: results
equal those of each graph alone, one graph never runs two requests at once,
a failing request stays with its ticket, admission follows the budget and
every worker stream is released.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MOCK = os.path.join(ROOT, "tests", "host_mock")


def _build(tmp_path, sanitize):
    exe = str(tmp_path / ("exec_tsan" if sanitize else "exec"))
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-pthread"] + (["-fsanitize=thread"] if sanitize else []) + [
        "-I", MOCK, "-I", os.path.join(ROOT, "include"),
        "-x", "c++", os.path.join(ROOT, "paper_2410_15451_amd", "csrc", "serve.hip"),
        "-x", "none", os.path.join(MOCK, "mock_leiden.cpp"), os.path.join(MOCK, "executor_driver.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    return exe if r.returncode == 0 else None, r.stderr


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
@pytest.mark.parametrize("sanitize", [True, False])
def test_executors_host_logic(tmp_path, sanitize):
    exe, err = _build(tmp_path, sanitize)
    if exe is None:
        if sanitize:
            pytest.skip("ThreadSanitizer build unavailable: " + err[-300:])
        raise AssertionError(err[-2000:])
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert r.stdout.strip().endswith("OK")
