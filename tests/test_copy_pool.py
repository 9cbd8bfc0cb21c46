"""The request server's host copy pool (csrc/copy_pool.h), built on its own
with g++ and run on the CPU: concurrent callers of assorted sizes and
alignments each get their bytes and nothing else, with ThreadSanitizer
watching for data races, and with 0 helpers (the caller copies alone)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1703_06256_amd", "csrc")
SRC = os.path.join(HERE, "native", "copy_pool_check.cpp")


def _build(tmp_path, extra):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "copy_pool_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-pthread", "-I", CSRC, SRC, "-o", exe] + extra
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


@pytest.mark.parametrize("helpers", [0, 1, 3])
def test_copy_pool_copies_exactly(tmp_path, helpers):
    exe = _build(tmp_path, [])
    r = subprocess.run([exe, str(helpers)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "OK", r.stdout + r.stderr


def test_copy_pool_has_no_data_races(tmp_path):
    exe = _build(tmp_path, ["-fsanitize=thread"])
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    r = subprocess.run([exe, "3"], capture_output=True, text=True, timeout=300, env=env)
    if r.returncode != 0 and "FATAL: ThreadSanitizer" in r.stderr and "unexpected memory mapping" in r.stderr:
        pytest.skip("ThreadSanitizer cannot run under this kernel's address layout")
    assert r.returncode == 0 and r.stdout.strip() == "OK", r.stdout + r.stderr[-4000:]
