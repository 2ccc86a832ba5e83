"""The threaded oracle under ThreadSanitizer (CPU): every threaded reference runs on small
inputs with -fsanitize=thread and must report no data race and agree with the closed
forms."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_threaded_oracle_is_race_free(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "tsan_driver"
    cmd = ["g++", "-std=c++20", "-O1", "-g", "-fsanitize=thread", "-pthread",
           os.path.join(ROOT, "oracle", "sp_oracle.cpp"),
           os.path.join(ROOT, "oracle", "tsan_driver.cpp"), "-o", str(exe)]
    subprocess.check_call(cmd)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    p = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert p.returncode == 0, (p.returncode, p.stderr[-4000:])
    assert "ThreadSanitizer" not in p.stderr, p.stderr[-4000:]
    assert "agree with the closed forms" in p.stdout
