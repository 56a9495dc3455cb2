"""The oracle's threaded entry points under ThreadSanitizer (CPU only).

tests/tsan_driver.c calls the oracle's threaded functions with several
threads each; built with gcc -fsanitize=thread together with the oracle, it
must finish with status 0 and no race report.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is not installed")
def test_oracle_threads_have_no_data_race(tmp_path):
    exe = str(tmp_path / "tsan_driver")
    build = subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-fsanitize=thread", "-pthread", "-o", exe,
                            os.path.join(HERE, "tsan_driver.c"), os.path.join(ROOT, "oracle", "imin_oracle.c")],
                           capture_output=True, text=True)
    if build.returncode != 0 and "sanitize" in build.stderr:
        pytest.skip("ThreadSanitizer runtime unavailable: " + build.stderr[-200:])
    assert build.returncode == 0, build.stderr
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                         env={**os.environ, "TSAN_OPTIONS": "halt_on_error=1"})
    assert "ThreadSanitizer" not in run.stderr, run.stderr[-4000:]
    assert run.returncode == 0, run.stdout + run.stderr
    assert run.stdout.startswith("status 0")
