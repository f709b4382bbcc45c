"""The oracle under AddressSanitizer + UndefinedBehaviorSanitizer (host
code only): every access stays in bounds and no undefined behaviour occurs
on small, duplicate-heavy and 1e5-element inputs."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_asan_ubsan(tmp_path):
    exe = str(tmp_path / "selfcheck")
    subprocess.run(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "oracle"),
                    os.path.join(ROOT, "tests", "oracle_selfcheck.c"),
                    os.path.join(ROOT, "oracle", "ksort_oracle.c"), "-o", exe], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "selfcheck failures: 0" in r.stdout
