"""Host-side checks of the server's admission policy and scratch allocator:
the pure C++ header is compiled with g++ on its own and run (no GPU)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_scheduler_policy(tmp_path):
    exe = tmp_path / "sched_check"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-fsanitize=address,undefined",
                    "-I", os.path.join(ROOT, "paper_1107_3622_amd", "csrc"),
                    os.path.join(ROOT, "tests", "sched_check.cpp"), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    assert "passed" in r.stdout
