"""Host-side checks of the server (no GPU): each pure C++ check is compiled
with g++ on its own, under ASan/UBSan, and run.

* sched_check.cpp: the admission policy and the scratch allocator.
* ticket_model.cpp: how a level pass hands out work tickets while a kernel
  of other code holds part of the device: fixed first tickets stall the
  pass for as long as that code keeps the slots (or, with the bounded wait,
  end it in an error); tickets from the counter, as the server takes them,
  let the pass finish on the slots it has.
* epoch_check.cpp: the look-back tag rule, that a wrap of the tags may clear
  the tag words only (clearing the stage counters too loses the work of the
  requests in flight), and the server's 64-bit pass numbering."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1107_3622_amd", "csrc")


def build_and_run(tmp_path, src: str) -> str:
    exe = tmp_path / os.path.splitext(src)[0]
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-fsanitize=address,undefined",
                    "-I", CSRC, os.path.join(ROOT, "tests", src), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr + r.stdout
    return r.stdout


def test_scheduler_policy(tmp_path):
    assert "passed" in build_and_run(tmp_path, "sched_check.cpp")


def test_ticket_protocol_under_partial_residency(tmp_path):
    assert "all checks passed" in build_and_run(tmp_path, "ticket_model.cpp")


@pytest.mark.parametrize("src", ["epoch_check.cpp"])
def test_epoch_wrap_and_pass_numbering(tmp_path, src):
    assert "passed" in build_and_run(tmp_path, src)
