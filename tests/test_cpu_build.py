"""The library on the host (no GPU): its own sources (host driver, server
and kernels) compiled with g++ against tests/cpu_sim/hip/hip_runtime.h, a
small HIP runtime that runs each workgroup's threads as fibers on a CPU
thread and keeps guard pages around every device allocation.

* plain sorts of arrays spanning many tiles against std::sort, with the
  first pivot against its closed form;
* the server with slot, scratch and buffer reuse over hundreds of requests
  of mixed sizes and key types, 256 in flight;
* the same with asynchronous in-order queues shared by several streams
  (a producer and a checker stream beside the server's), with and without
  kernels of those streams competing for the workgroup slots of the device;
* the literal arrangement (one level on many segments, and the whole sort
  with its call records) against the C oracle, which only this test program
  links, at sizes whose look-back spans more than one window of 64 blocks.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1107_3622_amd", "csrc")
SIM = os.path.join(ROOT, "tests", "cpu_sim")
LIB_SOURCES = [os.path.join(CSRC, f) for f in ("ksort_lib.hip", "ksort_server.hip", "ksort_tune.hip",
                                                 "ksort_exact.hip")]
ORACLE = os.path.join(ROOT, "oracle")


@pytest.fixture(scope="module")
def sim_build(tmp_path_factory):
    out = tmp_path_factory.mktemp("ksim")
    oracle_obj = str(out / "ksort_oracle.o")
    subprocess.run(["gcc", "-O1", "-g", "-c", os.path.join(ORACLE, "ksort_oracle.c"), "-I", ORACLE, "-o", oracle_obj],
                   check=True)
    exes = {}
    for drv in ("plain_sim", "server_sim", "serve_async_sim", "exact_sim"):
        exe = out / drv
        extra = [oracle_obj] if drv == "exact_sim" else []
        subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-rdynamic", "-Wall",
                        "-Wno-attributes", "-Wno-unknown-pragmas", "-Wno-unused-function", "-Wno-sign-compare",
                        "-I", SIM, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-I", ORACLE,
                        "-x", "c++", *LIB_SOURCES, "-x", "none", os.path.join(SIM, "ksim.cpp"),
                        os.path.join(SIM, drv + ".cpp"), *extra, "-o", str(exe), "-lpthread"], check=True)
        exes[drv] = str(exe)
    return exes


def run(exe, args, env_extra, timeout=600):
    env = dict(os.environ, KSIM_CUS="4", KSIM_OCC="2", **env_extra)
    r = subprocess.run([exe, *map(str, args)], capture_output=True, text=True, env=env, timeout=timeout)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    return r.stdout


@pytest.mark.parametrize("n", [1000, 70_000, 300_000])
def test_plain_sorts_on_the_host_build(sim_build, n):
    assert "ok" in run(sim_build["plain_sim"], [n], {})


def test_server_reuse_on_the_host_build(sim_build):
    out = run(sim_build["server_sim"], [400, 1000, 20000, 256, 1024, 500], {})
    assert "400 completed, 0 failed" in out and "0 wrong" in out


@pytest.mark.parametrize("hwq,slots", [(4, None), (1, None), (4, 8)])
def test_server_with_async_queues_on_the_host_build(sim_build, hwq, slots):
    env = {"KSIM_HWQ": str(hwq)}
    if slots:
        env["KSIM_SLOTS"] = str(slots)
    out = run(sim_build["serve_async_sim"], [120, 1000, 20000, 256, 1024, 2000], env)
    assert "120 completed, 0 failed" in out and "0 wrong" in out


@pytest.mark.parametrize("n,kinds", [(300, "01234"), (2000, "01"), (300_000, "0")])
def test_exact_arrangement_on_the_host_build(sim_build, n, kinds):
    out = run(sim_build["exact_sim"], [n, kinds], {})
    assert "MISMATCH" not in out and "0 failed" in out


def test_trace_file_on_the_host_build(sim_build, tmp_path):
    """KSORT_TRACE: one JSON line per level pass of every sorting call; the
    first pass partitions the whole array, and every pass of the call
    carries the variant that ran."""
    import json
    path = tmp_path / "trace.jsonl"
    n = 70_000
    assert "ok" in run(sim_build["plain_sim"], [n], {"KSORT_TRACE": str(path)})
    recs = [json.loads(x) for x in path.read_text().splitlines()]
    assert len(recs) >= 3
    assert recs[0]["stage"] == 0 and recs[0]["live_keys"] == n and recs[0]["dtype"] == "f64"
    assert [r["stage"] for r in recs] == list(range(len(recs)))
    assert len({(r["call"], r["block"], r["items"], r["cutoff"]) for r in recs}) == 1
