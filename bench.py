"""Benchmark of the MI355X K-sort hot path.

One step = one whole sort (every level pass, the LDS finish and the host
level loop) of one resident FP64 array of n = 7,000,000 i.i.d. U[0,1) keys
(seed 4).  Distinct input copies are drawn into device memory before the
timed region, so every step sorts unsorted data that is already in HBM.

Prints ONE JSON line:
  value / ms_per_step   K whole sorts timed between two device syncs
  roofline              the stage kernel (one level pass: partition tiles and
                        LDS finish work) against the HBM peak; each launch is
                        bracketed by HIP events on the sort's stream, in a
                        second timed pass over K fresh copies
  batched               4096 arrays (log-uniform lengths in [32, 65536]) in
                        one segmented call vs 4096 plain calls vs one plain
                        sort of the same key count
  serve                 the serving workload (c4): a seeded Poisson stream
                        of 20,000 requests of 1e3 .. 1e7 keys (drawn on the
                        device before the stream), 256 in flight, through the
                        sort server (p50/p99 latency and keys/s beside the
                        plain path), then a saturation run; in a child
                        process with a time limit
  statbound             the paper's run-time model (Section 3) fitted to
                        this sort over Table 1's sizes
  worst_case            sorted, reversed, all-equal and four-valued inputs:
                        level passes and time
  large                 2^28 FP64 and 2^29 FP32 arrays: whole-sort time and the
                        stage kernel's GB/s on the passes with >= half the
                        keys live (bandwidth-bound at these sizes)
  exact                 the same 7e6 workload sorted with every partition call
                        leaving the paper's literal arrangement (the
                        sequential algorithm's calls, pivots and keys)
  cpu_baseline          the literal CPU oracle on the host, one thread
  cpu_parallel          its task-parallel driver on up to 16 host cores

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--no-extras]
                  [--copy-probe BYTES] [--exact-only] [--profile-sort WORKLOAD]
                  [--serve-only REQUESTS INFLIGHT [--serve-oracle K] [--serve-alone K]]
  (the default run's serve leg is --serve-only 20000 256 --serve-oracle 200
  --serve-alone 200)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, AMD published peak
PAPER_7E6_S = 3.2892           # Table 1: K-sort mean time at n = 7,000,000 (CPU, Turbo C++ 5.02)
KERNEL_SRC = os.path.join(ROOT, "paper_1107_3622_amd", "csrc", "ksort_kernels.h")
PMC_SUMMARY = os.path.join(ROOT, "profiles", "stage_kernel_c1_n7e6_f64_pmc.txt")


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="c1_n7e6_f64")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline leg")
    p.add_argument("--no-extras", action="store_true", help="skip the batched and serving legs")
    p.add_argument("--cpu-seconds", type=float, default=12.0)
    p.add_argument("--readings", type=int, default=50, help="sorts per size in the statistical-bound leg")
    p.add_argument("--copy-probe", type=int, default=0,
                   help="only run device copies of this many bytes (counter calibration)")
    p.add_argument("--serve-only", type=int, nargs=2, default=None, metavar=("REQUESTS", "INFLIGHT"),
                   help="run only the serving leg, at this many requests and in-flight slots")
    p.add_argument("--serve-oracle", type=int, default=6, help="requests of the serving leg checked with the oracle")
    p.add_argument("--serve-alone", type=int, default=4, help="of those, requests also served alone and compared")
    p.add_argument("--exact-only", action="store_true",
                   help="only run the literal-arrangement leg on the workload (profiling)")
    p.add_argument("--profile-sort", default=None, metavar="WORKLOAD",
                   help="only sort WORKLOAD twice (the first with per-pass key counts, printed as JSON) and "
                        "copy it three times with the streaming copy kernel, for a profiler run")
    return p.parse_args()


def kernel_sha() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def stored_traffic(variant=None):
    """HBM bytes per stage-kernel launch from the committed counter summary,
    or None when the kernel source or the variant that ran changed since the
    counters were taken."""
    try:
        text = open(PMC_SUMMARY).read()
    except OSError:
        return None, "no counter summary"
    m_sha = re.search(r"kernel_sha256:\s*([0-9a-f]{64})", text)
    m_b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m_sha or not m_b:
        return None, "counter summary incomplete"
    if m_sha.group(1) != kernel_sha():
        return None, "kernel changed since the counters were taken"
    m_v = re.search(r"variant:\s*(\d+)\s+(\d+)\s+(\d+)", text)
    if variant is not None and (not m_v or [int(x) for x in m_v.groups()] != list(variant)):
        return None, "counters were taken with another kernel variant"
    return float(m_b.group(1)), os.path.relpath(PMC_SUMMARY, ROOT)


def cpu_baseline(workload: str, budget_s: float) -> dict:
    """The literal CPU oracle, single thread, on the same workload: repeats
    whole sorts of the n-key array until about budget_s seconds are spent."""
    import numpy as np

    import oracle
    import synth
    a = synth.make(workload)
    times = []
    t_start = time.perf_counter()
    while True:
        b = a.copy()
        t0 = time.perf_counter()
        oracle.sort_(b)
        times.append(time.perf_counter() - t0)
        if time.perf_counter() - t_start >= budget_s or len(times) >= 50:
            break
    mean = float(np.mean(times))
    return {"value": a.size / mean, "unit": "keys/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(times)} whole sorts of the same {a.size}-key array (mean {mean:.3f} s each)"}


def cpu_parallel(workload: str, budget_s: float) -> dict:
    """The oracle's task-parallel driver on the host's cores (at most 16):
    the same literal calls, independent sub-arrays on different threads."""
    import numpy as np

    import oracle
    import synth
    threads = max(1, min(len(os.sched_getaffinity(0)), 16))
    a = synth.make(workload)
    times = []
    t_start = time.perf_counter()
    while True:
        b = a.copy()
        t0 = time.perf_counter()
        oracle.sort_parallel_(b, threads)
        times.append(time.perf_counter() - t0)
        if time.perf_counter() - t_start >= budget_s or len(times) >= 50:
            break
    mean = float(np.mean(times))
    return {"value": a.size / mean, "unit": "keys/s", "cores": threads, "kind": "oracle, task-parallel",
            "sample": f"{len(times)} whole sorts of the same {a.size}-key array (mean {mean:.3f} s each)"}


def copy_probe(nbytes: int) -> int:
    """Copies of a known size with the library's streaming copy kernel, for
    scaling the memory counters: FETCH_SIZE and WRITE_SIZE of one copy should
    read nbytes each."""
    import torch

    from paper_1107_3622_amd import ksort
    n = nbytes // 8
    a = torch.empty(n, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(5):
        ksort.ksort_stream_copy(b, a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 8, "copies": 5}), flush=True)
    return 0


def profile_sort(workload: str) -> int:
    """One warm-up sort, one sort with per-pass key counts, one plain sort
    and three streaming copies of the same array: the dispatches a profiler
    run joins with these counts, pass by pass."""
    import torch

    import synth
    from paper_1107_3622_amd import ksort
    w = synth.WORKLOADS[workload]
    src = synth.torch_fill(w["kind"], w["seed"], w["n"], torch.device("cuda:0"))
    sort_fn = ksort.ksort_f64 if src.dtype == torch.float64 else ksort.ksort_f32
    kb = src.element_size()
    t = src.clone()
    log(f"profile-sort {workload}: input drawn")
    sort_fn(t)  # warm-up: workspace
    t.copy_(src)
    torch.cuda.synchronize()
    log("profile-sort: warm-up sort done")
    ksort.ksort_profile_read()
    ksort.ksort_profile_enable(True)
    sort_fn(t)
    ksort.ksort_profile_enable(False)
    recs = ksort.ksort_profile_read()
    t.copy_(src)
    torch.cuda.synchronize()
    log("profile-sort: counted sort done")
    sort_fn(t)
    torch.cuda.synchronize()
    log("profile-sort: plain sort done")
    ok = bool(torch.equal(t, torch.sort(src)[0]))
    log("profile-sort: checked against torch.sort")
    dst = torch.empty_like(src)
    for _ in range(3):
        ksort.ksort_stream_copy(dst, src)
    torch.cuda.synchronize()
    log("profile-sort: copies done")
    print(json.dumps({"workload": workload, "n": w["n"], "key_bytes": kb, "verified": ok,
                      "passes": [{"stage": r["stage"], "live_keys": r["live_keys"], "finish_keys": r["finish_keys"],
                                  "alg_bytes": 2 * kb * (r["live_keys"] + r["finish_keys"]), "event_ms": r["ms"]}
                                 for r in recs],
                      "copy_bytes": 2 * kb * w["n"], "copies": 3}), flush=True)
    return 0 if ok else 3


def batched_leg(ksort, torch) -> dict:
    """The batched workload (4096 arrays, lengths log-uniform in [32, 65536]
    from seed 9, keys from seed 10): one segmented call with the untuned
    default variant, then with the variant the autotuner picks for this
    batch (persisted in a JSON tuning file), vs 4096 plain calls and one
    plain sort of the same key count."""
    import tempfile

    import synth
    keys, offs = synth.batched(9, 10, 4096, 32, 65536)
    n = int(offs[-1])
    src = torch.from_numpy(keys).to("cuda")
    d_offs = torch.from_numpy(offs).to("cuda")
    ref = src.clone()
    reps = 5
    copies = [src.clone() for _ in range(2 * reps + 2)]
    torch.cuda.synchronize()

    def timed(first: int) -> float:
        for c in copies[first:first + reps + 1]:
            c.copy_(src)
        ksort.ksort_segmented(copies[first], d_offs, want_pivots=False)  # records the graph
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(reps):
            ksort.ksort_segmented(copies[first + 1 + k], d_offs, want_pivots=False)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    ksort.ksort_tune_file(None)  # untuned defaults
    default_variant = ksort.ksort_get_default(ksort.KSORT_F64)
    tune_path = os.path.join(tempfile.mkdtemp(prefix="ksort_tune_"), "tune.json")
    ksort.ksort_tune_file(tune_path)
    tuned = ksort.ksort_autotune_batch(src, d_offs)
    with open(tune_path) as f:
        tune_json = json.load(f)
    # the untuned default and the tuned choice timed in turn, three times
    # each (medians), so that drift between the two timings cancels
    t_default, t_tuned = [], []
    for _ in range(3):
        ksort.ksort_tune_file(None)
        t_default.append(timed(0))
        ksort.ksort_tune_file(tune_path)
        t_tuned.append(timed(reps + 1))
    seg_default_s = sorted(t_default)[1]
    seg_s = sorted(t_tuned)[1]
    # correctness: stable sort by key, then stable sort by array index
    seg_id = torch.repeat_interleave(torch.arange(4096, device="cuda"), d_offs[1:] - d_offs[:-1])
    v, idx = torch.sort(ref, stable=True)
    _, idx2 = torch.sort(seg_id[idx], stable=True)
    ok = all(torch.equal(c, v[idx2]) for c in copies)
    # plain loop: one ksort_f64 call per array on views of the packed buffer
    loop = src.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for u in range(4096):
        ksort.ksort_f64(loop[int(offs[u]):int(offs[u + 1])])
    torch.cuda.synchronize()
    loop_s = time.perf_counter() - t0
    ok = ok and torch.equal(loop, v[idx2])
    # one plain sort of the same key count
    one = synth.torch_fill("uniform_f64", 10, n, "cuda")
    ones = [one.clone() for _ in range(reps + 1)]
    ksort.ksort_f64(ones[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(reps):
        ksort.ksort_f64(ones[1 + k])
    torch.cuda.synchronize()
    one_s = (time.perf_counter() - t0) / reps
    ksort.ksort_tune_file(None)
    return {"arrays": 4096, "keys": n, "segmented_keys_per_s": n / seg_s, "segmented_ms": seg_s * 1e3,
            "tuned_variant": list(tuned), "default_variant": list(default_variant),
            "segmented_default_ms": seg_default_s * 1e3, "tuned_gain": seg_default_s / seg_s,
            "tuned_is_default": list(tuned) == list(default_variant),
            "tune_file_entries": tune_json["entries"],
            "plain_loop_keys_per_s": n / loop_s, "plain_loop_ms": loop_s * 1e3,
            "one_plain_sort_keys_per_s": n / one_s, "one_plain_sort_ms": one_s * 1e3,
            "verified": bool(ok)}


def _plain_rate(ksort, torch, sizes, kinds, sample: int) -> float:
    """Keys/s of the plain single-array path over the first `sample`
    requests of the stream, one call per request, inputs resident."""
    import synth
    total_keys, total_s = 0, 0.0
    for r in range(min(sample, len(sizes))):
        t = synth.torch_fill(kinds[r], synth.REQUEST_SEED_BASE + r, int(sizes[r]), "cuda")
        fn = ksort.ksort_f64 if t.dtype == torch.float64 else ksort.ksort_f32
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn(t)
        total_s += time.perf_counter() - t0
        total_keys += int(sizes[r])
        del t
    return total_keys / total_s


SERVE_REQUESTS = 160
SERVE_INFLIGHT = 128


def serve_leg(ksort, torch, count: int = SERVE_REQUESTS, inflight: int = SERVE_INFLIGHT,
              oracle_checks: int = 6, alone_checks: int = 4, plain_sample: int = 400) -> dict:
    """The serving workload: a seeded Poisson stream (arrivals seed 11) of
    `count` requests with sizes log-uniform in [1e3, 1e7] (seed 12), 70 %
    FP64 (seed 13), `inflight` in flight under a 64 GiB budget; lambda = 0.7
    x the plain path's keys/s on the first `plain_sample` requests / E[n].
    Every request's keys are drawn on the device before the server starts
    and each is submitted at its arrival time.  After the stream every result
    is compared with torch.sort of its input; `oracle_checks` requests
    (evenly spread, the three largest among them) with the oracle and their
    first pivots, and `alone_checks` of them with their results when served
    alone.  Then a saturation run: the same requests all submitted at t = 0."""
    import numpy as np

    import oracle
    import synth
    lo, hi, p64 = 1_000, 10_000_000, 0.7
    sizes, is_f64, _ = synth.serve_requests(count, 12, 13, 11, lo, hi, p64, 1.0)
    kinds = ["uniform_f64" if f else "uniform_f32" for f in is_f64]
    e_n = (hi - lo) / (np.log(hi) - np.log(lo))  # mean of the log-uniform size
    plain = _plain_rate(ksort, torch, sizes, kinds, plain_sample)
    lam = 0.7 * plain / e_n
    _, _, arrivals = synth.serve_requests(count, 12, 13, 11, lo, hi, p64, lam)
    keys = int(sizes.sum())
    deadline_s = 120.0 + 4.0 * arrivals[-1]

    def draw():
        ts = [synth.torch_fill(kinds[r], synth.REQUEST_SEED_BASE + r, int(sizes[r]), "cuda") for r in range(count)]
        torch.cuda.synchronize()
        return ts

    def wait_all(srv, tks, t0):
        codes = []
        for tk in tks:
            left = max(1.0, deadline_s - (time.perf_counter() - t0))
            codes.append(srv.wait(tk, left))
        return codes

    log(f"serve: {count} requests, {keys} keys; plain path {plain / 1e9:.2f} G keys/s; lambda {lam:.0f}/s; "
        f"{inflight} in flight")
    tensors = draw()
    tickets = []
    with ksort.Server(64 << 30, inflight) as srv:
        t0 = time.perf_counter()
        for r in range(count):
            dt = arrivals[r] - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            tickets.append(srv.submit(tensors[r]))
        codes = wait_all(srv, tickets, t0)
        wall = time.perf_counter() - t0
        st = srv.stats()
        infos = [srv.result(tk) for tk in tickets]
    ok = all(c == 0 for c in codes)
    log(f"serve: stream done in {wall:.2f} s, {st['completed']} completed; checking against torch.sort")
    n_equal = 0
    for r in range(count):
        ref = torch.sort(synth.torch_fill(kinds[r], synth.REQUEST_SEED_BASE + r, int(sizes[r]), "cuda"))[0]
        n_equal += int(bool(torch.equal(tensors[r], ref)))
    ok = ok and n_equal == count
    order = np.argsort(sizes)
    spread = np.linspace(0, count - 1, max(1, oracle_checks - 3)).astype(int).tolist()
    sample = sorted(set(spread + [int(x) for x in order[-3:]]))[:max(oracle_checks, 1)]
    n_oracle = 0
    for r in sample:
        a = (synth.uniform_f64 if is_f64[r] else synth.uniform_f32)(synth.REQUEST_SEED_BASE + r, int(sizes[r]))
        want, wp = oracle.sorted_copy(a)
        got = tensors[r].cpu().numpy()
        n_oracle += int(np.array_equal(got.view(np.uint8), want.view(np.uint8)) and infos[r]["first_pivot"] == wp)
    ok = ok and n_oracle == len(sample)
    # the first alone_checks requests of the sample, each served alone
    n_alone = 0
    with ksort.Server(64 << 30, inflight) as srv:
        for r in sample[:alone_checks]:
            t = synth.torch_fill(kinds[r], synth.REQUEST_SEED_BASE + r, int(sizes[r]), "cuda")
            tk = srv.submit(t)
            c = srv.wait(tk, 60.0)
            n_alone += int(c == 0 and bool(torch.equal(t, tensors[r])) and
                           srv.result(tk)["first_pivot"] == infos[r]["first_pivot"])
            del t
    ok = ok and n_alone == min(alone_checks, len(sample))
    del tensors
    torch.cuda.empty_cache()
    log("serve: saturation run")
    pre = draw()
    with ksort.Server(64 << 30, inflight) as srv:
        t0 = time.perf_counter()
        tks = [srv.submit(t) for t in pre]
        sat_codes = wait_all(srv, tks, t0)
        sat_wall = time.perf_counter() - t0
        sat = srv.stats()
    ok = ok and all(c == 0 for c in sat_codes)
    del pre
    torch.cuda.empty_cache()
    return {"workload": f"c4: {count} requests, Poisson arrivals (seed 11), sizes log-uniform [1e3, 1e7] "
                        f"(seed 12), 70 % FP64 (seed 13), keys of request r from seed 1,000,000 + r drawn on the "
                        f"device before the stream, {inflight} in flight, 64 GiB budget",
            "requests": count, "inflight": inflight, "keys": keys, "lambda_per_s": lam,
            "plain_keys_per_s_on_mix": plain, "plain_sample_requests": min(plain_sample, count),
            "wall_s": wall, "keys_per_s": keys / wall,
            "keys_per_busy_s": keys / st["busy_s"] if st["busy_s"] > 0 else None,
            "p50_latency_s": st["p50_latency_s"], "p99_latency_s": st["p99_latency_s"],
            "mean_latency_s": st["mean_latency_s"], "ticks": st["ticks"],
            "completed": st["completed"], "failed": st["failed"],
            "saturation": {"workload": "the same requests, all submitted at t = 0",
                           "wall_s": sat_wall, "keys_per_s": keys / sat_wall,
                           "p50_latency_s": sat["p50_latency_s"], "p99_latency_s": sat["p99_latency_s"],
                           "ticks": sat["ticks"], "completed": sat["completed"]},
            "equal_to_torch_sort": n_equal, "oracle_checked": len(sample), "oracle_equal": n_oracle,
            "alone_checked": min(alone_checks, len(sample)), "alone_equal": n_alone, "verified": bool(ok)}


SERVE_C4 = (20_000, 256, 200, 200)  # requests, in flight, oracle checks, alone checks


def serve_in_child(torch, timeout_s: float = 900.0) -> dict:
    """The serving leg at its configuration (20,000 requests, 256 in
    flight) in a child process with a time limit, so that a server that
    stops making progress costs this leg, not the whole run."""
    import subprocess
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    count, inflight, n_or, n_al = SERVE_C4
    cmd = [sys.executable, "-u", os.path.abspath(__file__), "--serve-only", str(count), str(inflight),
           "--serve-oracle", str(n_or), "--serve-alone", str(n_al)]
    try:
        r = subprocess.run(cmd, stdout=subprocess.PIPE, timeout=timeout_s, text=True)
    except subprocess.TimeoutExpired:
        return {"error": f"the serving leg did not finish within {timeout_s:.0f} s", "verified": False}
    lines = [x for x in r.stdout.strip().splitlines() if x.startswith("{")]
    if not lines:
        return {"error": f"the serving leg exited with status {r.returncode} and no result", "verified": False}
    res = json.loads(lines[-1])["serve"]
    if r.returncode != 0:
        res["verified"] = False
    return res


TABLE1_N = [100_000, 500_000, 1_000_000, 2_500_000, 5_000_000, 6_000_000, 7_000_000, 7_100_000, 7_500_000,
            10_000_000]


def statbound_leg(ksort, torch, readings: int) -> dict:
    """The paper's statistical-bound model (Section 3) fitted to this sort:
    mean time of `readings` sorts of fresh U[0,1) FP64 arrays at each size of
    Table 1, then the OLS fit of y = b0 + b1 n log2 n + b2 n."""
    import synth
    from paper_1107_3622_amd import statbound
    means = []
    for i, n in enumerate(TABLE1_N):
        src = synth.torch_fill("uniform_f64", 100 + i, n, "cuda")
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(readings)]
        t = src.clone()
        ksort.ksort_f64(t)  # warm
        for r in range(readings):
            t.copy_(src)
            ev[r][0].record()
            ksort.ksort_f64(t)
            ev[r][1].record()
        torch.cuda.synchronize()
        means.append(sum(a.elapsed_time(b) for a, b in ev) / readings / 1e3)
        del src, t
    fr = statbound.ols(TABLE1_N, means)
    log("statistical bound of the GPU sort (seconds):\n" + statbound.report(fr, "y(GPU)"))
    return {"n": TABLE1_N, "mean_s": means, "readings": readings,
            "coef": [float(c) for c in fr.coef], "se": [float(x) for x in fr.se], "t": [float(x) for x in fr.t],
            "p": [float(x) for x in fr.p], "r2": fr.r2, "r2_adj": fr.r2_adj, "r2_pred": fr.r2_pred, "s": fr.s,
            "f": fr.f, "seq_ss": [float(x) for x in fr.seq_ss], "large_residuals": fr.large}


def worstcase_leg(ksort, torch, n: int = 16_384) -> dict:
    """K-sort's worst cases at n keys: ordered inputs and heavy duplicates
    make each partition peel off one key, so the level passes grow to about
    n and the work to about n^2 / 2 key moves (no change to the key rule)."""
    import numpy as np

    import synth
    u = synth.uniform_f64(901, n)
    kinds = {"random": u, "sorted": np.sort(u), "reversed": np.sort(u)[::-1].copy(),
             "all_equal": np.full(n, 0.5), "four_values": np.floor(synth.uniform_f64(902, n) * 4.0) / 4.0}
    out = {}
    for name, a in kinds.items():
        src = torch.from_numpy(a).to("cuda")
        t = src.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ksort.ksort_f64(t)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        t2 = src.clone()
        ksort.ksort_profile_read()
        ksort.ksort_profile_enable(True)
        ksort.ksort_f64(t2)
        ksort.ksort_profile_enable(False)
        recs = ksort.ksort_profile_read()
        levels = sum(1 for r in recs if r["live_keys"] + r["finish_keys"] > 0)
        ok = bool(torch.equal(t, torch.sort(src)[0]))
        out[name] = {"ms": dt * 1e3, "levels": levels, "launches": len(recs), "verified": ok}
    return {"n": n, "inputs": out}


def exact_leg(ksort, torch, src, reps: int = 3) -> dict:
    """Whole sorts in the literal arrangement: every call, its key and its
    pivot index are the sequential algorithm's; the call count and the first
    pivot are reported with the time."""
    ref = torch.sort(src)[0]
    best = None
    ok = True
    for _ in range(reps):
        t = src.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fp, ncalls, _ = ksort.ksort_sort_exact(t)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
        ok = ok and bool(torch.equal(t, ref))
    n = src.numel()
    return {"n": n, "ms": best * 1e3, "keys_per_s": n / best, "calls": ncalls, "first_pivot": fp,
            "runs": reps, "verified": ok}


def copy_ceiling(ksort, torch, dst, src, reps: int) -> float:
    """Read + write GB/s of the library's streaming copy kernel
    (ksort_stream_copy) over the same bytes as one pass over src."""
    ksort.ksort_stream_copy(dst, src)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(reps):
        ksort.ksort_stream_copy(dst, src)
    c1.record()
    torch.cuda.synchronize()
    return reps * 2 * src.numel() * src.element_size() / (c0.elapsed_time(c1) * 1e-3) / 1e9


def large_leg(ksort, torch, reps: int = 2) -> dict:
    """The large single arrays (2^28 FP64, 2^29 FP32): whole-sort time, and
    the stage kernel's algorithmic GB/s on the passes with at least half of
    the keys live, each launch bracketed by HIP events."""
    import synth
    out = {}
    for name in ("c2_n2^28_f64", "c2_n2^29_f32"):
        w = synth.WORKLOADS[name]
        n = w["n"]
        src = synth.torch_fill(w["kind"], w["seed"], n, torch.device("cuda:0"))
        kb = src.element_size()
        sort_fn = ksort.ksort_f64 if kb == 8 else ksort.ksort_f32
        ref = torch.sort(src)[0]
        t = src.clone()
        sort_fn(t)  # warm-up: grows the workspace
        ok = bool(torch.equal(t, ref))
        best = None
        for _ in range(reps):
            t.copy_(src)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sort_fn(t)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
            ok = ok and bool(torch.equal(t, ref))
        t.copy_(src)
        ksort.ksort_profile_read()
        ksort.ksort_profile_enable(True)
        torch.cuda.synchronize()
        sort_fn(t)
        torch.cuda.synchronize()
        ksort.ksort_profile_enable(False)
        recs = ksort.ksort_profile_read()
        ok = ok and bool(torch.equal(t, ref))
        pass_bytes = [2 * kb * (r["live_keys"] + r["finish_keys"]) for r in recs]
        big = [r for r in recs if r["live_keys"] >= n // 2]
        big_bytes = sum(2 * kb * (r["live_keys"] + r["finish_keys"]) for r in big)
        big_ms = sum(r["ms"] for r in big)
        gbs = big_bytes / (big_ms * 1e-3) / 1e9 if big_ms > 0 else None
        # every pass that moves at least 512 MB (twice the Infinity Cache):
        # its own fraction of the HBM peak
        fr = sorted(b / (r["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS
                    for b, r in zip(pass_bytes, recs) if b >= 512 * 2**20 and r["ms"] > 0)
        tot_ms = sum(r["ms"] for r in recs)
        agg = sum(pass_bytes) / (tot_ms * 1e-3) / 1e9 if tot_ms > 0 else None
        out[name] = {"n": n, "ms": best * 1e3, "keys_per_s": n / best, "levels": len(recs),
                     "full_passes": len(big), "full_pass_avg_ms": big_ms / max(len(big), 1),
                     "full_passes_gbs": gbs, "full_passes_frac": gbs / HBM_PEAK_GBS if gbs else None,
                     "passes_ge_512MB": {"count": len(fr), "frac_min": fr[0] if fr else None,
                                         "frac_median": fr[len(fr) // 2] if fr else None,
                                         "frac_max": fr[-1] if fr else None},
                     "all_passes_gbs": agg, "all_passes_frac": agg / HBM_PEAK_GBS if agg else None,
                     "verified": ok}
        # the library's streaming copy of the same array: the read + write
        # rate a pass-shaped streaming kernel reaches on this GPU (the ceiling)
        copy_gbs = copy_ceiling(ksort, torch, t, src, 5)
        out[name]["copy_gbs"] = copy_gbs
        out[name]["copy_kernel"] = "ksort_stream_copy"
        out[name]["full_passes_of_copy"] = gbs / copy_gbs if gbs else None
        out[name]["passes_ge_512MB"]["frac_of_copy_median"] = (
            fr[len(fr) // 2] * HBM_PEAK_GBS / copy_gbs if fr else None)
        del src, ref, t
        torch.cuda.empty_cache()
    return out


def main() -> int:
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        return 2
    import torch

    import synth
    from paper_1107_3622_amd import ksort

    ksort.load()
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no HIP device"}), flush=True)
        return 1
    if args.copy_probe:
        return copy_probe(args.copy_probe)
    if args.profile_sort:
        return profile_sort(args.profile_sort)
    if args.serve_only:
        count, inflight = args.serve_only
        res = serve_leg(ksort, torch, count, inflight, oracle_checks=args.serve_oracle,
                        alone_checks=args.serve_alone)
        print(json.dumps({"serve": res}), flush=True)
        return 0 if res["verified"] else 3
    if args.exact_only:
        w = synth.WORKLOADS[args.workload]
        res = exact_leg(ksort, torch, synth.torch_fill(w["kind"], w["seed"], w["n"], torch.device("cuda:0")))
        print(json.dumps({"exact": res, "workload": args.workload}), flush=True)
        return 0 if res["verified"] else 3
    dev = torch.device("cuda:0")
    w = synth.WORKLOADS[args.workload]
    n = w["n"]
    assert w["kind"] in ("uniform_f64", "grid16_f64", "uniform_f32")
    log(f"workload {args.workload} n={n}; drawing {2 * args.steps + args.warmup} copies on the device")
    src = synth.torch_fill(w["kind"], w["seed"], n, dev)
    sort_fn = ksort.ksort_f64 if src.dtype == torch.float64 else ksort.ksort_f32
    key_bytes = src.element_size()
    copies = [src.clone() for _ in range(2 * args.steps + args.warmup)]
    torch.cuda.synchronize()

    for k in range(args.warmup):
        sort_fn(copies[k])
    torch.cuda.synchronize()
    log("warmup done")

    # timed region: K whole sorts; per-call HIP events give the spread
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record()
        sort_fn(copies[args.warmup + k])
        ev[k][1].record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    per_call = sorted(a.elapsed_time(b) for a, b in ev)
    log(f"timed {args.steps} steps in {elapsed:.4f} s")

    # second pass over fresh copies: every stage launch bracketed by HIP
    # events on the sort's stream (the current stream)
    ksort.ksort_profile_read()
    ksort.ksort_profile_enable(True)
    torch.cuda.synchronize()
    for k in range(args.steps):
        sort_fn(copies[args.warmup + args.steps + k])
    torch.cuda.synchronize()
    ksort.ksort_profile_enable(False)
    recs = ksort.ksort_profile_read()

    # roofline of the stage kernel: algorithmic bytes are 2 * key_bytes per
    # key partitioned plus 2 * key_bytes per key finished
    tot_ms = sum(r["ms"] for r in recs)
    tot_bytes = sum(2 * key_bytes * (r["live_keys"] + r["finish_keys"]) for r in recs)
    launches = len(recs)
    achieved = tot_bytes / (tot_ms * 1e-3) / 1e9 if tot_ms > 0 else 0.0
    big = [r for r in recs if 2 * key_bytes * r["live_keys"] >= 0.5 * 2 * key_bytes * n]
    big_gbs = (sum(2 * key_bytes * (r["live_keys"] + r["finish_keys"]) for r in big) /
               (sum(r["ms"] for r in big) * 1e-3) / 1e9) if big else None
    ran = [recs[0]["block"], recs[0]["items"], recs[0]["cutoff"]] if recs else None
    traffic, traffic_src = stored_traffic(ran)

    # the read + write rate of the library's streaming copy of the same
    # array (the practical ceiling of one pass at this size)
    dst = torch.empty_like(src)
    copy_gbs = copy_ceiling(ksort, torch, dst, src, 20)
    del dst

    # correctness of the timed outputs: equal to the library sort of torch
    ref = torch.sort(src.clone())[0]
    ok = all(torch.equal(copies[args.warmup + k], ref) for k in range(2 * args.steps))

    value = n * args.steps / elapsed
    q = lambda p: per_call[min(len(per_call) - 1, int(round(p * (len(per_call) - 1))))]
    out = {
        "metric": "sorted keys/s FP64 n=7e6 (+HBM GB/s/pass); batched vs plain; serve p50/p99",
        "value": value,
        "unit": "keys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        # the paper's own K-sort time at this n (Table 1; CPU, another machine): context
        "vs_baseline": value / (7_000_000 / PAPER_7E6_S) if args.workload == "c1_n7e6_f64" else None,
        "dtype": "f64" if key_bytes == 8 else "f32",
        "data": "synthetic: SplitMix64 U[0,1) keys drawn on the device",
        "config": {"workload": f"{args.workload}: n={n} {w['kind']} seed {w['seed']}, one array per call",
                   "variant": ([recs[0]["block"], recs[0]["items"], recs[0]["cutoff"]] if recs else
                               list(ksort.ksort_get_default(0 if key_bytes == 8 else 1)))},
        "per_call_ms": {"p10": q(0.1), "median": q(0.5), "p90": q(0.9)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "traffic_source": traffic_src,
                     "kernel": "stage_kernel (one level pass: partition tiles + LDS finish)",
                     "launches": launches, "avg_launch_ms": tot_ms / max(launches, 1),
                     "alg_bytes_per_launch": tot_bytes / max(launches, 1),
                     "full_passes_gbs": big_gbs, "full_passes": len(big),
                     "copy_gbs": copy_gbs, "copy_kernel": "ksort_stream_copy",
                     "full_passes_of_copy": big_gbs / copy_gbs if big_gbs else None,
                     "timing": "HIP events around every stage launch, second pass over fresh copies"},
        "levels_per_sort": launches / max(args.steps, 1),
        "partition_passes_per_key": sum(r["live_keys"] for r in recs) / (n * args.steps),
        "verified_sorted_equal_torch_sort": ok,
        "paper_table1_keys_per_s_n7e6": 7_000_000 / PAPER_7E6_S,
    }
    if not args.no_extras:
        log("batched leg")
        out["batched"] = batched_leg(ksort, torch)
        log("serving leg (child process)")
        out["serve"] = serve_in_child(torch)
        log("statistical-bound leg")
        out["statbound"] = statbound_leg(ksort, torch, args.readings)
        log("worst-case leg")
        out["worst_case"] = worstcase_leg(ksort, torch)
        ok = ok and all(v["verified"] for v in out["worst_case"]["inputs"].values())
        log("large-array leg")
        out["large"] = large_leg(ksort, torch)
        ok = ok and all(v["verified"] for v in out["large"].values())
        log("exact-arrangement leg")
        out["exact"] = exact_leg(ksort, torch, synth.torch_fill(w["kind"], w["seed"], n, dev))
        ok = ok and out["exact"]["verified"]
        ok = ok and out["batched"]["verified"] and out["serve"]["verified"]
    if not args.no_cpu:
        log("timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_seconds)
        log("timing the task-parallel CPU oracle")
        out["cpu_parallel"] = cpu_parallel(args.workload, args.cpu_seconds / 3)
    print(json.dumps(out), flush=True)
    return 0 if ok else 3


if __name__ == "__main__":
    sys.exit(main())
