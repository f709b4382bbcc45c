"""Checks that pin the CPU oracle to facts fixed by the paper or by
mathematics, independent of the oracle's own code.

Each check takes a loaded oracle library (so that the mutation tests can run
the same checks against deliberately broken copies of the oracle) and returns
a list of failure strings; an empty list means the pin holds.

Sources of truth:
  * illustration  - arXiv 1107.3622, Section 1.2 table (tests/golden)
  * closed forms  - the key's final index is left + #{x : key > a[x]};
                    the one-level arrangement (derived from Steps 1-4 by
                    following the two scan pointers; written out below)
  * brute force   - every permutation of n <= 8 and every small multiset:
                    output sorted, a permutation of the input, partition
                    property after every call, right-left comparisons per call
  * Knuth's mean  - over all n! orders of distinct keys, the mean total number
                    of comparisons of first-element Quick sort is
                    2(n+1)H_n - 4n (Knuth, TAOCP vol. 3, 5.2.2), cited by the
                    paper for K-sort's average case (Section 1)
  * library sort  - numpy's sort gives the same array, bit for bit
"""
from __future__ import annotations

import itertools
import os
from fractions import Fraction

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "illustration.txt")


def load_illustration() -> list[tuple[str, list[float], str]]:
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            label, keys, temp = (s.strip() for s in line.split("|"))
            rows.append((label, [float(x) for x in keys.split()], temp))
    return rows


# ---------------------------------------------------------------- closed forms

def closed_form_pivot(a: np.ndarray, left: int, right: int) -> int:
    key = a[left]
    seg = a[left + 1:right + 1]
    return left + int(np.count_nonzero(~(key <= seg)))


def closed_form_arrangement(a: np.ndarray, left: int, right: int) -> np.ndarray:
    """The array after one partition call, derived without running the steps.

    With key = a[left], c = #{x in (left, right] : key > a[x]} and i = left + c:
      * m = i + 1 if i < right and a[i+1] >= key, else m = i;
      * q_1 < q_2 < ... are the positions in (left, m] holding a key >= key,
        r_1 > r_2 > ... the positions in (m, right] holding a key < key;
    the steps move the key to i, a[q_1] (the temp) to i + 1, every smaller key
    at a position x <= m to x - 1, leave every larger-or-equal key at x > m
    where it is, move a[q_k] to r_{k-1} (k >= 2) and a[r_k] to q_k - 1.
    """
    b = a.copy()
    key = a[left]
    i = closed_form_pivot(a, left, right)
    m = i + 1 if (i < right and key <= a[i + 1]) else i
    q = [x for x in range(left + 1, m + 1) if key <= a[x]]
    r = [x for x in range(right, m, -1) if not (key <= a[x])]
    b[i] = key
    if q:
        b[i + 1] = a[q[0]]
    for x in range(left + 1, m + 1):
        if not (key <= a[x]):
            b[x - 1] = a[x]
    for k in range(1, len(q)):
        b[r[k - 1]] = a[q[k]]
    for k in range(len(r)):
        b[q[k] - 1] = a[r[k]]
    return b


# ---------------------------------------------------------------- individual pins

def check_illustration(lib) -> list[str]:
    """Section 1.2: rows 1-3 exactly, the final order exactly; the row printed
    for key 66 disagrees with the steps (the paper's hand trace swaps 75 and
    78), so for it only the key, its index and the temp are compared; the
    steps' own call on [7, 9] (key 75) is absent from the table; the row for
    key 78 matches in full."""
    fails = []
    rows = load_illustration()
    a = np.array(rows[0][1], dtype=np.float64)
    info = oracle.sort_(a.copy(), trace_cap=16, lib=lib)
    tr = info["trace"]
    if info["first_pivot"] != 4:
        fails.append(f"illustration: first pivot {info['first_pivot']} != 4")
    if info["comparisons"] != 20:
        fails.append(f"illustration: {info['comparisons']} comparisons != 20")
    expect_ranges = [(0, 9), (0, 3), (2, 3), (5, 9), (7, 9), (8, 9)]
    got_ranges = [(t["left"], t["right"]) for t in tr]
    if got_ranges != expect_ranges:
        fails.append(f"illustration: call ranges {got_ranges} != {expect_ranges}")
        return fails
    # Replay the calls one at a time to see the array after each.
    b = a.copy()
    states, temps = [], []
    for (lft, rgt) in expect_ranges:
        _, rec = oracle.partition_(b, lft, rgt, lib=lib)
        states.append(b.copy())
        temps.append(rec["temp"] if rec["flag"] else None)
    by_label = {lbl: (keys, temp) for lbl, keys, temp in rows}
    for call, label in ((0, "key=55"), (1, "key=8"), (2, "key=50"), (5, "key=78")):
        keys, temp = by_label[label]
        if list(states[call]) != keys:
            fails.append(f"illustration {label}: {list(states[call])} != {keys}")
        want_t = None if temp == "Nil" else float(temp)
        if temps[call] != want_t:
            fails.append(f"illustration {label}: temp {temps[call]} != {want_t}")
    keys66, temp66 = by_label["key=66"]
    if states[3][6] != 66 or keys66[6] != 66 or temps[3] != float(temp66):
        fails.append("illustration key=66: key index or temp differ")
    if list(states[3][:7]) != keys66[:7] or states[3][9] != keys66[9]:
        fails.append("illustration key=66: positions outside the 75/78 swap differ")
    if list(states[-1]) != by_label["sorted"][0]:
        fails.append("illustration: final order differs")
    return fails


def _check_tree(a: np.ndarray, lib, fails: list[str], tag: str) -> None:
    """Run the recursion of Steps 5-6 from Python, one oracle partition call at
    a time, checking each call against the closed forms and the partition
    property; then compare with the oracle's own driver."""
    orig = a.copy()
    b = a.copy()
    stack = [(0, len(b) - 1)] if len(b) >= 2 else []
    ncalls = 0
    while stack:
        left, right = stack.pop()
        before = b.copy()
        i, rec = oracle.partition_(b, left, right, lib=lib)
        ncalls += 1
        if i != closed_form_pivot(before, left, right):
            fails.append(f"{tag}: pivot {i} != closed form on [{left},{right}]")
            return
        if rec["comparisons"] != right - left:
            fails.append(f"{tag}: {rec['comparisons']} comparisons != {right - left}")
            return
        if rec["k_minus_i"] != 1:
            fails.append(f"{tag}: k - i = {rec['k_minus_i']} at exit")
            return
        key = before[left]
        if not (np.all(b[left:i] < key) and b[i] == key and np.all(key <= b[i + 1:right + 1])):
            fails.append(f"{tag}: partition property fails on [{left},{right}]")
            return
        if not np.array_equal(b, closed_form_arrangement(before, left, right)):
            fails.append(f"{tag}: arrangement differs from the closed form on [{left},{right}]")
            return
        if right > i + 1:
            stack.append((i + 1, right))
        if left < i - 1:
            stack.append((left, i - 1))
    c = orig.copy()
    info = oracle.sort_(c, lib=lib)
    if not np.array_equal(c, b):
        fails.append(f"{tag}: driver output differs from the call-by-call replay")
    if not np.array_equal(c, np.sort(orig)):
        fails.append(f"{tag}: output is not the sorted input")
    if info["calls"] != ncalls:
        fails.append(f"{tag}: driver made {info['calls']} calls, replay {ncalls}")
    if len(orig) >= 2 and info["first_pivot"] != closed_form_pivot(orig, 0, len(orig) - 1):
        fails.append(f"{tag}: first pivot differs from the closed form")


def check_permutations(lib, nmax: int = 8, stop_after: int = 1) -> list[str]:
    """Every permutation of 0..n-1 for n = 1..nmax."""
    fails: list[str] = []
    for n in range(1, nmax + 1):
        for perm in itertools.permutations(range(n)):
            _check_tree(np.array(perm, dtype=np.float64), lib, fails, f"perm{perm}")
            if len(fails) >= stop_after:
                return fails
    return fails


def check_multisets(lib, spec=((3, 9), (4, 7)), stop_after: int = 1) -> list[str]:
    """Every sequence over {0..v-1} of length <= nmax, for (v, nmax) in spec:
    duplicates of the key must go right."""
    fails: list[str] = []
    for v, nmax in spec:
        for n in range(2, nmax + 1):
            for seq in itertools.product(range(v), repeat=n):
                _check_tree(np.array(seq, dtype=np.float64), lib, fails, f"seq{seq}")
                if len(fails) >= stop_after:
                    return fails
    return fails


def knuth_mean_comparisons(n: int) -> Fraction:
    h = sum(Fraction(1, k) for k in range(1, n + 1))
    return 2 * (n + 1) * h - 4 * n


def check_mean_comparisons(lib, nmax: int = 8) -> list[str]:
    fails = []
    for n in range(2, nmax + 1):
        total, count = 0, 0
        for perm in itertools.permutations(range(n)):
            info = oracle.sort_(np.array(perm, dtype=np.float64), lib=lib)
            total += info["comparisons"]
            count += 1
        mean = Fraction(total, count)
        if mean != knuth_mean_comparisons(n):
            fails.append(f"mean comparisons n={n}: {mean} != {knuth_mean_comparisons(n)}")
    return fails


def check_library_sort(lib, sizes=(2, 3, 17, 1000, 65_537, 200_000), seed0: int = 100) -> list[str]:
    import synth
    fails = []
    for s, n in enumerate(sizes):
        for name, a in (("f64", synth.uniform_f64(seed0 + s, n)),
                        ("f32", synth.uniform_f32(seed0 + s, n)),
                        ("grid", synth.grid16_f64(seed0 + s, n))):
            b, fp = oracle.sorted_copy(a, lib=lib)
            if not np.array_equal(b.view(np.uint8), np.sort(a).view(np.uint8)):
                fails.append(f"library sort {name} n={n}: differs from numpy")
            if fp != closed_form_pivot(a, 0, n - 1):
                fails.append(f"library sort {name} n={n}: first pivot differs from closed form")
    return fails


def check_levels_and_batches(lib) -> list[str]:
    """partition_level and segmented agree with the single-array entry points."""
    import synth
    fails = []
    a = synth.uniform_f64(77, 5000)
    left = np.array([0, 10, 2000, 4999], dtype=np.int64)
    length = np.array([10, 1990, 2999, 1], dtype=np.int64)
    b = a.copy()
    piv = oracle.partition_level_(b, left, length, lib=lib)
    for s in range(left.size):
        lft, rgt = int(left[s]), int(left[s] + length[s] - 1)
        if piv[s] != closed_form_pivot(a, lft, rgt):
            fails.append(f"partition_level seg {s}: pivot differs")
        if not np.array_equal(b[lft:rgt + 1], closed_form_arrangement(a, lft, rgt)[lft:rgt + 1]):
            fails.append(f"partition_level seg {s}: arrangement differs")
    keys, offs = synth.batched(9, 10, 64, 1, 3000)
    offs[5] = offs[4]  # one empty array
    k2 = keys.copy()
    fps = oracle.segmented_(k2, offs, lib=lib)
    for s in range(offs.size - 1):
        seg = keys[offs[s]:offs[s + 1]]
        if not np.array_equal(k2[offs[s]:offs[s + 1]], np.sort(seg)):
            fails.append(f"segmented array {s}: not sorted")
        want = -1 if seg.size == 0 else (0 if seg.size == 1 else closed_form_pivot(seg, 0, seg.size - 1))
        if fps[s] != want:
            fails.append(f"segmented array {s}: first pivot {fps[s]} != {want}")
    return fails


ALL_PINS = {
    "illustration": check_illustration,
    "permutations": lambda lib: check_permutations(lib, nmax=7),
    "multisets": lambda lib: check_multisets(lib, spec=((3, 7), (4, 5))),
    "mean_comparisons": lambda lib: check_mean_comparisons(lib, nmax=7),
    "library_sort": lambda lib: check_library_sort(lib, sizes=(2, 17, 1000, 20_000)),
    "levels_and_batches": check_levels_and_batches,
}
