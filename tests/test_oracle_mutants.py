"""The pins catch plausible mistakes: each test plants one mistake in a copy
of the oracle source (on the CPU), builds it, and checks that at least one
pin fails.  Every mutant runs in its own process so that a mutant that
writes out of bounds cannot take the test run down."""
import json
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
IMPL = os.path.join(ROOT, "oracle", "ksort_oracle_impl.h")

MUTANTS = {
    # Step-2 read as "j - i > 2" instead of ">= 2"
    "loop_gt2": ("    while (j - i >= 2) {", "    while (j - i > 2) {"),
    # flag kept across calls instead of cleared on entry
    "flag_persistent": ("    int flag = 0;\n", "    static int flag = 0;\n"),
    # Step-6 exactly as printed: "if (left > i + 1)"
    "step6_as_printed": ("if (right > i + 1) {", "if (left > i + 1) {"),
    # Step-5 on [left, i] instead of [left, i-1]
    "step5_includes_key": ("stk[2 * top + 1] = i - 1;", "stk[2 * top + 1] = i;"),
    # temp written over the key instead of next to it
    "temp_at_i": ("a[i + 1] = temp;", "a[i] = temp;"),
    # ties go left instead of right
    "ties_left": ("if (key <= a[p]) {", "if (key < a[p]) {"),
    # k not advanced in Step-3.2
    "k_not_advanced": ("            k = k + 1;\n", ""),
    # Step-1 with j = right instead of right + 1
    "j_init_right": ("int64_t j = right + 1;", "int64_t j = right;"),
    # Step-3.1 move one slot short of the hole
    "move_off_by_one": ("                a[j] = a[p];", "                a[j - 1] = a[p];"),
}

RUNNER = r"""
import json, sys
sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
import oracle, pins
lib = oracle.load({lib!r})
out = {{}}
for name, f in pins.ALL_PINS.items():
    try:
        out[name] = len(f(lib))
    except Exception as e:
        out[name] = "error: " + type(e).__name__
print(json.dumps(out))
"""


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(IMPL).read()
    assert src.count(old) == 1, f"mutant {name}: target text must occur exactly once in the oracle"
    d = tmp_path / "src"
    d.mkdir()
    (d / "ksort_oracle_impl.h").write_text(src.replace(old, new, 1))
    for f in ("ksort_oracle.c", "ksort_oracle.h"):
        (d / f).write_text(open(os.path.join(ROOT, "oracle", f)).read())
    lib = str(tmp_path / "libmutant.so")
    subprocess.run(["gcc", *oracle.CFLAGS, "-w", "-o", lib, str(d / "ksort_oracle.c"), "-I", str(d)],
                   check=True)
    code = RUNNER.format(root=ROOT, tests=os.path.join(ROOT, "tests"), lib=lib)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    if r.returncode != 0:
        return  # the mutant crashed the checks: caught
    res = json.loads(r.stdout.strip().splitlines()[-1])
    caught = [k for k, v in res.items() if v != 0]
    assert caught, f"mutant {name} passed every pin: {res}"


def test_unmutated_oracle_passes_fast_pins(oracle_lib):
    import pins
    for name, f in pins.ALL_PINS.items():
        assert f(oracle_lib) == [], name
