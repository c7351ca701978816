"""Planted mistakes: each mutant copy of the oracle must fail at least one pin.

The mutations are applied to a temporary copy of the oracle's C source and
compiled on the CPU; the committed oracle is never modified.  This shows the
pins are strong enough that a plausible slip anywhere in the oracle (a dropped
term, a wrong sign or index, a lost sort, a miscounted pattern) is caught.
"""
import os
import subprocess
import sys
import tempfile

import pytest

import oracle
from pins import ALL_PINS

SRC = os.path.join(os.path.dirname(oracle.__file__), "spgemm_oracle.c")

MUTANTS = {
    "overwrite_instead_of_add": ("s->acc[j] = s->acc[j] + prod;", "s->acc[j] = prod;"),
    "wrong_sign": ("s->acc[j] = s->acc[j] + prod;", "s->acc[j] = s->acc[j] - prod;"),
    "drop_first_product": ("                s->acc[j] = prod;\n", "                s->acc[j] = 0.0;\n"),
    "drop_factor_a": ("double prod = a * b_val[q];", "double prod = b_val[q];"),
    "drop_last_b_entry": ("        for (int64_t q = b_rp[k]; q < b_rp[k + 1]; ++q) {\n            int32_t j = b_col[q];\n            double prod",
                          "        for (int64_t q = b_rp[k]; q < b_rp[k + 1] - 1; ++q) {\n            int32_t j = b_col[q];\n            double prod"),
    "no_sort": ("    qsort(s->touched, (size_t)count, sizeof(int32_t), cmp_int32);\n", ""),
    "count_products_not_columns": ("if (s->mark[j] != stamp) { s->mark[j] = stamp; ++count; }", "++count;"),
    "emit_scale_not_value": ("out_val[t] = s->acc[j];", "out_val[t] = s->sabs[j];"),
    "position_not_column": ("        int32_t k = a_col[p];\n        double a", "        int32_t k = (int32_t)(p - a_rp[i]);\n        double a"),
    "wrong_a_value": ("double a = a_val[p];", "double a = a_val[a_rp[i]];"),
    "skip_last_a_entry": ("    for (int64_t p = a_rp[i]; p < a_rp[i + 1]; ++p) {\n        int32_t k = a_col[p];\n        double a",
                          "    for (int64_t p = a_rp[i]; p < a_rp[i + 1] - 1; ++p) {\n        int32_t k = a_col[p];\n        double a"),
    "descending_order": ("return (a > b) - (a < b);", "return (a < b) - (a > b);"),
    "row_state_not_reset": ("int64_t count = 0, stamp = ++s->stamp;", "int64_t count = 0, stamp = s->stamp;"),
}


def _compile(src_text, workdir, name):
    c = os.path.join(workdir, name + ".c")
    so = os.path.join(workdir, name + ".so")
    with open(c, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                           "-w", c, "-o", so, "-lm"])
    return so


_DRIVER = r"""
import sys
sys.path[:0] = [{root!r}, {tests!r}]
import oracle
from pins import ALL_PINS
lib = oracle.load_library({so!r})
failed = []
for pin in ALL_PINS:
    try:
        pin(lib=lib)
    except Exception:
        failed.append(pin.__name__)
print("FAILED:" + ",".join(failed))
"""


def _pins_fail(so):
    """Run every pin against the library in a child process (a planted
    mistake may also crash it, which counts as caught)."""
    here = os.path.dirname(os.path.abspath(__file__))
    code = _DRIVER.format(root=os.path.dirname(here), tests=here, so=so)
    p = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    if p.returncode != 0:
        return ["crashed(%d)" % p.returncode]
    line = [l for l in p.stdout.splitlines() if l.startswith("FAILED:")][-1]
    return [x for x in line[len("FAILED:"):].split(",") if x]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    with open(SRC) as f:
        text = f.read()
    old, new = MUTANTS[name]
    assert text.count(old) >= 1, "mutation anchor not found: the oracle source changed"
    mutated = text.replace(old, new, 1)
    with tempfile.TemporaryDirectory() as d:
        failed = _pins_fail(_compile(mutated, d, name))
    assert failed, "planted mistake %r passed every pin" % name


def test_unmutated_copy_passes():
    with open(SRC) as f:
        text = f.read()
    with tempfile.TemporaryDirectory() as d:
        assert _pins_fail(_compile(text, d, "clean")) == []
