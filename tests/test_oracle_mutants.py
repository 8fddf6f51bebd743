"""Planted mistakes in the oracle must fail at least one pin (CPU only).

Each mutant is a copy of ``oracle/cubeoracle.c`` with one plausible mistake
(a dropped term, a wrong sign, a transposed index or operand, an off-by-one),
compiled into a temporary library and run through every pin.  A mutant that
passes all pins would mean the pins could not tell that mistake from a
correct oracle.
"""
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

import oracle
from tests import oracle_pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "cubeoracle.c")

MUTANTS = {
    "drop_sum_term": ("neumaier_add(&s->sum, &s->sum_c, (double)v);", ""),
    "compensation_sign": ("*c += (*s - t) + x;", "*c += (*s - t) - x;"),
    "min_compare_swapped": ("if (before(v, s->min)) s->min = v;",
                            "if (before(s->min, v)) s->min = v;"),
    "signed_zero_ignored": ("if (a == b && signbit(a) && !signbit(b)) return 1;", ""),
    "nan_counted_valid": ("s->n_nan++;\n                    continue;", "s->n_nan++;"),
    "index_transposed": ("float v = p[x + sy * y + sz * z];\n                s->n_total++;",
                         "float v = p[y + sy * x + sz * z];\n                s->n_total++;"),
    "sweep2_plane_pitch": ("float v = p[x + sy * y + sz * z];\n                if (v != v) continue;",
                           "float v = p[x + sy * y + sy * z];\n                if (v != v) continue;"),
    "deviation_sign": ("double d = (double)v - mean;", "double d = mean + (double)v;"),
    "sample_std": ("out->std = sqrt(m2 / n);", "out->std = sqrt(m2 / (n - 1.0));"),
    "mean_abs_signed": ("fabs((double)v));", "(double)v);"),
    "inf_through_compensation": ("if (isinf(v)) {\n                    /* kept apart",
                                 "if (0) {\n                    /* kept apart"),
    "inf_both_signs_not_nan": ("if (s->n_pinf && s->n_ninf) return NAN;", ""),
    "inf_std_finite": ("out->m2 = out->std = NAN;\n        return;", "out->m2 = out->std = 0.0;"),
    "slab_min_from_empty": ("if (a->n_valid == 0) {\n            a->min = b->min;\n            a->max = b->max;\n        } else {",
                            "{"),
    "slab_max_order": ("if (before(a->max, b->max)) a->max = b->max;",
                       "if (before(b->max, a->max)) a->max = b->max;"),
    "slab_sum_compensation_dropped": ("a->sum_c += b->sum_c;", ""),
    "slab_sq_not_added": ("neumaier_add(&a->sq, &a->sq_c, b->sq);", ""),
    "clamp_off_by_one": ("if (b > nbins - 1) b = nbins - 1;", "if (b > nbins) b = nbins;"),
    "below_above_swapped": ("counts[nbins]++;\n                } else if (v > hi) {\n                    counts[nbins + 1]++;",
                            "counts[nbins + 1]++;\n                } else if (v > hi) {\n                    counts[nbins]++;"),
    "bin_rule_reassociated": ("float u = (v - lo) * scale;", "float u = v * scale - lo * scale;"),
    "scale_inverted": ("float s = (float)nbins / width;", "float s = width / (float)nbins;"),
    "lower_edge_open": ("} else if (v < lo) {", "} else if (v <= lo) {"),
    "degenerate_range_rejected": ("if (width == 0.0f) {\n        *scale = 0.0f;\n        return 0;",
                                  "if (width == 0.0f) {\n        *scale = 0.0f;\n        return -1;"),
    "ftz_like_truncation": ("int64_t b = (int64_t)floorf(u);", "int64_t b = (int64_t)floorf(u + 1e-7f);"),
    "select_includes_nan": ("if (f == f) v[n++] = f;", "v[n++] = f;"),
    "select_reversed": ("if (before(x, y)) return -1;", "if (before(x, y)) return 1;"),
    "median_upper_only": ("*median = ((double)a + (double)b) / 2.0;", "*median = (double)b;"),
    "quantile_includes_nan": ("if (w != w) continue;  /* blank */", ""),
    "quantile_upper_rank": ("double a = v[(uint64_t)j];", "double a = v[(uint64_t)ceil(h)];"),
    "quantile_fraction_flipped": ("r = a + f * (b - a);", "r = b - f * (b - a);"),
    "quantile_rank_of_n": ("double h = q[i] * (double)(n - 1);", "double h = q[i] * (double)n;"),
    "quantile_inf_not_kept": ("        else if (isinf(a))\n            r = a;\n", ""),
    "project_wrong_axis": ("float f = p[x + sy * y + sz * z];\n                if (f != f) continue;",
                           "float f = p[x + sy * z + sz * y];\n                if (f != f) continue;"),
    "project_min_not_max": ("if (n == 0 || before(mx, f)) mx = f;",
                            "if (n == 0 || before(f, mx)) mx = f;"),
    "project_empty_is_zero": ("if (mom0) mom0[i] = n ? sum : NAN;",
                              "if (mom0) mom0[i] = sum;"),
    "project_inf_cancel": ("sum = (pinf && ninf) ? NAN : (pinf ? INFINITY : -INFINITY);",
                           "sum = pinf ? INFINITY : -INFINITY;"),
    "project_counts_blank": ("if (f != f) continue;\n                if (n == 0",
                             "if (f != f) { ++n; continue; }\n                if (n == 0"),
}


@pytest.fixture(scope="module")
def workdir():
    d = tempfile.mkdtemp(prefix="oracle_mut_")
    yield d
    shutil.rmtree(d, ignore_errors=True)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, workdir):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique/found"
    mutated = src.replace(old, new)
    c_path = os.path.join(workdir, f"{name}.c")
    so_path = os.path.join(workdir, f"lib{name}.so")
    with open(c_path, "w") as f:
        f.write(mutated)
    subprocess.check_call(["gcc", *oracle.CFLAGS, "-o", so_path, c_path, "-lm"],
                          stderr=subprocess.DEVNULL)
    # Run the pins in a child process: a mutant may also crash (an index
    # mistake can read outside the array), which counts as caught.
    code = ("import sys, oracle\n"
            "from tests import oracle_pins\n"
            "o = oracle.Oracle(sys.argv[1])\n"
            "failed = []\n"
            "for pin in oracle_pins.ALL_PINS:\n"
            "    try:\n"
            "        pin(o)\n"
            "    except (AssertionError, ValueError):\n"
            "        failed.append(pin.__name__)\n"
            "print('FAILED:' + ','.join(failed))\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code, so_path], cwd=root,
                       capture_output=True, text=True, timeout=300)
    if r.returncode != 0:
        return  # crashed on a pin input: caught
    line = [l for l in r.stdout.splitlines() if l.startswith("FAILED:")][-1]
    assert line != "FAILED:", f"mutant {name} passed every pin"
