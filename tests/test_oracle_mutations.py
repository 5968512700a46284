"""The oracle's pins catch plausible mistakes in the oracle itself.

Each case below plants one mistake in a copy of ``oracle/lnf_oracle.c`` (on the
CPU, in a temporary directory), compiles it, and runs a battery of pins from
``test_oracle_pins.py`` against it: exact-fraction brute force of both rules
and several cluster geometries, the hand-derived step-edge and impulse
fixtures, and the gate.  Every mutant must fail at least one pin, and the
unmodified source must pass them all.  Rewrites that compute the same
function (for example (2s + n) / 2n written as (s + (n - 1) / 2) / n, both
the rounded mean since n is odd) are not mistakes and are not listed.
"""
import os

import numpy as np
import pytest

import oracle
import test_oracle_pins as pins
from paper_1807_03119_amd import phantom as ph

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
SRC = os.path.join(os.path.dirname(os.path.abspath(oracle.__file__)), "lnf_oracle.c")

# (name, text in lnf_oracle.c, replacement)
MUTANTS = [
    ("centre cluster dropped from the MEAN9 total",
     "for (int k = 0; k < 9; ++k) total += s[k];", "for (int k = 1; k < 9; ++k) total += s[k];"),
    ("MEAN9 truncates instead of rounding",
     "out = (2 * total + 9 * n) / (18 * n);", "out = total / (9 * n);"),
    ("MEAN9 divides by 8n",
     "out = (2 * total + 9 * n) / (18 * n);", "out = (2 * total + 8 * n) / (16 * n);"),
    ("variance numerator without the factor n",
     "(int64_t)(n * q[k]) - (int64_t)(s[k] * s[k])", "(int64_t)(q[k]) - (int64_t)(s[k] * s[k])"),
    ("variance numerator with the wrong sign",
     "(int64_t)(n * q[k]) - (int64_t)(s[k] * s[k])", "(int64_t)(n * q[k]) + (int64_t)(s[k] * s[k])"),
    ("ties go to the last cluster", "v < best_v", "v <= best_v"),
    ("largest variance selected", "v < best_v", "v > best_v"),
    ("MINVAR9 mean truncated", "out = (2 * s[best] + n) / (2 * n);", "out = s[best] / n;"),
    ("gate also zeroes the threshold value",
     "out = (2 * s[best] + n) / (2 * n);\n    }\n    if (out < gate_T) out = 0;",
     "out = (2 * s[best] + n) / (2 * n);\n    }\n    if (out <= gate_T) out = 0;"),
    ("diagonal offsets with flipped signs", "off[axis] = ((j >> axis) & 1) ? d : -d;",
     "off[axis] = ((j >> axis) & 1) ? -d : d;"),
    ("cluster index bits in z, y, x order", "off[axis] = ((j >> axis) & 1) ? d : -d;",
     "off[axis] = ((j >> (2 - axis)) & 1) ? d : -d;"),
    ("samples wrap around instead of clamping",
     "if (v < 0) return 0;\n    if (v > n - 1) return n - 1;",
     "if (v < 0) return (v % n + n) % n;\n    if (v > n - 1) return v % n;"),
    ("upper clamp one voxel short", "if (v > n - 1) return n - 1;",
     "if (v > n - 1) return n > 1 ? n - 2 : 0;"),
    ("box one voxel short in x",
     "for (int64_t ax = -r; ax <= r; ++ax) {\n                        uint64_t v = sample(g, cx",
     "for (int64_t ax = -r; ax < r; ++ax) {\n                        uint64_t v = sample(g, cx"),
    ("x and y swapped in the voxel index", "int64_t idx = (cz * g->ny + cy) * g->nx + cx;",
     "int64_t idx = (cz * g->nx + cx) * g->ny + cy;"),
    ("cross counts its centre once in the sum", "sum += vx + vy + vz;",
     "sum += vx + (t ? vy + vz : 0);"),
    ("cross size counts the centre once", "return shape == LNFO_CROSS ? 3 * m : m * m * m;",
     "return shape == LNFO_CROSS ? 3 * m - 2 : m * m * m;"),
    ("offset 2r+1 taken as 2r", "offset_mode == 1 ? 1 : 2 * r + 1;", "offset_mode == 1 ? 1 : 2 * r;"),
    ("default offset fixed at 1", "geo->d = offset_mode == 0 ? r :", "geo->d = offset_mode == 0 ? 1 :"),
]


def _battery():
    """Names of the pins that fail against the oracle now loaded."""
    failed = []

    def run(name, fn):
        try:
            fn()
        except AssertionError:
            failed.append(name)

    for rule in (oracle.MEAN9, oracle.MINVAR9):
        for r in (1, 2):
            for dims, kind, dtype in [((5, 4, 3), "uniform", np.uint8),
                                      ((4, 4, 4), "extreme", np.uint16),
                                      ((6, 3, 4), "low", np.uint8)]:
                run(f"bruteforce rule {rule} r {r} {kind}",
                    lambda: pins.test_bruteforce_fractions(rule, r, dims, kind, dtype))
    run("step edge", lambda: pins.test_step_edge_golden(GOLDEN))
    run("impulse", lambda: pins.test_impulse_golden(GOLDEN))
    run("gate", pins.test_gate_writes_zero_below_threshold)
    for shape, off in [(oracle.CROSS, oracle.OFFSET_R), (oracle.BOX, oracle.OFFSET_TILE),
                       (oracle.CROSS, oracle.OFFSET_ONE)]:
        for rule in (oracle.MEAN9, oracle.MINVAR9):
            run(f"geometry {shape} {off} rule {rule}",
                lambda: pins.test_geometry_bruteforce_fractions(shape, off, rule, 2))
    return failed


@pytest.fixture
def use_library(monkeypatch):
    def use(path):
        monkeypatch.setattr(oracle, "_lib", oracle.open_library(path))
    return use


def test_pins_pass_on_the_oracle_as_written(tmp_path, use_library):
    use_library(oracle.build(SRC, str(tmp_path / "liblnfo_control.so")))
    assert _battery() == []


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_the_planted_mistake(tmp_path, use_library, name, old, new):
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation site not unique in the oracle: {old!r}"
    src = tmp_path / "lnf_oracle_mutant.c"
    src.write_text(text.replace(old, new))
    use_library(oracle.build(str(src), str(tmp_path / "liblnfo_mutant.so")))
    assert _battery(), f"no pin notices: {name}"
