"""Plant plausible mistakes in copies of the oracle and check that the pins catch
every one of them (on the CPU; the GPU path is not involved)."""
import os

import pytest

import oracle
from tests import pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "gp_oracle.c")

# (name, original text, mutated text)
MUTANTS = [
    ("crossing_le", "if (lhs < rhs)", "if (lhs <= rhs)"),
    ("straddle_open_low", "if (loy <= py && py < hiy)", "if (loy < py && py <= hiy)"),
    ("drop_holes", "for (int64_t r = fro[f]; r < fro[f + 1]; ++r)",
     "for (int64_t r = fro[f]; r < fro[f] + 1; ++r)"),
    ("wrong_index", "double rhs = (hix - lox) * (py - loy);", "double rhs = (hix - lox) * (py - hiy);"),
    ("swapped_lohi", "if (ay < by) {", "if (ay > by) {"),
    ("wrong_endpoint", "double ex = px - bx, ey = py - by;", "double ex = px - ax, ey = py - ay;"),
    ("dropped_term", "return (c * c) / L2;", "return (c * c) / (dx * dx);"),
    ("cross_sign", "double c = wx * dy - wy * dx;", "double c = wx * dy + wy * dx;"),
    ("range_exclusive", "if (d2 <= D2 && d2 < best)", "if (d2 < D2 && d2 < best)"),
    ("ties_to_largest", "if (d2 <= D2 && d2 < best)", "if (d2 <= D2 && d2 <= best)"),
    ("no_endpoint_a", "if (t <= 0.0)\n        return wx * wx + wy * wy;",
     "if (t < -1.0e300)\n        return wx * wx + wy * wy;"),
    ("extent_short", "*nx = (int64_t)floor((hx - lx) / cs) + 1;", "*nx = (int64_t)floor((hx - lx) / cs);"),
    ("pad_inward", "mbb[4 * f + 0] = mnx - pad;", "mbb[4 * f + 0] = mnx + pad;"),
    ("cell_upper_closed", "fx < (double)nx", "fx <= (double)nx"),
    ("no_expand", "mnx = mnx - D; mny = mny - D;", "mnx = mnx; mny = mny - D;"),
    ("unstable_sort", "perm[pos[c]++] = i;", "perm[pos[c + 1] - 1 - (pos[c]++ - pt_off[c])] = i;"),
    ("count_first_hit", "cnt += polygon_inside(px[i], py[i], f, fro, rvo, x, y);",
     "if (polygon_inside(px[i], py[i], f, fro, rvo, x, y)) { cnt = 1; break; }"),
    ("count_clamped", "cnt += polygon_inside(px[i], py[i], f, fro, rvo, x, y);",
     "cnt = cnt | polygon_inside(px[i], py[i], f, fro, rvo, x, y);"),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, name
    mpath = tmp_path / f"mut_{name}.c"
    mpath.write_text(src.replace(old, new))
    lib = oracle.load(oracle.build(str(mpath), str(tmp_path / f"lib_{name}.so")))
    for pin in pins.ALL_PINS:
        try:
            pin(lib)
        except AssertionError:
            return
    pytest.fail(f"no pin detects mutant {name}")
