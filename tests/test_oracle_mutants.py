"""The median-filter pins have the power to see plausible mistakes: each test
here copies oracle.c, plants one mistake in the median step (a stencil one
row off, a seam that clamps instead of wrapping, a side-wall stencil turned
across the wall, the pre-collision Delta S as the filtered field, delta as
the landing target, ...), builds the copy, and requires the independent
checks of `median_pins` to reject it.  The unchanged copy, built the same
way, must pass them.  Everything runs on the CPU."""
import importlib.util
import os
import subprocess

import pytest

import median_pins as mp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_C = os.path.join(ROOT, "oracle", "oracle.c")
ORACLE_PY = os.path.join(ROOT, "oracle", "oracle.py")

# (name, text in oracle.c, replacement); each text must occur exactly once
MUTANTS = [
    ("stencil_one_row_off", "sy[k] = wrap(y + dy, ny);", "sy[k] = wrap(y + dy + 1, ny);"),
    ("seam_clamped", "sx[k] = wrap(x + dx, nx);", "sx[k] = (x + dx < 0 ? 0 : (x + dx >= nx ? nx - 1 : x + dx));"),
    ("pre_collision_field", "vals[a] = dpost[sy[a] * nx + sx[a]];", "vals[a] = dpre[sy[a] * nx + sx[a]];"),
    ("delta_as_target", "double pm = homothety_phi(p, q, fpn, fsn, d, t);",
     "double pm = homothety_phi(p, q, fpn, fsn, d, p->delta_median);"),
    ("floor_without_delta", "t = med > p->delta_median ? med : p->delta_median;", "t = med;"),
    ("gate_without_delta", "hit = d > p->delta_median && d > med;", "hit = d > med;"),
    ("side_wall_stencil_across", "sx[k] = x;\n            sy[k] = y - 1 + k;",
     "sx[k] = x - 1 + k;\n            sy[k] = y;"),
    ("wall_row_stencil_across", "sx[k] = x - 1 + k;\n            sy[k] = y;",
     "sx[k] = x;\n            sy[k] = y - 1 + k;"),
    ("corner_stencil_outer_side", "sx[1] = x + ix; sy[1] = y;", "sx[1] = x - ix; sy[1] = y;"),
    ("tube_ends_filtered", "if (p->bc == ORC_BC_TUBE && (x == 0 || x == nx - 1)) return 0;", ""),
    ("d1q3_stencil_shifted", "sx[k] = wrap(x - 1 + k, nx);", "sx[k] = wrap(x + k, nx);"),
]


def build_copy(tmp_path, name, old=None, new=None):
    with open(ORACLE_C) as fh:
        src = fh.read()
    if old is not None:
        assert src.count(old) == 1, f"{name}: the planted text must occur once in oracle.c"
        src = src.replace(old, new)
    d = tmp_path / name
    d.mkdir()
    c = d / "oracle.c"
    c.write_text(src)
    lib = d / "liboracle.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                    "-I", os.path.join(ROOT, "oracle"), "-o", str(lib), str(c), "-lm"], check=True)
    spec = importlib.util.spec_from_file_location(f"oracle_copy_{name}", ORACLE_PY)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod.LIB_PATH = str(lib)
    mod.build = lambda force=False: str(lib)     # load the copy, never rebuild it
    mod._lib = None
    return mod


def test_unchanged_copy_passes(tmp_path):
    mp.all_checks(build_copy(tmp_path, "unchanged"))


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_rejected(tmp_path, name, old, new):
    mod = build_copy(tmp_path, name, old, new)
    with pytest.raises(AssertionError):
        mp.all_checks(mod)
