"""Mutation checks of the oracle's pins (CPU only).

Each case plants one plausible mistake in a copy of the oracle -- a flipped
sign, swapped operands, a wrong neighbour, an inverted rule -- builds or
loads that copy in a temporary directory, and runs the pins named for it.
The case passes only when at least one of those pins fails on the broken
copy, so every pin listed here is shown to see the mistake it is there for.
The product library is not involved; the default oracle build is restored
after each case.
"""
from __future__ import annotations

import os
import subprocess
import types

import pytest

import oracle
import test_oracle_contour as tc
import test_oracle_densify as td

_SRC = os.path.join(os.path.dirname(oracle.__file__), "dco_oracle.c")
_DZ = os.path.join(os.path.dirname(oracle.__file__), "densify.py")


def _call(fn, *args):
    try:
        fn(*args)
    except AssertionError:
        return False
    return True


# (name, exact text in dco_oracle.c, replacement, pins that must catch it)
C_MUTANTS = [
    ("diagonal sector sign flipped",
     "else if ((gx[i] > 0) == (gy[i] > 0))", "else if ((gx[i] > 0) != (gy[i] > 0))",
     [(tc.test_diagonal_step_edge_keeps_its_two_central_diagonals, False),
      (tc.test_diagonal_step_edge_keeps_its_two_central_diagonals, True)]),
    ("vertical sector stepping along x",
     "else if (128 * ax < 53 * ay) { dx = 0; dy = 1; }",
     "else if (128 * ax < 53 * ay) { dx = 1; dy = 0; }",
     [(tc.test_horizontal_step_edge_is_one_row,)]),
    ("ex and ey swapped in the projection",
     "float f1 = F[2 * j1] * ex + F[2 * j1 + 1] * ey;\n"
     "    float f0 = F[2 * j0] * ex + F[2 * j0 + 1] * ey;",
     "float f1 = F[2 * j1] * ey + F[2 * j1 + 1] * ex;\n"
     "    float f0 = F[2 * j0] * ey + F[2 * j0 + 1] * ex;",
     [(tc.test_score_projects_on_the_flow_direction_at_p,)]),
    ("vertical step taken from ex",
     "int sx = (int)rintf(ex), sy = (int)rintf(ey);",
     "int sx = (int)rintf(ex), sy = (int)rintf(ex);",
     [(tc.test_score_of_a_vertical_flow,)]),
    ("sign of the vertical step dropped",
     "int sx = (int)rintf(ex), sy = (int)rintf(ey);",
     "int sx = (int)rintf(ex), sy = absi((int)rintf(ey));",
     [(tc.test_score_direction_with_a_negative_component,)]),
    ("p1 and p0 exchanged",
     "int x1 = clampi(x + sx, 0, w - 1), y1 = clampi(y + sy, 0, h - 1);\n"
     "    int x0 = clampi(x - sx, 0, w - 1), y0 = clampi(y - sy, 0, h - 1);",
     "int x1 = clampi(x - sx, 0, w - 1), y1 = clampi(y - sy, 0, h - 1);\n"
     "    int x0 = clampi(x + sx, 0, w - 1), y0 = clampi(y + sy, 0, h - 1);",
     [(tc.test_score_projects_on_the_flow_direction_at_p,),
      (tc.test_score_of_a_vertical_flow,)]),
    ("vertical amplitude from the next column",
     "float gv = y + 1 < h ? fabsf(flow_r(F, i + w) - r) : 0.0f;",
     "float gv = y + 1 < h ? fabsf(flow_r(F, i + 1 < w * h ? i + 1 : i) - r) : 0.0f;",
     [(tc.test_amplitude_of_a_vertical_speed_ramp,)]),
    ("Eq. 12 inverted",
     "fu[y * w + x] = sp > sf ? mp : (sf > sp ? mf : (mp > mf ? mp : mf));",
     "fu[y * w + x] = sp < sf ? mp : (sf < sp ? mf : (mp > mf ? mp : mf));",
     [(tc.test_fusion_with_amplitudes_of_different_shape,)]),
    ("hysteresis grows only 4-connected",
     "if (yy >= 0 && yy < H && xx >= 0 && xx < W && st[(size_t)yy * W + xx] == 1) {",
     "if ((yy == y || xx == x) && yy >= 0 && yy < H && xx >= 0 && xx < W &&\n"
     "                    st[(size_t)yy * W + xx] == 1) {",
     [(tc.test_weak_chain_touching_a_strong_pixel_diagonally_is_kept,)]),
]

# (name, exact text in densify.py, replacement, pins) -- the text is replaced
# in its first occurrence only, which is edge_weights (energy() keeps its own
# copy of the rule, so the pins must not lean on energy()).
PY_MUTANTS = [
    ("min swapped for max in w_pq",
     "out[y, x] = max(1.0 - min(s[y, x], s[yy, xx]), 0.0)",
     "out[y, x] = max(1.0 - max(s[y, x], s[yy, xx]), 0.0)",
     [(td.test_pair_weight_uses_the_smaller_product, False),
      (td.test_two_by_two_grid_with_every_weight_different,)]),
    ("s as a sum of the two maps",
     "s = np.asarray(Mfuse, np.float64) * np.asarray(MI, np.float64)",
     "s = np.asarray(Mfuse, np.float64) + np.asarray(MI, np.float64)",
     [(td.test_pair_weight_uses_the_smaller_product, False)]),
    ("clamp of w_pq at zero removed",
     "out[y, x] = max(1.0 - min(s[y, x], s[yy, xx]), 0.0)",
     "out[y, x] = 1.0 - min(s[y, x], s[yy, xx])",
     [(td.test_pair_weight_is_clamped_at_zero,)]),
    ("every edge touching the contour cut",
     "if B[y, x] + B[yy, xx] == 1:\n                    out[y, x] = 0.0",
     "if B[y, x] + B[yy, xx] >= 1:\n                    out[y, x] = 0.0",
     [(td.test_pair_on_the_contour_stays_coupled,)]),
    ("transposed s in the edge weights",
     "out[y, x] = max(1.0 - min(s[y, x], s[yy, xx]), 0.0)",
     "out[y, x] = max(1.0 - min(s[x, y], s[xx, yy]), 0.0)",
     [(td.test_two_by_two_grid_with_every_weight_different,)]),
]


@pytest.mark.parametrize("name,old,new,pins", C_MUTANTS, ids=[m[0] for m in C_MUTANTS])
def test_c_oracle_mutant_is_caught(tmp_path, name, old, new, pins):
    src = open(_SRC).read()
    assert src.count(old) == 1, f"mutation site of '{name}' not found once"
    mut = tmp_path / "dco_oracle_mut.c"
    mut.write_text(src.replace(old, new))
    so = str(tmp_path / "libdco_oracle_mut.so")
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-std=c99", "-fPIC", "-shared",
                           "-o", so, str(mut), "-lm"])
    # every pin passes on the real oracle ...
    for fn, *args in pins:
        assert _call(fn, *args), f"{fn.__name__} fails on the unmodified oracle"
    prev = oracle.swap_library(so)
    try:
        caught = [fn.__name__ for fn, *args in pins if not _call(fn, *args)]
    finally:
        oracle.swap_library(prev)
    # ... and at least one fails on the broken copy
    assert caught, f"no pin catches '{name}'"


@pytest.mark.parametrize("name,old,new,pins", PY_MUTANTS, ids=[m[0] for m in PY_MUTANTS])
def test_densify_oracle_mutant_is_caught(monkeypatch, name, old, new, pins):
    src = open(_DZ).read()
    assert old in src, f"mutation site of '{name}' not found"
    mod = types.ModuleType("densify_mutant")
    exec(compile(src.replace(old, new, 1), "densify_mutant.py", "exec"), mod.__dict__)
    for fn, *args in pins:
        assert _call(fn, *args), f"{fn.__name__} fails on the unmodified oracle"
    for attr in ("edge_weights", "system", "densify", "energy"):
        monkeypatch.setattr(td.dz, attr, getattr(mod, attr))
    caught = [fn.__name__ for fn, *args in pins if not _call(fn, *args)]
    assert caught, f"no pin catches '{name}'"
