"""Plant plausible mistakes in a copy of the C oracle (on the CPU) and check
that the pins catch every one of them."""
import os
import shutil
import subprocess

import pytest

import oracle.core as oc
from oracle_pins import ALL_CHECKS

MUTANTS = {
    "half_width_floor": ("while ((int64_t)(2 * s + 1) * (2 * s + 1) < 2LL * r * r)",
                         "while ((int64_t)(2 * s + 2) * (2 * s + 2) < 2LL * r * r)"),
    "diamond_strict": ("int in_diamond = (adx + ady <= r);", "int in_diamond = (adx + ady < r);"),
    "square_asym": ("int in_square = (adx <= s && ady <= s);",
                    "int in_square = (adx < s && ady <= s);"),
    "union_not_superposition": ("return in_square + in_diamond;",
                                "return in_square | in_diamond;"),
    "grad_no_abs": ("G[(int64_t)y * W + x] = iabs(gx) + iabs(gy);",
                    "G[(int64_t)y * W + x] = iabs(gx) + gy;"),
    "grad_one_sided": ("int xr = clampi(x + 1, 0, W - 1), xl = clampi(x - 1, 0, W - 1);",
                       "int xr = clampi(x + 1, 0, W - 1), xl = clampi(x, 0, W - 1);"),
    "star_offset_off_by_one": ("int64_t v = img[(int64_t)(y + dy) * stride + (x + dx)];",
                               "int64_t v = img[(int64_t)(y + dy) * stride"
                               " + (x + (dx > 0 ? dx - 1 : dx))];"),
    "grad_sum_wrong_index": ("fg += (int64_t)w * G[(int64_t)(y + dy) * W + (x + dx)];",
                             "fg += (int64_t)w * G[(int64_t)(y + dx) * W + (x + dx)];"),
    "squares_not_squared": ("f2 += w * v * v;", "f2 += w * v;"),
    "grad_factor_swapped": ("i128 c_ref = (f == 2) ? r : 1;", "i128 c_ref = (f == 2) ? rho : 1;"),
    "area_factor_swapped": ("i128 x_ref = (i128)F * area_rho * c_ref;",
                            "i128 x_ref = (i128)F * area_r * c_ref;"),
    "tolerance_sign": ("i128 lhs = (i128)(Q - P) * x_t;", "i128 lhs = (i128)(Q + P) * x_t;"),
    "moment_axes_swapped": ("mx += (int64_t)w * dx * v;", "mx += (int64_t)w * dy * v;"),
    "moment_unweighted": ("my += (int64_t)w * dy * v;", "my += (int64_t)dy * v;"),
    "ring_radius_halved": ("rj = oracle_square_half(rj);", "rj = rj / 2;"),
    "ring_template_outer_radius": ("int rho_j = rho[t * n_rings + j];",
                                   "int rho_j = rho[t * n_rings];"),
    "ring_template_outer_features": ("const int64_t *ft = FT + 3 * ((int64_t)t * n_rings + j);",
                                     "const int64_t *ft = FT + 3 * ((int64_t)t * n_rings);"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    src = open(oc._SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, f"mutation anchor for {name} not found once"
    msrc = tmp_path / "mutant.c"
    msrc.write_text(src.replace(old, new))
    lib_path = str(tmp_path / "libmutant.so")
    subprocess.run(["gcc", "-O1", "-fopenmp", "-shared", "-fPIC", "-o", lib_path, str(msrc)],
                   check=True, capture_output=True)
    lib = oc.load(lib_path)
    caught = []
    for check in ALL_CHECKS:
        try:
            check(lib)
        except AssertionError:
            caught.append(check.__name__)
    assert caught, f"mutant {name} passed every pin"
