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


# Mistakes planted in the Python parts of the oracle (the template centre,
# Algorithm 1 and the paper's own features): (module, anchor, replacement).
PY_MUTANTS = {
    "alg1_band_count_off_by_one": ("alg1", "while Fraction(2) ** B < ratio2:",
                                   "while Fraction(2) ** B <= ratio2:"),
    "alg1_band_low_exponent": ("alg1", "k_lo = _ceil_over_sqrt2_pow(v, b + 1)",
                               "k_lo = _ceil_over_sqrt2_pow(v, b)"),
    "alg1_resize_corner_aligned": ("alg1", "num = (2 * i + 1) * n - k",
                                   "num = 2 * i * n - k"),
    "alg1_resize_round_down": ("alg1", "return ((2 * val + den) // (2 * den))",
                               "return ((2 * val) // (2 * den))"),
    "alg1_quantise_floor": ("alg1", "return floor(Fraction(f) / q + Fraction(1, 2))",
                            "return floor(Fraction(f) / q)"),
    "alg1_mark_drop_low": ("alg1", "cells.append(sorted({quantise(F[f] - h, q[f]), "
                                   "quantise(F[f], q[f]),",
                           "cells.append(sorted({quantise(F[f], q[f]),"),
    "alg1_mark_drop_high": ("alg1", "quantise(F[f] + h, q[f])}))", "quantise(F[f], q[f])}))"),
    "alg1_step_without_area": ("alg1", "q = [qbar[f] * A for f in range(3)]",
                               "q = [qbar[f] for f in range(3)]"),
    "core_template_centre_rounded_up": ("core", "cx, cy = (w - 1) // 2, (h - 1) // 2",
                                        "cx, cy = w // 2, h // 2"),
    "moments_mean_areas_swapped": (
        "moments", "(Q - P[0]) * t1 * A_r <= Q * f1 * A_rho <= (Q + P[0]) * t1 * A_r",
        "(Q - P[0]) * t1 * A_rho <= Q * f1 * A_r <= (Q + P[0]) * t1 * A_rho"),
    "moments_var_areas_swapped": ("moments", "V, VT = A_r * f2 - f1 * f1, A_rho * t2 - t1 * t1",
                                  "V, VT = A_rho * f2 - f1 * f1, A_r * t2 - t1 * t1"),
    "moments_var_sign": ("moments", "V, VT = A_r * f2 - f1 * f1,", "V, VT = A_r * f2 + f1 * f1,"),
    "moments_mag_without_lever_arm": ("moments", "N_r, N_rho = r * A_r, rho * A_rho",
                                      "N_r, N_rho = A_r, A_rho"),
    "moments_mag_bound_unsquared": ("moments", "(Q + P[2]) ** 2 * MT * N_r ** 2",
                                    "(Q + P[2]) * MT * N_r ** 2"),
}


@pytest.mark.parametrize("name", sorted(PY_MUTANTS))
def test_python_mutant_is_caught(name, monkeypatch, oracle_lib):
    import sys
    import types

    import oracle
    import oracle_pins
    modname, old, new = PY_MUTANTS[name]
    path = os.path.join(os.path.dirname(oc.__file__), modname + ".py")
    src = open(path).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not found once"
    mod = types.ModuleType("oracle." + modname)
    mod.__file__ = path
    mod.__package__ = "oracle"
    exec(compile(src.replace(old, new), path, "exec"), mod.__dict__)
    monkeypatch.setitem(sys.modules, "oracle." + modname, mod)
    monkeypatch.setattr(oracle, modname, mod, raising=False)
    check = {"alg1": oracle_pins.check_alg1, "moments": oracle_pins.check_moments,
             "core": oracle_pins.check_planted_exact}[modname]
    if modname == "core":
        # the pins call the oracle through the module-level name
        monkeypatch.setattr(oracle_pins, "oc", mod)
    with pytest.raises(AssertionError):
        check(oracle_lib)
