"""The paper's own patch features over the star, and the screen that
compares them (Sec. "Patch Features": mean, Eq. S_sigma variance, the
horizontal and vertical gradients as inner products with the extended
Prewitt ramps, Eq. S_x / Eq. T_x; Sec. "Rotation Invariance": the gradient
magnitude S_m = sqrt(S_x^2 + S_y^2)).

TEST INFRASTRUCTURE.  Only the test suite uses this module.

Per star of radius r at (x, y), with its 0/1/2 weights w and area A(r):
  F1 = sum w I,  F2 = sum w I^2,  Sx = sum w (i - x) I,  Sy = sum w (j - y) I
  mean  = F1 / A(r)
  var   = F2 / A(r) - mean^2 = (A(r) F2 - F1^2) / A(r)^2
  mag   = sqrt(Sx^2 + Sy^2)
Across a reference radius r and a template radius rho (a probe), the mean
and the variance are compared as they are (they do not depend on the
patch size), and the magnitude after dividing by N(r) = r A(r): a first
moment grows with the area and with the lever arm.  Each compared feature
must lie within the relative tolerance P/Q of the template's, checked in
exact integers (the magnitude squared):
  mean:  (Q-P) FT1 A(r)          <= Q F1 A(rho)            <= (Q+P) FT1 A(r)
  var:   (Q-P) VT A(r)^2         <= Q V A(rho)^2           <= (Q+P) VT A(r)^2
         with V = A F2 - F1^2
  mag:   (Q-P)^2 MT N(r)^2       <= Q^2 M N(rho)^2         <= (Q+P)^2 MT N(r)^2
         with M = Sx^2 + Sy^2 (the lower bound is void when P > Q)
"""
from __future__ import annotations

import numpy as np

from . import core as oc

MEAN, VAR, MAG = 1, 2, 4


def moments(img, xs, ys, r: int, lib=None) -> np.ndarray:
    """[n, 4] (F1, F2, Sx, Sy) at the positions; -1 rows where the star does
    not fit."""
    lib = lib or oc.load()
    a = oc._img16(img)
    H, W = a.shape
    xs = np.ascontiguousarray(xs, np.int32)
    ys = np.ascontiguousarray(ys, np.int32)
    F = np.zeros((len(xs), 4), np.int64)
    lib.oracle_moments(a, H, W, W, xs, ys, len(xs), int(r), F)
    return F


def template_moments(tmpl, rho: int, lib=None):
    a = oc._img16(tmpl)
    h, w = a.shape
    F = moments(a, [(w - 1) // 2], [(h - 1) // 2], rho, lib)[0]
    if F[0] < 0:
        raise ValueError("template star does not fit")
    return tuple(int(v) for v in F)


def probe_pass(F, FT, r: int, rho: int, P, Q: int, tests: int, lib=None) -> bool:
    """The three tests of one probe, in Python integers."""
    A_r, A_rho = oc.star_area(r, lib), oc.star_area(rho, lib)
    f1, f2, sx, sy = (int(v) for v in F)
    t1, t2, tx, ty = (int(v) for v in FT)
    if tests & MEAN:
        if not ((Q - P[0]) * t1 * A_r <= Q * f1 * A_rho <= (Q + P[0]) * t1 * A_r):
            return False
    if tests & VAR:
        V, VT = A_r * f2 - f1 * f1, A_rho * t2 - t1 * t1
        if not ((Q - P[1]) * VT * A_r ** 2 <= Q * V * A_rho ** 2 <= (Q + P[1]) * VT * A_r ** 2):
            return False
    if tests & MAG:
        M, MT = sx * sx + sy * sy, tx * tx + ty * ty
        N_r, N_rho = r * A_r, rho * A_rho
        lo = (Q - P[2]) ** 2 * MT * N_r ** 2 if Q >= P[2] else 0
        if not (lo <= Q * Q * M * N_rho ** 2 <= (Q + P[2]) ** 2 * MT * N_r ** 2):
            return False
    return True


def screen_full(img, templates, probes, P, Q: int, tests: int, lib=None) -> np.ndarray:
    """bits[n_tmpl, H, W]; templates: list of (pixels, rho); probes: (t, k, r)."""
    lib = lib or oc.load()
    a = oc._img16(img)
    H, W = a.shape
    ys, xs = np.meshgrid(np.arange(H, dtype=np.int32), np.arange(W, dtype=np.int32),
                         indexing="ij")
    xs, ys = xs.ravel(), ys.ravel()
    FT = [template_moments(px, rho, lib) for px, rho in templates]
    bits = np.zeros((len(templates), H * W), np.uint32)
    cache = {}
    for t, k, r in probes:
        if r not in cache:
            cache[r] = moments(a, xs, ys, r, lib)
        F = cache[r]
        rho = templates[t][1]
        for i in np.nonzero(F[:, 0] >= 0)[0]:
            if probe_pass(F[i], FT[t], r, rho, P, Q, tests, lib):
                bits[t, i] |= 1 << k
    return bits.reshape(len(templates), H, W)
