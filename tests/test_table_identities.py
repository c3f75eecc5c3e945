"""CPU checks of the table definitions the HIP path builds and of the
8-lookup star formula it evaluates, against brute force and the oracle.
(The GPU tests compare the HIP tables with the same numpy definitions.)"""
import numpy as np
import pytest

import oracle.core as oc
from gpu_util import tables_numpy


def brute_tables(img, fm):
    H, W = img.shape
    from gpu_util import quantities
    qs = quantities(img, fm)
    nq = len(qs)
    L = np.zeros((H + 1, W + 1, nq), np.int64)
    R = np.zeros_like(L)
    Rp = np.zeros_like(L)
    for qi, q in enumerate(qs):
        for y in range(-1, H):
            for x in range(-1, W):
                sl = sr = sp = 0
                for j in range(0, y + 1):
                    for i in range(0, W):
                        v = q[j, i]
                        if i <= x:
                            sl += v
                        if abs(i - x) <= y - j:
                            sr += v
                        if x - (y - j) <= i <= x + 1 + (y - j):
                            sp += v
                L[y + 1, x + 1, qi] = sl
                R[y + 1, x + 1, qi] = sr
                Rp[y + 1, x + 1, qi] = sp
    return L, R, Rp


@pytest.mark.parametrize("shape", [(6, 9), (9, 5), (1, 7)])
def test_numpy_tables_equal_brute_force(shape):
    rng = np.random.default_rng(sum(shape))
    img = rng.integers(0, 256, shape).astype(np.uint8)
    for a, b in zip(tables_numpy(img, 7), brute_tables(img, 7)):
        assert np.array_equal(a, b)


def star_from_tables(tabs, x, y, r):
    """The HIP kernel's inclusion-exclusion, on host arrays indexed [y+1, x+1]."""
    L, R, Rp = tabs
    s = oc.square_half(r)

    def at(T, xx, yy):
        return T[yy + 1, xx + 1]
    sq = at(L, x + s, y + s) - at(L, x - s - 1, y + s) - at(L, x + s, y - s - 1) \
        + at(L, x - s - 1, y - s - 1)
    dm = at(R, x, y + r) - at(Rp, x - r - 1, y - 1) - at(Rp, x + r, y - 1) + at(R, x, y - r - 1)
    return sq + dm


@pytest.mark.parametrize("seed", range(3))
def test_star_formula_matches_oracle(seed):
    rng = np.random.default_rng(seed)
    H, W = int(rng.integers(8, 30)), int(rng.integers(8, 30))
    img = rng.integers(0, 4096, (H, W)).astype(np.uint16)
    tabs = tables_numpy(img, 7)
    for r in range(0, min(H, W) // 2):
        ys, xs = np.mgrid[r:H - r, r:W - r]
        F = oc.star_features(img, xs.ravel(), ys.ravel(), r)
        for i, (x, y) in enumerate(zip(xs.ravel(), ys.ravel())):
            assert (star_from_tables(tabs, int(x), int(y), r) == F[i]).all(), (r, x, y)
