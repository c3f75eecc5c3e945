"""The oracle against the paper's worked example, closed forms, a library
routine, an independent enumerator and the exact-copy guarantee."""
import numpy as np
import pytest

import oracle.core as oc
from oracle_pins import ALL_CHECKS


@pytest.mark.parametrize("check", ALL_CHECKS, ids=lambda c: c.__name__)
def test_pin(check, oracle_lib):
    check(oracle_lib)


def test_screen_matches_feature_pass(oracle_lib):
    """The screen loop agrees with star_features + feature_pass applied probe
    by probe (two code paths of the oracle, several templates and radii)."""
    from synth import make_workload
    w = make_workload(3, 1, H=64, n_templates=3, blobs_per_512sq=1500, sig_hi=10)
    tm = [(t.pixels, t.rho) for t in w.templates]
    probes = [p for p in w.probes if p[2] <= 20]
    P, Q = (30, 60, 80), 100
    rng = np.random.default_rng(0)
    xs = rng.integers(0, 64, 200).astype(np.int32)
    ys = rng.integers(0, 64, 200).astype(np.int32)
    bits = oc.screen_positions(w.ref, tm, probes, 7, P, Q, xs, ys, oracle_lib)
    want = np.zeros_like(bits)
    for t, k, r in probes:
        FT = oc.template_features(tm[t][0], tm[t][1], oracle_lib)
        F = oc.star_features(w.ref, xs, ys, r, oracle_lib)
        for i in range(len(xs)):
            if F[i, 0] < 0:
                continue
            if all(oc.feature_pass(f, F[i, f], FT[f], r, tm[t][1], P[f], Q, oracle_lib)
                   for f in range(3)):
                want[t, i] |= 1 << k
    assert (bits == want).all()
    assert want.any() and not want.all()


def test_mask_and_list():
    rng = np.random.default_rng(1)
    bits = (rng.random((3, 9, 11)) < 0.1).astype(np.uint32) * rng.integers(1, 9, (3, 9, 11)).astype(np.uint32)
    mask, lst = oc.mask_and_list(bits)
    assert mask.sum() == len(lst) == np.count_nonzero(bits)
    keys = lst[:, 0] * 99 * 99 + lst[:, 1] * 99 + lst[:, 2]
    assert (np.diff(keys) > 0).all()
    assert (bits[lst[:, 0], lst[:, 1], lst[:, 2]] == lst[:, 3]).all()


def test_radius_grid_cfg5():
    from synth import radius_grid_cfg5
    assert radius_grid_cfg5() == [24, 25, 26, 27, 29, 30, 31, 33, 34, 36, 38, 39, 41, 43, 45, 47,
                                  49, 51, 54, 56, 59, 61, 64, 67, 70, 73, 77, 80, 84, 88, 92, 96]
