"""GPU parity of the preserved region (oss_region) with the oracle's union
of candidate star footprints, on the candidate lists of real screens."""
import numpy as np
import pytest

import oracle.core as oc
from gpu_util import Runner, say
from synth import make_workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def runner():
    r = Runner()
    yield r
    r.close()


def _region(runner, H, W, T, probes, lst, cap=None):
    torch = runner.torch
    L = runner.L
    dev = runner.dev
    lst = np.asarray(lst, np.int64).reshape(-1, 4)
    cap = len(lst) if cap is None else cap
    d = torch.zeros((max(1, len(lst)), 4), dtype=torch.int32, device=dev)
    if len(lst):
        d[:len(lst)] = torch.from_numpy(lst.astype(np.uint32).view(np.int32)).to(dev)
    count = torch.tensor([len(lst)], dtype=torch.int64, device=dev)
    region = torch.full((T, H, W), 7, dtype=torch.uint8, device=dev)
    L.oss_region(runner.ctx.handle, H, W, T, probes, d, cap, count, region)
    torch.cuda.synchronize()
    return region.cpu().numpy()


CASES = {
    2: dict(H=230, W=270, blobs_per_512sq=800, sig_hi=24),
    3: dict(H=200, W=260, n_templates=5, blobs_per_512sq=1200, sig_hi=20),
    5: dict(H=224, W=240, n_templates=3, blobs_per_512sq=1200, sig_hi=20),
}


@pytest.mark.parametrize("cfg", sorted(CASES))
def test_region_equals_oracle(runner, cfg):
    w = make_workload(cfg, 3, **CASES[cfg])
    tm = [(t.pixels, t.rho) for t in w.templates]
    mask, cands, n = runner.screen(w.ref, tm, w.probes, w.feat_mask, w.tol_P, w.tol_Q)
    T = len(tm)
    say(f"region cfg{cfg}: {n} candidates")
    got = _region(runner, w.H, w.W, T, w.probes, cands)
    radius_of = {(t, k): r for t, k, r in w.probes}
    want = oc.region_full(w.H, w.W, T, cands, radius_of)
    assert np.array_equal(got, want)
    assert got.sum() > 0


def test_region_edges(runner):
    H, W = 40, 50
    probes = [(0, 0, 3), (0, 1, 7), (1, 0, 19)]
    radius_of = {(t, k): r for t, k, r in probes}
    # candidates on the borders of where their stars fit, several scales
    lst = [(0, 3, 3, 1), (0, 7, 42, 3), (0, 36, 46, 1), (0, 32, 7, 2), (1, 19, 19, 1),
           (1, 20, 30, 1)]
    got = _region(runner, H, W, 2, probes, lst)
    assert np.array_equal(got, oc.region_full(H, W, 2, lst, radius_of))
    # only the first list_cap entries count; an empty list preserves nothing
    got = _region(runner, H, W, 2, probes, lst, cap=2)
    assert np.array_equal(got, oc.region_full(H, W, 2, lst[:2], radius_of))
    assert not _region(runner, H, W, 2, probes, []).any()
    # a probe radius that cannot fit the image is ignored
    got = _region(runner, H, W, 2, probes + [(1, 5, 30)], lst)
    assert np.array_equal(got, oc.region_full(H, W, 2, lst, radius_of))
