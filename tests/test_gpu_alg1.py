"""GPU parity of Algorithm 1 taken literally (oss_alg1_probes +
oss_screen_intervals) with the oracle's quantised-membership screen,
element by element, on exact cuts and resampled templates."""
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle.core as oc
from gpu_util import Runner, say
from oracle import alg1
from synth import blob_image, cut_patch, make_rng, make_workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def runner():
    r = Runner()
    yield r
    r.close()


def _screen(runner, img, templates, alpha, beta, qbar, fm, depth=8):
    L = runner.L
    torch = runner.torch
    probes = []
    for t, tm in enumerate(templates):
        probes += L.oss_alg1_probes(tm, t, alpha, beta, qbar, fm, bit_depth=depth)
    max_r = max(p.r for p in probes)
    ref = runner.ctx.reference(L.device_image(img, runner.dev), fm, depth, max_radius=max_r)
    T = len(templates)
    H, W = img.shape
    mask = torch.empty((T, H, W), dtype=torch.uint8, device=runner.dev)
    cap = T * H * W
    cands = torch.empty((cap, 4), dtype=torch.int32, device=runner.dev)
    count = torch.zeros(1, dtype=torch.int64, device=runner.dev)
    L.oss_screen_intervals(runner.ctx.handle, ref.handle, T, probes, fm, mask, cands, cap, count)
    torch.cuda.synchronize()
    n = int(count.item())
    c = cands[:n].cpu().numpy().astype(np.int64)
    c[:, 3] &= 0xFFFFFFFF
    out = mask.cpu().numpy(), c, n, len(probes)
    ref.release()
    return out


@pytest.mark.parametrize("fm", [3, 7])
def test_alg1_exact_cuts(runner, fm):
    img = blob_image(150, 170, make_rng(96, 0), blobs_per_512sq=1500, sig_hi=10)
    tms = [cut_patch(img, 70, 60, 12), cut_patch(img, 100, 90, 9, quarter_turns=1)]
    qbar = (2, 120, 3)
    mask, lst, n, npb = _screen(runner, img, tms, Fr(1, 2), Fr(2), qbar, fm)
    want = alg1.screen(img, tms, Fr(1, 2), Fr(2), qbar, fm)
    wmask, wlist = oc.mask_and_list(want)
    say(f"alg1 exact fm={fm}: {npb} probes, {n} candidates")
    assert n == len(wlist) and np.array_equal(mask, wmask) and np.array_equal(lst, wlist)


@pytest.mark.parametrize("cfg", [2, 5])
def test_alg1_resampled(runner, cfg):
    size = dict(H=180, W=200) if cfg == 2 else dict(H=230, W=250)
    w = make_workload(cfg, 1, n_templates=2, blobs_per_512sq=1200, sig_hi=20, **size)
    tms = [t.pixels for t in w.templates]
    qbar = (4, 300, 6) if w.depth == 8 else (64, 80000, 90)
    mask, lst, n, npb = _screen(runner, w.ref, tms, Fr(1, 2), Fr(2), qbar, w.feat_mask, w.depth)
    want = alg1.screen(w.ref, tms, Fr(1, 2), Fr(2), qbar, w.feat_mask)
    wmask, wlist = oc.mask_and_list(want)
    say(f"alg1 cfg{cfg}: {npb} probes, {n} candidates")
    assert n == len(wlist) and np.array_equal(lst, wlist)
