"""GPU parity of the multi-central-area screen (oss_screen_rings) with the
oracle's ring screen, element by element, on every workload shape and
entry layout, and its reduction to the plain screen at one ring."""
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


def _rings(runner, w, n_rings, max_r=-1):
    L = runner.L
    img = L.device_image(w.ref, runner.dev)
    if max_r == -2:
        max_r = max(p[2] for p in w.probes)
    ref = runner.ctx.reference(img, w.feat_mask, w.depth, max_radius=max_r)
    tm = [L.oss_template_features_rings(t.pixels, t.rho, w.feat_mask, n_rings, bit_depth=w.depth)
          for t in w.templates]
    torch = runner.torch
    T = len(tm)
    mask = torch.empty((T, w.H, w.W), dtype=torch.uint8, device=runner.dev)
    cap = T * w.H * w.W
    cands = torch.empty((cap, 4), dtype=torch.int32, device=runner.dev)
    count = torch.zeros(1, dtype=torch.int64, device=runner.dev)
    L.oss_screen_rings(runner.ctx.handle, ref.handle, tm, w.probes, (*w.tol_P, w.tol_Q),
                       w.feat_mask, mask, cands, cap, count)
    torch.cuda.synchronize()
    n = int(count.item())
    c = cands[:n].cpu().numpy().astype(np.int64)
    c[:, 3] &= 0xFFFFFFFF
    out = (mask.cpu().numpy(), c, n, ref.entry_bytes)
    ref.release()
    return out


def _oracle(w, n_rings):
    bits = oc.screen_rings_full(w.ref, [(t.pixels, t.rho) for t in w.templates], w.probes,
                                w.feat_mask, w.tol_P, w.tol_Q, n_rings)
    return oc.mask_and_list(bits)


CASES = {
    1: dict(),
    2: dict(H=230, W=270, blobs_per_512sq=800, sig_hi=24),
    3: dict(H=200, W=260, n_templates=5, blobs_per_512sq=1200, sig_hi=20),
    5: dict(H=224, W=240, n_templates=3, blobs_per_512sq=1200, sig_hi=20),
}


@pytest.mark.parametrize("n_rings", [1, 2, 3])
@pytest.mark.parametrize("cfg", sorted(CASES))
def test_rings_equal_oracle(runner, cfg, n_rings):
    w = make_workload(cfg, 2, **CASES[cfg])
    say(f"rings cfg{cfg} n_rings={n_rings} probes={len(w.probes)}")
    mask, lst, n, eb = _rings(runner, w, n_rings, -2)
    wmask, wlist = _oracle(w, n_rings)
    say(f"  {eb} B entries, {n} candidates (oracle {len(wlist)})")
    assert n == len(wlist) and np.array_equal(mask, wmask) and np.array_equal(lst, wlist)


def test_one_ring_is_the_plain_screen(runner):
    w = make_workload(2, 4, **CASES[2])
    tm = [(t.pixels, t.rho) for t in w.templates]
    plain = runner.screen(w.ref, tm, w.probes, w.feat_mask, w.tol_P, w.tol_Q)
    mask, lst, n, _ = _rings(runner, w, 1)
    assert n == plain[2] and np.array_equal(lst, plain[1])


@pytest.mark.parametrize("max_r", [-2, 1 << 20], ids=["narrow", "w64"])
def test_rings_many_templates(runner, max_r):
    """12 templates: the 32-slot register accumulators of the ring kernel."""
    w = make_workload(3, 6, H=180, W=200, n_templates=12, blobs_per_512sq=1500, sig_hi=16)
    mask, lst, n, _ = _rings(runner, w, 3, max_r)
    wmask, wlist = _oracle(w, 3)
    assert n == len(wlist) and np.array_equal(lst, wlist)
