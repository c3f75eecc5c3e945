"""The no-allocation screen (oss_screen_noalloc, scratch in the library's
fixed device array) against oss_screen: mask, list and count identical,
element by element, on two calls in a row (the second smaller, so stale
scratch contents from the first would show), and a screen larger than the
scratch refused with OSS_E_LIMIT before anything runs."""
import numpy as np
import pytest

from gpu_util import say
from synth import make_workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1707_05647_amd.screen import Context
    c = Context(0)
    yield c
    c.close()


def _both(ctx, w, poison=True):
    import torch

    from paper_1707_05647_amd import _lib as L
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream()
    img = L.device_image(w.ref, dev)
    ref = ctx.reference(img, w.feat_mask, w.depth, stream)
    tm = [L.oss_template_features(t.pixels, t.rho, w.feat_mask, bit_depth=w.depth)
          for t in w.templates]
    T = len(tm)
    cap = T * w.H * w.W
    out = []
    for fn in (L.oss_screen, L.oss_screen_noalloc):
        # outputs filled with values neither screen writes, so an unwritten
        # element shows
        mask = torch.full((T, w.H, w.W), 7 if poison else 0, dtype=torch.uint8, device=dev)
        cands = torch.full((cap, 4), -5, dtype=torch.int32, device=dev)
        count = torch.full((1,), -9, dtype=torch.int64, device=dev)
        fn(ctx.handle, ref.handle, tm, w.probes, (*w.tol_P, w.tol_Q), w.feat_mask, mask, cands,
           cap, count, stream)
        torch.cuda.synchronize()
        n = int(count.item())
        out.append((mask.cpu().numpy(), cands[:n].cpu().numpy(), n))
    ref.release()
    return out


def _check(ctx, w, what):
    (m0, l0, n0), (m1, l1, n1) = _both(ctx, w)
    say(f"noalloc {what}: {w.H}x{w.W}, {len(w.templates)} templates, {n0} candidates")
    assert n0 > 0
    assert n1 == n0
    assert np.array_equal(m1, m0)
    assert np.array_equal(l1, l0)


def test_noalloc_equals_screen_then_smaller(ctx):
    # a larger screen with several templates, then a smaller one right after:
    # the second call's scratch holds the first's leftovers
    big = make_workload(3, 0, H=900, W=1000, n_templates=3, blobs_per_512sq=900, sig_hi=24)
    small = make_workload(2, 1, H=260, W=330, blobs_per_512sq=1500, sig_hi=16)
    _check(ctx, big, "first call")
    _check(ctx, small, "second call (smaller)")


def test_noalloc_full_strip_shape(ctx):
    # the rotation + scale screen at a width that leaves a ragged last strip
    w = make_workload(2, 0, H=1024, W=1100, blobs_per_512sq=600, sig_hi=32)
    _check(ctx, w, "ragged strip")


def test_noalloc_beyond_scratch_is_refused(ctx):
    import torch

    from paper_1707_05647_amd import _lib as L
    dev = torch.device("cuda", 0)
    H = W = 8192  # one template needs ~537 MB of counts and staging
    img = torch.zeros((H, W), dtype=torch.uint8, device=dev)
    ref = ctx.reference(img, L.OSS_F_SUM, 8, build=False, max_radius=16)
    tm = [L.oss_template_features(np.zeros((33, 33), np.uint8), 16, L.OSS_F_SUM, bit_depth=8)]
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    with pytest.raises(L.OssError) as e:
        L.oss_screen_noalloc(ctx.handle, ref.handle, tm, [(0, 0, 16)], (1, 0, 0, 20),
                             L.OSS_F_SUM, None, None, 0, count)
    assert e.value.status == L.OSS_E_LIMIT
    ref.release()
