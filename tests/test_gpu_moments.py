"""GPU parity of the screen with the paper's own features (mean, variance,
first-moment gradient magnitude; oss_screen_moments) with the oracle,
element by element, on 8-bit (32-bit tables) and 12-bit (64-bit tables)
workloads and for each test alone."""
import numpy as np
import pytest

import oracle.core as oc
from gpu_util import Runner, say
from oracle import moments as om
from synth import blob_image, cut_patch, make_rng, make_workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def runner():
    r = Runner()
    yield r
    r.close()


def _screen(runner, img, templates, probes, tol, tests, fm, depth, max_r, planar=1):
    L = runner.L
    torch = runner.torch
    h = runner.ctx.handle
    L.oss_ctx_set_option(h, L.OSS_OPT_TABLE_PLANAR, planar)
    try:
        ref = runner.ctx.reference(L.device_image(img, runner.dev), fm, depth, max_radius=max_r)
    finally:
        L.oss_ctx_set_option(h, L.OSS_OPT_TABLE_PLANAR, 1)
    assert (ref.plane_bytes > 0) == bool(planar)
    tm = [L.oss_template_moments(px, rho, bit_depth=depth) for px, rho in templates]
    T = len(tm)
    H, W = img.shape
    mask = torch.empty((T, H, W), dtype=torch.uint8, device=runner.dev)
    cap = T * H * W
    cands = torch.empty((cap, 4), dtype=torch.int32, device=runner.dev)
    count = torch.zeros(1, dtype=torch.int64, device=runner.dev)
    L.oss_screen_moments(runner.ctx.handle, ref.handle, tm, probes, tol, tests, mask, cands, cap,
                         count)
    torch.cuda.synchronize()
    n = int(count.item())
    c = cands[:n].cpu().numpy().astype(np.int64)
    c[:, 3] &= 0xFFFFFFFF
    out = mask.cpu().numpy(), c, n, ref.value_bits
    ref.release()
    return out


def _check(runner, img, templates, probes, tol, tests, fm, depth, max_r, planar=1):
    mask, lst, n, vb = _screen(runner, img, templates, probes, tol, tests, fm, depth, max_r,
                               planar)
    want = om.screen_full(img, templates, probes, tol[:3], tol[3], tests)
    wmask, wlist = oc.mask_and_list(want)
    say(f"  moments tests={tests} fm={fm} {vb}-bit: {n} candidates (oracle {len(wlist)})")
    assert n == len(wlist) and np.array_equal(mask, wmask) and np.array_equal(lst, wlist)
    return n


PLANAR = pytest.mark.parametrize("planar", [1, 0], ids=["planar", "interleaved"])


@PLANAR
@pytest.mark.parametrize("tests", [1, 2, 4, 7])
def test_moments_cfg2(runner, tests, planar):
    """Planar tables take the staged lookups (the mean first; without a mean
    test every position goes on); interleaved ones read every quantity."""
    w = make_workload(2, 2, H=150, W=170, blobs_per_512sq=1200, sig_hi=20)
    tms = [(t.pixels, t.rho) for t in w.templates]
    probes = [p for p in w.probes if 2 * p[2] + 1 <= 150]
    n = _check(runner, w.ref, tms, probes, (6, 30, 40, 100), tests, 27, 8,
               max(p[2] for p in probes), planar)
    assert n > 0


@PLANAR
def test_moments_cfg5_64bit(runner, planar):
    w = make_workload(5, 3, H=230, W=250, n_templates=2, blobs_per_512sq=1200, sig_hi=20)
    tms = [(t.pixels, t.rho) for t in w.templates]
    probes = [p for p in w.probes if p[2] <= 60]
    _check(runner, w.ref, tms, probes, (8, 40, 50, 100), 7, 27, 12, max(p[2] for p in probes),
           planar)


def test_moments_mean_and_magnitude_only(runner):
    """Sum and moments only (no squares), exact cuts at P = 0 survive."""
    img = blob_image(120, 140, make_rng(94, 0), blobs_per_512sq=1500, sig_hi=10)
    tms = [(cut_patch(img, 60, 55, 12), 11), (cut_patch(img, 90, 70, 9, quarter_turns=1), 8)]
    probes = [(0, 0, 11), (0, 1, 9), (1, 0, 8), (1, 2, 12)]
    mask, lst, n, _ = _screen(runner, img, tms, probes, (0, 0, 0, 1), 5, 25, 8, 12)
    want = om.screen_full(img, tms, probes, (0, 0, 0), 1, 5)
    assert np.array_equal(lst, oc.mask_and_list(want)[1])
    assert mask[0, 55, 60] == 1 and mask[1, 70, 90] == 1


def _var_limit_radius(maxv):
    """Largest radius whose variance terms A(r)^2 maxv^2 stay below the
    library's int64 bound (9.2e18, just under 2^63)."""
    r = 1
    while oc.star_area(r + 1) ** 2 * maxv * maxv < 9.2e18:
        r += 1
    return r


def test_moments_16bit_variance_at_its_limit(runner):
    """16-bit data at the largest radius whose int64 variance terms cannot
    overflow: element by element equal to the oracle (exact integers); one
    radius more is refused with OSS_E_OVERFLOW before anything runs."""
    L = runner.L
    r_ok = _var_limit_radius(65535)
    H, W = 2 * r_ok + 27, 2 * r_ok + 45
    img = (blob_image(H, W, make_rng(97, 0), blobs_per_512sq=1500, sig_hi=12,
                      depth=12).astype(np.uint32) * 16).astype(np.uint16)
    cy, cx = H // 2, W // 2
    tms = [(cut_patch(img, cx, cy, r_ok), r_ok)]
    probes = [(0, 0, r_ok)]
    say(f"  16-bit variance limit radius {r_ok} on {H}x{W}")
    n = _check(runner, img, tms, probes, (6, 30, 40, 100), 7, 27, 16, r_ok)
    assert n > 0
    # one radius more: the template features at r_ok + 1 need a bigger cut
    img2 = np.zeros((H + 4, W + 4), np.uint16)
    img2[:H, :W] = img
    ref = runner.ctx.reference(L.device_image(img2, runner.dev), 27, 16, max_radius=r_ok + 1)
    tm = [L.oss_template_moments(cut_patch(img2, cx + 1, cy + 1, r_ok + 1), r_ok + 1,
                                 bit_depth=16)]
    count = runner.torch.zeros(1, dtype=runner.torch.int64, device=runner.dev)
    with pytest.raises(L.OssError) as e:
        L.oss_screen_moments(runner.ctx.handle, ref.handle, tm, [(0, 0, r_ok + 1)],
                             (6, 30, 40, 100), 7, None, None, 0, count)
    assert e.value.status == L.OSS_E_OVERFLOW
    ref.release()
