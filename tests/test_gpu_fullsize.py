"""Full-size parity of the batched workloads, in the launch configuration the
benchmark times: 8192^2 uint8 with 64 templates x 7 scales (interleaved and
planar tables) and 16384^2 12-bit with 16 rotations x 32 radii (planar
tables with split 64-bit squares), each after the autotuner has picked the
launch shape.  The oracle cannot screen these images whole, so:
  * on sampled positions (uniform, the planted centres, the first and last
    valid rows and columns of the smallest and largest radius) the scale
    bits of every template, read from the candidate list, and the mask are
    bit-exact against the oracle;
  * everywhere: the list is strictly increasing in (t, y, x), holds exactly
    the mask's positions, and carries non-zero scale bits;
  * every position of a 64-row band (all columns for the 8192^2 workload,
    4096 columns for the 16384^2 one) bit-exact against the oracle.
"""
import numpy as np
import pytest

import oracle.core as oc
from synth import make_workload

from gpu_util import Runner, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def runner():
    r = Runner()
    yield r
    r.close()


def _sample(w, n, rng):
    rmin = min(p[2] for p in w.probes)
    rmax = max(p[2] for p in w.probes)
    xs = [rng.integers(0, w.W, n)]
    ys = [rng.integers(0, w.H, n)]
    edge = []
    for r in (rmin, rmax):
        for v in (r - 1, r, w.W - 1 - r, w.W - r):
            edge.append((v, w.H // 2))
        for v in (r - 1, r, w.H - 1 - r, w.H - r):
            edge.append((w.W // 3, v))
        edge += [(r, r), (w.W - 1 - r, w.H - 1 - r)]
    edge += [(t.cx, t.cy) for t in w.templates]
    xs.append(np.array([e[0] for e in edge]))
    ys.append(np.array([e[1] for e in edge]))
    xs = np.clip(np.concatenate(xs), 0, w.W - 1).astype(np.int32)
    ys = np.clip(np.concatenate(ys), 0, w.H - 1).astype(np.int32)
    return xs, ys


def _band_check(w, T, HW, c, keys, mask, y0, dev, x0=0, x1=None):
    """A 64-row band, every position of columns [x0, x1): the oracle's scale
    bits of every template against the list's, and the mask."""
    import torch
    y1 = min(w.H, y0 + 64)
    x1 = w.W if x1 is None else x1
    ys, xs = np.mgrid[y0:y1, x0:x1]
    xs = xs.ravel().astype(np.int32)
    ys = ys.ravel().astype(np.int32)
    # probes sorted by radius: the oracle sums each star once per radius
    probes = sorted(w.probes, key=lambda p: p[2])
    say(f"  oracle on rows {y0}..{y1 - 1}, columns {x0}..{x1 - 1} ({len(xs)} positions)")
    want = oc.screen_positions(w.ref, [(t.pixels, t.rho) for t in w.templates], probes,
                               w.feat_mask, w.tol_P, w.tol_Q, xs, ys)
    got = np.zeros_like(want)
    bw = x1 - x0
    for t in range(T):
        a = int(torch.searchsorted(keys, torch.tensor([t * HW + y0 * w.W], device=dev)))
        b = int(torch.searchsorted(keys, torch.tensor([t * HW + y1 * w.W], device=dev)))
        sel = c[a:b].cpu().numpy().astype(np.int64)
        sel = sel[(sel[:, 2] >= x0) & (sel[:, 2] < x1)]
        if len(sel):
            idx = (sel[:, 1] - y0) * bw + (sel[:, 2] - x0)
            got[t, idx] = sel[:, 3].astype(np.uint32)
    bad = np.argwhere(got != want)
    assert len(bad) == 0, f"band rows {y0}..{y1 - 1}: {len(bad)} (t, position) pairs differ"
    gm = mask[:, y0:y1, x0:x1].reshape(T, -1).cpu().numpy()
    assert np.array_equal(gm, (want != 0).astype(np.uint8))
    return int((want != 0).sum())


def _full_size(runner, cfg, planar, n_sample, band):
    torch, L = runner.torch, runner.L
    dev = runner.dev
    h = runner.ctx.handle
    w = make_workload(cfg, 0, device=dev)
    T = len(w.templates)
    say(f"full size workload {cfg}: {w.H}x{w.W}, {T} templates, {len(w.probes)} probes, "
        f"planar={planar}")
    img = L.device_image(w.ref, dev)
    L.oss_ctx_set_option(h, L.OSS_OPT_TABLE_PLANAR, planar)
    try:
        ref = runner.ctx.reference(img, w.feat_mask, w.depth, max_radius=max(w.radii()))
    finally:
        L.oss_ctx_set_option(h, L.OSS_OPT_TABLE_PLANAR, 1)
    assert (ref.plane_bytes > 0) == bool(planar)
    tm = [L.oss_template_features(t.pixels, t.rho, w.feat_mask, bit_depth=w.depth)
          for t in w.templates]
    tol = (*w.tol_P, w.tol_Q)
    opts = (L.OSS_OPT_STAR_STRIP, L.OSS_OPT_STAR_BLOCKS_PER_XCD, L.OSS_OPT_BATCH_BUCKET)
    old = [L.oss_ctx_get_option(h, o) for o in opts]
    try:
        tr = L.oss_autotune_batched(h, ref.handle, tm, w.probes, tol, w.feat_mask)
        say(f"  autotuned: strip {tr.strip}, {tr.blocks_per_xcd} blocks per XCD, "
            f"bucket {tr.bucket_radii}, {tr.ms:.2f} ms")
        HW = w.H * w.W
        mask = torch.empty((T, w.H, w.W), dtype=torch.uint8, device=dev)
        cap = int(0.4 * T * HW)
        cands = torch.empty((cap, 4), dtype=torch.int32, device=dev)
        count = torch.zeros(1, dtype=torch.int64, device=dev)
        L.oss_screen(h, ref.handle, tm, w.probes, tol, w.feat_mask, mask, cands, cap, count,
                     batched=True)
        torch.cuda.synchronize()
    finally:
        for o, v in zip(opts, old):
            L.oss_ctx_set_option(h, o, v)
    ref.release()
    del img
    n = int(count.item())
    say(f"  {n} candidates")
    assert 0 < n <= cap
    # everywhere: list sorted, list == mask, scale bits non-zero
    c = cands[:n]
    keys = c[:, 0].to(torch.int64) * HW + c[:, 1].to(torch.int64) * w.W + c[:, 2].to(torch.int64)
    assert bool((keys[1:] > keys[:-1]).all())
    assert int(mask.sum(dtype=torch.int64)) == n
    assert bool((mask.view(-1)[keys] == 1).all())
    assert bool((c[:, 3] != 0).all())
    # sampled positions against the oracle
    rng = np.random.default_rng(cfg)
    xs, ys = _sample(w, n_sample, rng)
    say(f"  oracle on {len(xs)} sampled positions")
    want = oc.screen_positions(w.ref, [(t.pixels, t.rho) for t in w.templates], w.probes,
                               w.feat_mask, w.tol_P, w.tol_Q, xs, ys)
    pos = torch.from_numpy(ys.astype(np.int64) * w.W + xs).to(dev)
    got = np.zeros_like(want)
    for t in range(T):
        k = pos + t * HW
        i = torch.searchsorted(keys, k).clamp_(max=n - 1)
        hit = keys[i] == k
        got[t] = torch.where(hit, c[i, 3], torch.zeros_like(c[i, 3])).cpu().numpy().view(np.uint32)
    bad = np.argwhere(got != want)
    assert len(bad) == 0, (f"{len(bad)} of {want.size} (template, position) pairs differ; first "
                           f"(t, i): {bad[:5].tolist()}")
    gm = mask[:, torch.from_numpy(ys.astype(np.int64)).to(dev),
              torch.from_numpy(xs.astype(np.int64)).to(dev)].cpu().numpy()
    assert np.array_equal(gm, (want != 0).astype(np.uint8))
    assert want.any(axis=1).all()  # every template has sampled candidates
    nb = _band_check(w, T, HW, c, keys, mask, band[0], dev, band[1], band[2])
    say(f"  band: {nb} candidates, bit-exact")
    del mask, cands, count, c, keys, pos
    torch.cuda.empty_cache()


@pytest.mark.parametrize("planar", [0, 1], ids=["interleaved", "planar"])
def test_cfg3_full_size_sampled(runner, planar):
    # the band: the top 64 rows, every column, where radii turn valid one by one
    _full_size(runner, 3, planar, 400, (0, 0, None))


def test_cfg5_full_size_sampled(runner):
    # the band: 64 rows through the middle (every radius valid), 4096 columns
    # (eight 512-column strips: strip and XCD boundaries inside); every
    # column of it would take minutes of oracle time
    _full_size(runner, 5, 1, 1500, (16384 // 2 - 32, 6144, 10240))
