"""GPU parity of the batched screen (one persistent launch for every
template and probe) against the per-template screen and the oracle, for
several bucketings and launch shapes, and the autotuner's contract."""
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


def _screen(runner, w, batched, max_r=-1):
    L = runner.L
    torch = runner.torch
    img = L.device_image(w.ref, runner.dev)
    ref = runner.ctx.reference(img, w.feat_mask, w.depth, max_radius=max_r)
    tm = [L.oss_template_features(t.pixels, t.rho, w.feat_mask, bit_depth=w.depth)
          for t in w.templates]
    res = runner.ctx.screen(ref, tm, w.probes, (*w.tol_P, w.tol_Q), w.feat_mask,
                            list_cap=len(tm) * w.H * w.W, batched=batched)
    torch.cuda.synchronize()
    out = res.host()
    ref.release()
    return out


def _with_options(runner, opts, fn):
    L = runner.L
    h = runner.ctx.handle
    old = {o: L.oss_ctx_get_option(h, o) for o in opts}
    for o, v in opts.items():
        L.oss_ctx_set_option(h, o, v)
    try:
        return fn()
    finally:
        for o, v in old.items():
            L.oss_ctx_set_option(h, o, v)


@pytest.mark.parametrize("bucket", [0, 1, 3])
def test_batched_equals_oracle_cfg3(runner, bucket):
    w = make_workload(3, 0, H=200, W=260, n_templates=6, blobs_per_512sq=1200, sig_hi=20)
    say(f"batched cfg3 bucket={bucket} probes={len(w.probes)}")
    got = _with_options(runner, {runner.L.OSS_OPT_BATCH_BUCKET: bucket},
                        lambda: _screen(runner, w, True))
    want = oc.screen_full(w.ref, [(t.pixels, t.rho) for t in w.templates], w.probes,
                          w.feat_mask, w.tol_P, w.tol_Q)
    wmask, wlist = oc.mask_and_list(want)
    assert got[2] == len(wlist) and np.array_equal(got[0], wmask)
    assert np.array_equal(got[1], wlist)


@pytest.mark.parametrize("n_t", [40, 70])
def test_batched_equals_plain_many_templates(runner, n_t):
    """40 templates: one group, its slots 32.. in the second register half;
    70: two groups (64 + 6).  The per-template screen equals the oracle;
    every batched launch shape equals it."""
    w = make_workload(3, 2, H=192, W=224, n_templates=n_t, blobs_per_512sq=1500, sig_hi=16)
    say(f"batched vs plain: {len(w.templates)} templates, {len(w.probes)} probes")
    a = _screen(runner, w, False)
    want = oc.screen_full(w.ref, [(t.pixels, t.rho) for t in w.templates],
                          sorted(w.probes, key=lambda p: p[2]), w.feat_mask, w.tol_P, w.tol_Q)
    wmask, wlist = oc.mask_and_list(want)
    assert a[2] == len(wlist) and np.array_equal(a[0], wmask) and np.array_equal(a[1], wlist)
    for opts in ({}, {runner.L.OSS_OPT_BATCH_BUCKET: 2},
                 {runner.L.OSS_OPT_STAR_STRIP: 128, runner.L.OSS_OPT_STAR_BLOCKS_PER_XCD: 5}):
        b = _with_options(runner, opts, lambda: _screen(runner, w, True))
        assert a[2] == b[2] and np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), opts


@pytest.mark.parametrize("max_r", [-2, 1 << 20], ids=["w32", "w64"])
def test_batched_cfg5_rotations(runner, max_r):
    w = make_workload(5, 1, H=230, W=250, n_templates=4, blobs_per_512sq=1200, sig_hi=20)
    if max_r == -2:
        max_r = max(p[2] for p in w.probes)
    a = _screen(runner, w, False, max_r)
    b = _screen(runner, w, True, max_r)
    assert a[2] == b[2] and np.array_equal(a[1], b[1])
    want = oc.screen_full(w.ref, [(t.pixels, t.rho) for t in w.templates], w.probes,
                          w.feat_mask, w.tol_P, w.tol_Q)
    assert np.array_equal(b[1], oc.mask_and_list(want)[1])


def test_batched_template_without_probes(runner):
    w = make_workload(3, 4, H=160, W=160, n_templates=3, blobs_per_512sq=1500, sig_hi=16)
    probes = [p for p in w.probes if p[0] != 1]
    w.probes = probes
    a = _screen(runner, w, False)
    b = _screen(runner, w, True)
    assert np.array_equal(a[1], b[1]) and not b[0][1].any()


def test_autotune_picks_a_candidate_and_keeps_results(runner):
    L = runner.L
    w = make_workload(3, 5, H=256, W=320, n_templates=5, blobs_per_512sq=1200, sig_hi=20)
    before = _screen(runner, w, True)
    img = L.device_image(w.ref, runner.dev)
    ref = runner.ctx.reference(img, w.feat_mask, 8)
    tm = [L.oss_template_features(t.pixels, t.rho, w.feat_mask) for t in w.templates]
    h = runner.ctx.handle
    opts = (L.OSS_OPT_STAR_STRIP, L.OSS_OPT_STAR_BLOCKS_PER_XCD, L.OSS_OPT_BATCH_BUCKET)
    old = [L.oss_ctx_get_option(h, o) for o in opts]
    try:
        res = L.oss_autotune_batched(h, ref.handle, tm, w.probes, (*w.tol_P, w.tol_Q),
                                     w.feat_mask)
        runner.torch.cuda.synchronize()
        assert res.n_tried >= 6 and res.ms > 0
        times = [res.tried_ms[i] for i in range(res.n_tried)]
        assert abs(min(times) - res.ms) < 1e-6
        assert [L.oss_ctx_get_option(h, o) for o in opts] == [res.strip, res.blocks_per_xcd,
                                                               res.bucket_radii]
        after = _screen(runner, w, True)
    finally:
        for o, v in zip(opts, old):
            L.oss_ctx_set_option(h, o, v)
        ref.release()
    assert before[2] == after[2] and np.array_equal(before[1], after[1])
