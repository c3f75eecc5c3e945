"""GPU tests of the serving loop (oss_server_*): every served result equals
the oracle's screen of that request alone, whatever it was merged with;
resident tables are reused, evicted under a budget and rebuilt when a
request needs a larger radius or another feature."""
from time import monotonic_ns as time_ns

import numpy as np
import pytest

import oracle.core as oc
from gpu_util import say
from synth import serving_requests

pytestmark = pytest.mark.gpu

TOL = (4, 8, 65, 100)


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_1707_05647_amd import _lib as L
    from paper_1707_05647_amd.screen import Server
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    return torch, L, Server, dev


def _oracle(img, templates, probes, fm, tol):
    bits = oc.screen_full(img, [(t.pixels, t.rho) for t in templates], probes, fm, tol[:3],
                          tol[3])
    return oc.mask_and_list(bits)


def _feats(L, templates, fm):
    return [L.oss_template_features(t.pixels, t.rho, fm) for t in templates]


def _small_stream(n, seed):
    return serving_requests(n, 1000.0, seed, side_lo=96, side_hi=224, reuse=0.4,
                            max_templates=3, rho_lo=6, rho_hi=20, max_scales=4,
                            blobs_per_512sq=1500)


def _check(srv, rid, img, templates, probes, fm, tol):
    mask, lst, n = srv.host_result(rid)
    wmask, wlist = _oracle(img, templates, probes, fm, tol)
    assert n == len(wlist)
    assert np.array_equal(mask, wmask)
    assert np.array_equal(lst, wlist)


def test_mixed_stream_matches_oracle(env):
    torch, L, Server, dev = env
    reqs, images = _small_stream(10, 0)
    imgs = {k: L.device_image(v, dev) for k, v in images.items()}
    srv = Server(0, 4 << 30, lanes=2, max_batch_templates=8)
    try:
        ids = []
        for q in reqs:
            say(f"serve: request {q.rid} key {q.ref_key} side {q.side} "
                f"T={len(q.templates)} probes={len(q.probes)}")
            ids.append(srv.submit(q.ref_key, imgs[q.ref_key], _feats(L, q.templates, 7),
                                  q.probes, TOL, 7, len(q.templates) * q.side * q.side))
        srv.drain()
        st = srv.stats()
        say(f"serve stats {st}")
        assert st["completed"] == len(reqs) and st["failed"] == 0
        assert st["launches"] < len(reqs)  # requests on one reference were merged
        merged = 0
        for q, rid in zip(reqs, ids):
            r = srv.result(rid)
            merged += r.batch_requests > 1
            _check(srv, rid, images[q.ref_key], q.templates, q.probes, 7, TOL)
            srv.release(rid)
        assert merged > 0
    finally:
        srv.close()


def test_merged_requests_keep_their_own_tolerance_and_features(env):
    torch, L, Server, dev = env
    reqs, images = _small_stream(6, 3)
    key = reqs[0].ref_key
    same = [q for q in reqs if q.ref_key == key][:1] * 3
    img = images[key]
    dimg = L.device_image(img, dev)
    cases = [(7, (4, 8, 65, 100)), (1, (3, 0, 0, 100)), (6, (0, 10, 40, 100))]
    srv = Server(0, 4 << 30, lanes=1, max_batch_templates=64)
    try:
        ids = [srv.submit(key, dimg, _feats(L, q.templates, fm), q.probes, tol, fm,
                          len(q.templates) * img.size)
               for q, (fm, tol) in zip(same, cases)]
        srv.drain()
        for q, (fm, tol), rid in zip(same, cases, ids):
            r = srv.result(rid)
            assert r.batch_requests == 3
            _check(srv, rid, img, q.templates, q.probes, fm, tol)
    finally:
        srv.close()


def test_resident_hit_and_rebuild_for_larger_radius(env):
    torch, L, Server, dev = env
    reqs, images = _small_stream(4, 5)
    q = reqs[0]
    img = images[q.ref_key]
    dimg = L.device_image(img, dev)
    small = [p for p in q.probes if p[2] <= 8] or q.probes[:1]
    srv = Server(0, 4 << 30, lanes=2)
    try:
        a = srv.submit(q.ref_key, dimg, _feats(L, q.templates, 7), small, TOL, 7, img.size * 4)
        srv.drain()
        b = srv.submit(q.ref_key, dimg, _feats(L, q.templates, 7), small, TOL, 7, img.size * 4)
        srv.drain()
        assert srv.result(a).resident_hit == 0 and srv.result(b).resident_hit == 1
        c = srv.submit(q.ref_key, dimg, _feats(L, q.templates, 7), q.probes, TOL, 7,
                       img.size * 4)
        srv.drain()
        st = srv.stats()
        need_more = max(p[2] for p in q.probes) > max(p[2] for p in small)
        assert st["builds"] == (2 if need_more else 1)
        for rid, pr in ((a, small), (b, small), (c, q.probes)):
            _check(srv, rid, img, q.templates, pr, 7, TOL)
    finally:
        srv.close()


def test_budget_evicts_and_results_stay_exact(env):
    torch, L, Server, dev = env
    reqs, images = _small_stream(8, 7)
    imgs = {k: L.device_image(v, dev) for k, v in images.items()}
    # room for the largest single request (tables, mask, list, workspace) and a
    # little more: most new references need an eviction
    def foot(q):
        hw = q.side * q.side
        T = len(q.templates)
        tables = L.oss_ref_bytes(L.desc_of(images[q.ref_key]), 7, max(p[2] for p in q.probes))
        return tables + T * hw * (1 + 16 + 4) + (1 << 20)
    budget = int(1.25 * max(foot(q) for q in reqs))
    srv = Server(0, budget, lanes=2)
    try:
        ids = []
        for q in reqs:
            ids.append(srv.submit(q.ref_key, imgs[q.ref_key], _feats(L, q.templates, 7),
                                  q.probes, TOL, 7, len(q.templates) * q.side * q.side))
        # pump like a serving loop, releasing results as they complete
        done = set()
        while len(done) < len(ids):
            srv.pump(2000)
            for q, rid in zip(reqs, ids):
                if rid in done:
                    continue
                r = srv.result(rid)
                if r.status == L.OSS_E_STATE:
                    continue
                assert r.status == L.OSS_OK
                _check(srv, rid, images[q.ref_key], q.templates, q.probes, 7, TOL)
                srv.release(rid)
                done.add(rid)
        st = srv.stats()
        say(f"budget {budget}: {st}")
        assert st["bytes_peak"] <= budget
        if len(images) > 1:
            assert st["evictions"] > 0
    finally:
        srv.close()


def test_request_larger_than_budget_is_refused(env):
    torch, L, Server, dev = env
    reqs, images = _small_stream(1, 9)
    q = reqs[0]
    img = images[q.ref_key]
    srv = Server(0, 1 << 16, lanes=1)
    try:
        with pytest.raises(L.OssError) as e:
            srv.submit(q.ref_key, L.device_image(img, dev), _feats(L, q.templates, 7), q.probes,
                       TOL, 7, 16)
        assert e.value.status == L.OSS_E_NOMEM
    finally:
        srv.close()


def _sampled_check(srv, rid, w, n_pos=400, seed=5):
    """A large request: the oracle at random positions (scale bits from the
    list, the mask), and the mask and list describing the same candidates."""
    mask, lst, n = srv.host_result(rid)
    assert n == len(lst) and n == int(mask.sum())
    T = len(w.templates)
    bits = np.zeros((T,) + mask.shape[1:], np.uint32)
    if n:
        bits[lst[:, 0], lst[:, 1], lst[:, 2]] = lst[:, 3].astype(np.uint32)
    assert np.array_equal(mask, (bits != 0).astype(np.uint8))
    rng = np.random.default_rng(seed)
    xs = rng.integers(0, w.W, n_pos).astype(np.int32)
    ys = rng.integers(0, w.H, n_pos).astype(np.int32)
    want = oc.screen_positions(w.ref, [(t.pixels, t.rho) for t in w.templates], w.probes,
                               w.feat_mask, w.tol_P, w.tol_Q, xs, ys)
    got = np.stack([bits[t, ys, xs] for t in range(T)])
    assert np.array_equal(got, want)


def _long_request():
    """A request whose launch runs for milliseconds: 4096^2, 8 templates x 7
    scales (the batched workload's shape) at the rotation + scale screen's
    tolerances (a few percent of positions survive)."""
    from synth import make_workload
    w = make_workload(3, 4, H=4096, W=4096, n_templates=8)
    w.tol_P = (4, 8, 65)
    return w


def test_requests_submitted_while_a_launch_runs(env):
    """Continuous batching: a request submitted while another one's launch is
    on the GPU is admitted on the second lane before the first completes; both
    results equal the oracle (the long one at sampled positions, the short one
    element by element)."""
    torch, L, Server, dev = env
    big = _long_request()
    reqs, images = _small_stream(2, 11)
    small = reqs[0]
    simg = images[small.ref_key]
    dbig = L.device_image(big.ref, dev)
    dsmall = L.device_image(simg, dev)
    srv = Server(0, 32 << 30, lanes=2, max_batch_templates=64)
    try:
        fa = [L.oss_template_features(t.pixels, t.rho, big.feat_mask) for t in big.templates]
        fb = _feats(L, small.templates, 7)
        ta = time_ns()
        a = srv.submit(1001, dbig, fa, big.probes, (*big.tol_P, big.tol_Q), big.feat_mask,
                       len(fa) * big.H * big.W, arrival_ns=ta)
        srv.pump(0)  # a launches on lane 0
        tb = time_ns()
        b = srv.submit(1002, dsmall, fb, small.probes, TOL, 7, len(fb) * simg.size,
                       arrival_ns=tb)
        srv.pump(0)  # b launches on lane 1 while a runs
        st = srv.stats()
        say(f"serve overlap: after the second pump {st}")
        srv.drain()
        ra, rb = srv.result(a), srv.result(b)
        assert ra.status == L.OSS_OK and rb.status == L.OSS_OK
        assert ra.lane != rb.lane
        b_launch = tb + rb.queue_ms * 1e6
        a_done = ta + ra.latency_ms * 1e6
        say(f"serve overlap: a done {ra.latency_ms:.2f} ms after arrival, b launched "
            f"{(b_launch - ta) / 1e6:.2f} ms after a's arrival")
        assert b_launch < a_done
        _check(srv, b, simg, small.templates, small.probes, 7, TOL)
        _sampled_check(srv, a, big)
    finally:
        srv.close()


def test_cancel_a_queued_request(env):
    torch, L, Server, dev = env
    big = _long_request()
    reqs, images = _small_stream(3, 12)
    q = reqs[0]
    img = images[q.ref_key]
    dbig = L.device_image(big.ref, dev)
    dimg = L.device_image(img, dev)
    srv = Server(0, 32 << 30, lanes=1)
    try:
        fa = [L.oss_template_features(t.pixels, t.rho, big.feat_mask) for t in big.templates]
        a = srv.submit(2001, dbig, fa, big.probes, (*big.tol_P, big.tol_Q), big.feat_mask,
                       len(fa) * big.H * big.W)
        srv.pump(0)  # a runs on the only lane
        c = srv.submit(2002, dimg, _feats(L, q.templates, 7), q.probes, TOL, 7,
                       len(q.templates) * img.size)
        d = srv.submit(2003, dimg, _feats(L, q.templates, 7), q.probes, TOL, 7,
                       len(q.templates) * img.size)
        srv.cancel(c)  # still queued
        with pytest.raises(L.OssError) as e:
            srv.cancel(a)  # launched: not interrupted
        assert e.value.status == L.OSS_E_STATE
        assert srv.result(c).status == L.OSS_E_CANCELLED
        srv.drain()
        assert srv.result(a).status == L.OSS_OK
        assert srv.result(c).status == L.OSS_E_CANCELLED
        _check(srv, d, img, q.templates, q.probes, 7, TOL)
        st = srv.stats()
        assert st["failed"] == 1 and st["completed"] == 2
        for rid in (a, c, d):
            srv.release(rid)
    finally:
        srv.close()


def test_queue_timeout(env):
    """A request that has waited past the server's queue timeout fails with
    OSS_E_TIMEOUT instead of running; a fresh one runs and equals the oracle."""
    torch, L, Server, dev = env
    reqs, images = _small_stream(2, 13)
    q = reqs[0]
    img = images[q.ref_key]
    dimg = L.device_image(img, dev)
    srv = Server(0, 4 << 30, lanes=1, queue_timeout_ns=1_000_000_000)
    try:
        late = srv.submit(q.ref_key, dimg, _feats(L, q.templates, 7), q.probes, TOL, 7,
                          len(q.templates) * img.size, arrival_ns=time_ns() - 5_000_000_000)
        fresh = srv.submit(q.ref_key, dimg, _feats(L, q.templates, 7), q.probes, TOL, 7,
                           len(q.templates) * img.size)
        srv.drain()
        assert srv.result(late).status == L.OSS_E_TIMEOUT
        assert srv.result(fresh).status == L.OSS_OK
        _check(srv, fresh, img, q.templates, q.probes, 7, TOL)
        assert srv.stats()["launches"] == 1
    finally:
        srv.close()
