#!/usr/bin/env python3
"""Screening throughput on one MI355X.

Default line (no --workload): the large batched screen, a 16384x16384
12-bit blob + noise reference, one radius-48 template at 16 rotations, 32
radii from 24 to 96 (512 probes), features sum / sum of squares / gradient
sum, int64 arithmetic, all probes in one batched persistent launch.  One
step is the whole hot path on inputs already in HBM: template features
(host), the integral-table build, the star + compare pass and the candidate
compaction (mask + list).  The same line nests a short run of the
rotation + scale screen (4096x4096 uint8, 7 radii) under ``workload_2`` and
of the serving loop (Poisson requests, served p50 / p99) under ``serving``.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload {2,3,4,5}]

Prints one JSON line.  ``value`` is screened pixel-scales per second (one
pixel-scale = one valid (position, probe) pair), in G/s.  ``roofline``
reports the dominant kernel's algorithmic HBM bytes per launch (the tables
read once plus the method's own outputs) over its average duration, timed
with HIP events recorded by the library on the launch stream over the
timed steps; ``copy_peak_GBps`` is a plain device copy timed the same way.
``cpu_baseline`` times the CPU oracle on a bounded random sample of the
same workload (and checks the GPU result at those positions bit for bit).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, AMD published peak
L1_PEAK_GBPS = 256 * 64 * 2.4  # 256 CUs x 64 B/clk x 2.4 GHz vector L1 delivery
METRIC = "screened pixel-scales/s (G/s) & % HBM peak; bit-exact mask; served p50/p99 ms"
# arithmetic: star sums and compares in int64; table entries stored modulo
# 2^32 wherever every region sum they serve is provably below 2^32
DTYPE = "int64 (sums and compares; tables mod 2^32 where exact)"
BATCH_GROUP = 64        # templates per batched group (no rings)
BATCH_GROUP_RINGS = 32  # templates per batched group with central-star rings


def pixel_scales(H, W, probes):
    """Valid (position, probe) pairs."""
    return sum(max(0, H - 2 * r) * max(0, W - 2 * r) for _, _, r in probes)


def lookup_pairs(w, batched=False, group=None, rings=1):
    """Valid (position, radius) pairs whose star sums a launch evaluates, each
    8 table lookups per quantity: one per (template, distinct radius) for
    per-template launches; one per (template group, distinct radius) for the
    batched launch (templates sorted by radius, groups of 64, 32 with
    rings)."""
    if group is None:
        group = BATCH_GROUP_RINGS if rings > 1 else BATCH_GROUP

    def chain(r):
        out = [r]
        for _ in range(rings - 1):  # central-star radii s(r), s(s(r)), ...
            out.append((math.isqrt(2 * out[-1] ** 2) + 1) // 2 if out[-1] else 0)
        return out
    if batched:
        order = sorted(range(len(w.templates)), key=lambda t: w.templates[t].rho)
        gid = {t: i // group for i, t in enumerate(order)}
        pairs = set((gid[t], rj) for t, _, r in w.probes for rj in chain(r))
    else:
        pairs = set((t, rj) for t, _, r in w.probes for rj in chain(r))
    return sum(max(0, w.H - 2 * r) * max(0, w.W - 2 * r) for _, r in pairs)


def ref_nq(feat_mask):
    return bin(feat_mask).count("1")


def algorithmic_bytes(H, W, n_tmpl, px_bytes, entry_bytes, n_cand=0):
    """Minimum HBM bytes per launch of each kernel, counting only what the
    method itself must move: the image once, the three tables once (written
    by the build, read by the screen: entry_bytes per entry), the uint8 mask
    (one byte per template and position) and the candidate list (16 bytes
    per candidate).  Scratch of the implementation (scale-bit words, staged
    candidates, segment counts) is not algorithmic."""
    table = 3 * (H + 1) * (W + 1) * entry_bytes
    hw = H * W
    return {
        # writes every table entry once, reads the image once
        "band_final": table + hw * px_bytes,
        # reads every table entry once, writes the mask
        "star_plain": table + n_tmpl * hw,
        "star_batch": table + n_tmpl * hw,
        "star_moments": table + n_tmpl * hw,
        # writes the candidate list
        "compact_list": 16 * n_cand,
        "row_base": hw * px_bytes,
        "band_agg": hw * px_bytes,
    }


# committed rocprofv3 counter summaries, per workload
TRAFFIC_FILES = {
    2: os.path.join(ROOT, "profiles", "traffic_4096_u8_7radii.json"),
    5: os.path.join(ROOT, "profiles", "traffic_16384_12bit_512probes.json"),
}


def traffic_for(kernel: str, workload: int):
    """HBM bytes per launch from the committed rocprofv3 counter runs of this
    workload, if they were taken on the current kernel source."""
    path = TRAFFIC_FILES.get(workload)
    if path is None:
        return None
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    ent = t.get("kernels", {}).get(kernel)
    from paper_1707_05647_amd.traffic import KERNELS, kernel_sha
    if not ent or kernel not in KERNELS or ent.get("source_sha") != kernel_sha(kernel):
        return None
    return ent.get("hbm_bytes_per_launch")


def cpu_baseline(w, bits_gpu, seconds: float, seed: int = 1, gpu_bits=None, gpu_mask=None,
                 list_complete=True, rings=1):
    """The oracle as it stands, on a random sample of positions of the same
    workload, timed; and the GPU's scale bits (and mask) at those positions
    compared with the oracle's."""
    import numpy as np

    import oracle.core as oc
    tm = [(t.pixels, t.rho) for t in w.templates]
    G = oc.gradient(w.ref)
    rng = np.random.default_rng(seed)
    rmin = min(p[2] for p in w.probes)

    def sample(n):
        xs = rng.integers(rmin, w.W - rmin, n).astype(np.int32)
        ys = rng.integers(rmin, w.H - rmin, n).astype(np.int32)
        return xs, ys

    def valid_pairs(xs, ys):
        tot = 0
        for _, _, r in w.probes:
            tot += int(((xs >= r) & (xs <= w.W - 1 - r) & (ys >= r) & (ys <= w.H - 1 - r)).sum())
        return tot

    def screen(xs, ys):
        if rings > 1:
            return oc.screen_rings_positions(w.ref, tm, w.probes, w.feat_mask, w.tol_P, w.tol_Q,
                                             rings, xs, ys, G=G)
        return oc.screen_positions(w.ref, tm, w.probes, w.feat_mask, w.tol_P, w.tol_Q, xs, ys,
                                   G=G)

    # size the sample from a probe run long enough (>= 0.5 s) that the
    # oracle's fixed cost per call does not inflate the per-position time
    n0 = 512 if len(w.probes) > 50 else 4096
    while True:
        xs, ys = sample(n0)
        t0 = time.perf_counter()
        screen(xs, ys)
        dt = max(time.perf_counter() - t0, 1e-4)
        if dt >= 0.5 or n0 >= 2_000_000 or 4 * dt > seconds:
            break
        n0 *= 4
    n = int(max(n0, min(8_000_000, n0 * seconds / dt)))
    xs, ys = sample(n)
    t0 = time.perf_counter()
    bits = screen(xs, ys)
    dt = time.perf_counter() - t0
    pairs = valid_pairs(xs, ys)
    if gpu_bits is None:
        got = np.stack([bits_gpu[t, ys, xs] for t in range(len(tm))])
    else:
        got = gpu_bits(ys, xs)
    exact = bool((got == bits).all()) if list_complete else None
    res = {
        "value": pairs / dt / 1e9,
        "unit": "G pixel-scales/s",
        "cores": oc.threads(),
        "kind": "oracle",
        "sample": f"{n} uniform random positions x {len(w.probes)} probes "
                  f"({pairs} valid pixel-scales), {dt:.1f} s",
        "gpu_bit_exact_on_sample": exact,
    }
    if gpu_mask is not None:
        res["gpu_mask_exact_on_sample"] = bool((gpu_mask(ys, xs) == (bits != 0)).all())
    return res


WORKLOAD_TEXT = {
    2: "rotation+scale: 4096x4096 uint8 blob+noise reference, 1 template (bilinear rotate + "
       "scale), radii 16..64 step 8, sum/squares/gradient",
    3: "batched: 8192x8192 uint8 reference, 64 templates of radius U{8..96} (rotated + scaled), "
       "7 scales 0.5..2.0 each, one batched launch",
    5: "large batched: 16384x16384 12-bit reference, one radius-48 template at 16 rotations, "
       "32 radii 24..96, one batched launch",
    4: "serving: Poisson requests at 80% of the per-request scheme's capacity; square uint8 "
       "references, side log-uniform 1024..8192, 30% resident reuse, 1..8 templates rho U{8..128}, "
       "1..9 scales geometric in [0.5, 2]",
}


class ScreenGate:
    """Keeps the lanes' screens from running at the same time: a lane's
    screen waits (on the GPU, through an event) for the previous lane's
    screen to end, while its build does not wait, so builds still overlap
    screens but two star passes never share the L2."""

    def __init__(self, torch):
        self.torch = torch
        self.last = None

    def wait(self, st):
        if self.last is not None:
            st.wait_event(self.last)

    def record(self, st):
        ev = self.torch.cuda.Event()
        ev.record(st)
        self.last = ev


def run_pipelined(lanes, make_lane, steps, warmup, L, torch):
    """Steps dealt round-robin to `lanes` lanes (a context, a stream, tables
    and outputs each): step i runs on lane i mod lanes, so the builder of one
    batch can run beside the star pass of the previous one.  Returns seconds
    per step and the lanes' summed kernel profiles."""
    ls = [make_lane() for _ in range(lanes)]
    for i in range(warmup * lanes):
        ls[i % lanes]["step"]()
    torch.cuda.synchronize()
    for ln in ls:
        L.oss_ctx_profile(ln["ctx"].handle, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        ls[i % lanes]["step"]()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = {}
    for ln in ls:
        L.oss_ctx_profile(ln["ctx"].handle, False)
        for k, v in L.oss_ctx_profile_read(ln["ctx"].handle).items():
            a = prof.setdefault(k, [0, 0.0, 0.0])
            a[0] += v[0]
            a[1] += v[1]
            a[2] = max(a[2], v[2])
    return (t1 - t0) / steps, prof, ls


OPTIONS = ("OSS_OPT_STAR_STRIP", "OSS_OPT_STAR_BLOCKS_PER_XCD", "OSS_OPT_STAR_LDS",
           "OSS_OPT_BATCH_BUCKET", "OSS_OPT_TABLE_PLANAR", "OSS_OPT_STAR_PIPE",
           "OSS_OPT_STAR_STAGED", "OSS_OPT_BUILD_STREAM", "OSS_OPT_TABLE_REC")


_LANE_STREAMS = []


def lane_stream(torch, dev, i):
    """Lane i's stream, created once per process and reused by every
    workload: HIP maps streams onto a few hardware queues in turn, so fresh
    streams for a later workload can share a queue (and serialise) with each
    other."""
    while len(_LANE_STREAMS) <= i:
        _LANE_STREAMS.append(torch.cuda.Stream(device=dev))
    return _LANE_STREAMS[i]


def pipelined(args, n_lanes, w, L, torch, dev, ctx, img, ref_fm, max_r, cap, batched,
              screen_step, n, mask, cands):
    """The same steps over `n_lanes` lanes (contexts with the main context's
    options, own streams, tables and outputs).  Returns seconds per step, the
    lanes' kernel profile and whether every lane's last result equals the
    single-lane run's."""
    from paper_1707_05647_amd.screen import Context
    gate = ScreenGate(torch) if args.serial_screens else None
    made = []

    def make_lane():
        c = Context(0)
        for o in OPTIONS:
            L.oss_ctx_set_option(c.handle, getattr(L, o),
                                 L.oss_ctx_get_option(ctx.handle, getattr(L, o)))
        st = lane_stream(torch, dev, len(made))
        made.append(st)
        r = c.reference(img, ref_fm, w.depth, build=False, max_radius=max_r)
        m = torch.empty_like(mask)
        cd = torch.empty((cap, 4), dtype=torch.int32, device=dev)
        cn = torch.zeros(1, dtype=torch.int64, device=dev)

        def step():
            screen_step(c.handle, r, st, m, cd, cn, batched, gate)
        return {"ctx": c, "ref": r, "step": step, "mask": m, "cands": cd, "count": cn}

    sec, prof, lanes = run_pipelined(n_lanes, make_lane, args.steps, args.warmup, L, torch)
    k = min(n, cap)
    same = all(int(ln["count"].item()) == n and torch.equal(ln["mask"], mask)
               and torch.equal(ln["cands"][:k], cands[:k]) for ln in lanes)
    for ln in lanes:
        ln["ref"].release()
        ln["ctx"].close()
    return sec, prof, same


def run_steps(step, steps, warmup, ctx, L, torch):
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    L.oss_ctx_profile(ctx.handle, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    L.oss_ctx_profile(ctx.handle, False)
    return (t1 - t0) / steps, L.oss_ctx_profile_read(ctx.handle)


def sampled_check(w, cands, n, cap, mask_dev, seconds, rings=1):
    """CPU baseline on a random sample plus the GPU/oracle comparison there,
    from the sorted candidate list (scale bits) and the mask."""
    import numpy as np
    import torch
    T = len(w.templates)
    dev = cands.device
    m = min(n, cap)
    # list keys (t, y, x) -> t*H*W + y*W + x, sorted because the list is in
    # canonical order; looked up on the device
    c = cands[:m]
    keys = c[:, 0].to(torch.int64) * (w.H * w.W)
    keys += c[:, 1].to(torch.int64) * w.W
    keys += c[:, 2].to(torch.int64)

    def gpu_bits(ys, xs):
        out = np.zeros((T, len(xs)), np.uint32)
        if m == 0:
            return out
        pos = torch.from_numpy(ys.astype(np.int64) * w.W + xs).to(dev)
        for t in range(T):
            k = pos + t * (w.H * w.W)
            i = torch.searchsorted(keys, k).clamp_(max=m - 1)
            hit = keys[i] == k
            v = torch.where(hit, c[i, 3], torch.zeros_like(c[i, 3]))
            out[t] = v.cpu().numpy().view(np.uint32)
        return out

    def gpu_mask(ys, xs):
        import torch
        yt = torch.from_numpy(ys.astype(np.int64)).to(mask_dev.device)
        xt = torch.from_numpy(xs.astype(np.int64)).to(mask_dev.device)
        return mask_dev[:, yt, xt].cpu().numpy()

    return cpu_baseline(w, None, seconds, gpu_bits=gpu_bits, gpu_mask=gpu_mask,
                        list_complete=n <= cap, rings=rings)


SERVE_TOL = (4, 8, 65, 100)
SERVE_CAP = 1 << 22


def _pct(v, q):
    import numpy as np
    return float(np.percentile(np.asarray(v, np.float64), q)) if len(v) else None


def run_serving(args, n_requests=None):
    """Workload 4.  The per-request scheme (tables built for every request,
    one launch per template, one request at a time) is timed back to back to
    find its capacity; the same Poisson stream, at 80% of that rate, is then
    served by (a) that scheme, first come first served, and (b) the server
    (resident tables, merged batched launches, several lanes; requests are
    submitted as they arrive, while earlier launches run).  Latency runs from
    a request's arrival to its result being ready.  Every served result
    (mask and list) is compared element by element with the same request
    screened alone.  Returns the result dict."""
    import numpy as np
    import torch

    from paper_1707_05647_amd import _lib as L
    from paper_1707_05647_amd.screen import Context, Server
    from synth import serving_requests

    n_req = n_requests or args.requests
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    print(f"serving: generating {n_req} requests", file=sys.stderr, flush=True)
    reqs, images = serving_requests(n_req, 1.0, args.seed, device=dev)
    imgs = {k: L.device_image(v, dev) for k, v in images.items()}
    feats = [[L.oss_template_features(t.pixels, t.rho, L.OSS_F_ALL) for t in q.templates]
             for q in reqs]
    ctx = Context(0)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    cands = torch.empty((SERVE_CAP, 4), dtype=torch.int32, device=dev)
    alone = [None] * len(reqs)

    def plain_one(i, keep=False):
        q = reqs[i]
        ref = ctx.reference(imgs[q.ref_key], L.OSS_F_ALL, 8, stream,
                            max_radius=max([p[2] for p in q.probes] + [0]))
        mask = torch.empty((len(q.templates), q.side, q.side), dtype=torch.uint8, device=dev)
        L.oss_screen(ctx.handle, ref.handle, feats[i], q.probes, SERVE_TOL, L.OSS_F_ALL, mask,
                     cands, SERVE_CAP, count, stream)
        torch.cuda.synchronize()
        n = int(count.item())
        if keep:
            alone[i] = (mask, cands[:min(n, SERVE_CAP)].clone(), n)
        ref.release()

    # warm-up and the per-request scheme's capacity (back to back); the
    # results of this pass are kept as each request's screen alone
    plain_one(0)
    t0 = time.perf_counter()
    for i in range(len(reqs)):
        plain_one(i, keep=True)
    plain_busy = time.perf_counter() - t0
    capacity = len(reqs) / plain_busy
    rate = 0.8 * capacity
    arrivals = [q.arrival_s / rate for q in reqs]  # the stream was drawn at rate 1
    print(f"serving: plain capacity {capacity:.1f} req/s, offered {rate:.1f} req/s",
          file=sys.stderr, flush=True)

    # (a) the per-request scheme under the Poisson stream
    lat_plain = []
    start = time.perf_counter()
    for i in range(len(reqs)):
        now = time.perf_counter() - start
        if now < arrivals[i]:
            time.sleep(arrivals[i] - now)
        plain_one(i)
        lat_plain.append((time.perf_counter() - start - arrivals[i]) * 1e3)
    span_plain = time.perf_counter() - start

    # (b) the server under the same stream
    srv = Server(0, 96 << 30, lanes=args.lanes, max_batch_templates=64)
    w = srv.submit(reqs[0].ref_key, imgs[reqs[0].ref_key], feats[0], reqs[0].probes, SERVE_TOL,
                   L.OSS_F_ALL, SERVE_CAP)
    srv.drain()
    srv.release(w)
    ids = [None] * len(reqs)
    base = time.monotonic_ns()
    nxt = 0
    done = 0
    while done < len(reqs):
        now_s = (time.monotonic_ns() - base) * 1e-9
        while nxt < len(reqs) and arrivals[nxt] <= now_s:
            q = reqs[nxt]
            ids[nxt] = srv.submit(q.ref_key, imgs[q.ref_key], feats[nxt], q.probes, SERVE_TOL,
                                  L.OSS_F_ALL, SERVE_CAP,
                                  arrival_ns=base + int(arrivals[nxt] * 1e9))
            nxt += 1
        wait = 200 if nxt == len(reqs) else max(0, min(200, int((arrivals[nxt] - now_s) * 1e6)))
        got = srv.pump(wait)
        done += got
        if nxt == len(reqs) and got == 0:
            stt = srv.stats()
            if stt["queued"] == 0 and stt["running"] == 0:
                raise RuntimeError(f"server idle with {len(reqs) - done} requests unfinished: "
                                   f"{stt}")
    span_srv = (time.monotonic_ns() - base) * 1e-9
    lat_srv, q_srv, batch, hits, same = [], [], [], 0, 0
    for i, rid in enumerate(ids):
        r = srv.result(rid)
        if r.status != L.OSS_OK:
            raise RuntimeError(f"request {i} failed: {L.status_string(r.status)}")
        lat_srv.append(r.latency_ms)
        q_srv.append(r.queue_ms)
        batch.append(r.batch_requests)
        hits += r.resident_hit
        mask_t = torch.empty((r.n_tmpl, r.H, r.W), dtype=torch.uint8, device=dev)
        m = min(r.count, SERVE_CAP)
        lst = torch.empty((m, 4), dtype=torch.int32, device=dev)
        _dev_copy(mask_t, r.dev_mask)
        if m:
            _dev_copy(lst, r.dev_list)
        a_mask, a_list, a_n = alone[i]
        same += int(r.count == a_n and torch.equal(mask_t, a_mask) and torch.equal(lst, a_list))
        srv.release(rid)
    st = srv.stats()
    srv.close()
    ctx.close()
    del alone

    ps = [pixel_scales(q.side, q.side, q.probes) for q in reqs]
    total_ps = float(sum(ps))
    return {
        "metric": METRIC,
        "value": total_ps / span_srv / 1e9,
        "unit": "G pixel-scales/s",
        "n_gpus": 1,
        "steps": len(reqs),
        "warmup": 1,
        "ms_per_step": span_srv * 1e3 / len(reqs),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE,
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[4], "requests": len(reqs),
                   "distinct_references": len(images), "lanes": args.lanes, "seed": args.seed,
                   "tolerance_P_over_Q": [p / SERVE_TOL[3] for p in SERVE_TOL[:3]],
                   "list_cap": SERVE_CAP},
        "served": {
            "p50_ms": _pct(lat_srv, 50), "p99_ms": _pct(lat_srv, 99),
            "queue_p50_ms": _pct(q_srv, 50), "queue_p99_ms": _pct(q_srv, 99),
            "requests_per_s": len(reqs) / span_srv,
            "mean_requests_per_launch": float(np.mean(batch)),
            "resident_hits": hits, "launches": st["launches"], "builds": st["builds"],
            "evictions": st["evictions"], "bytes_peak": st["bytes_peak"],
            "identical_to_alone": same, "of": len(reqs),
            "compared": "mask and candidate list element by element, and the count",
        },
        "per_request_scheme": {
            "capacity_requests_per_s": capacity,
            "p50_ms": _pct(lat_plain, 50), "p99_ms": _pct(lat_plain, 99),
            "requests_per_s": len(reqs) / span_plain,
            "value": total_ps / span_plain / 1e9,
        },
        "offered_requests_per_s": rate,
    }


def _dev_copy(dst, src_ptr: int):
    """Device-to-device copy of dst.nbytes bytes from a raw device pointer."""
    import ctypes as C

    import torch  # noqa: F401
    global _HIP
    if "_HIP" not in globals():
        _HIP = C.CDLL("libamdhip64.so.7")
        _HIP.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        _HIP.hipMemcpy.restype = C.c_int
    rc = _HIP.hipMemcpy(dst.data_ptr(), src_ptr, dst.numel() * dst.element_size(), 3)
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed ({rc})")


def evaluate_regions(w, ctx, L, torch, dev, cands, count, cap):
    """Exp. I's quality columns on the synthetic stand-in: the preserved
    region (union of the candidates' star footprints, oss_region), the pruned
    share of the image, and the overlap of the preserved region with the
    ground truth, the star footprint of the planted object (radius = the
    object's radius in the reference, at the planted centre); a screen
    succeeds for a template when that overlap is at least 90%."""
    T = len(w.templates)
    region = torch.empty((T, w.H, w.W), dtype=torch.uint8, device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    L.oss_region(ctx.handle, w.H, w.W, T, w.probes, cands, cap, count, region)
    e1.record()
    torch.cuda.synchronize()
    gt = torch.empty((T, w.H, w.W), dtype=torch.uint8, device=dev)
    one = torch.zeros((T, 4), dtype=torch.int32, device=dev)
    gt_probes = []
    for t, tp in enumerate(w.templates):
        r = int(round(tp.obj_radius))
        one[t] = torch.tensor([t, tp.cy, tp.cx, 1], dtype=torch.int32)
        gt_probes.append((t, 0, r))
    n1 = torch.tensor([T], dtype=torch.int64, device=dev)
    L.oss_region(ctx.handle, w.H, w.W, T, gt_probes, one, T, n1, gt)
    torch.cuda.synchronize()
    hw = float(w.H * w.W)
    kept = region.flatten(1).sum(1, dtype=torch.int64).cpu().tolist()
    both = (region & gt).flatten(1).sum(1, dtype=torch.int64).cpu().tolist()
    gts = gt.flatten(1).sum(1, dtype=torch.int64).cpu().tolist()
    overlap = [100.0 * b / g for b, g in zip(both, gts)]
    return {
        "pruned_region_pct": 100.0 * (1 - sum(kept) / (T * hw)),
        "overlap_pct_mean": sum(overlap) / T,
        "overlap_pct_min": min(overlap),
        "success_90": sum(o >= 90.0 for o in overlap),
        "templates": T,
        "region_ms": e0.elapsed_time(e1),
        "ground_truth": "star footprint of radius round(object radius) at the planted centre",
    }


def copy_peak(torch, dev, mib=4096, reps=5):
    """Achievable HBM rates: a plain device-to-device copy of `mib` MiB timed
    with events (bytes read + bytes written per second, best of `reps`), and
    a fill of the same buffer (bytes written per second)."""
    src = torch.ones(mib << 20, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    # write-only: a fill of the same buffer (the rate a store-bound kernel,
    # such as the table builder's final pass, can reach)
    fbest = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.fill_(7)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        fbest = ms if fbest is None else min(fbest, ms)
    del src, dst
    torch.cuda.empty_cache()
    return {"GBps": 2.0 * (mib << 20) / (best / 1e3) / 1e9, "bytes_per_copy": 2 * (mib << 20),
            "ms": best, "kernel": "torch device copy (read + write)",
            "fill_GBps": (mib << 20) / (fbest / 1e3) / 1e9, "fill_ms": fbest}


def run_fixed(args, workload, *, steps, warmup, cpu_seconds, evaluate, cpu_baseline=True,
              compare_plain=True):
    """Workloads 2, 3 and 5: the timed steps on one lane, then on `lanes`
    lanes (the faster of the two runs is the headline figure, both are
    reported), the batched-over-plain comparison for the batched workloads,
    the roofline figures and the sampled CPU oracle.  Returns the result
    dict."""
    import torch

    from paper_1707_05647_amd import _lib as L
    from paper_1707_05647_amd.screen import Context
    from synth import make_workload

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    big = workload in (3, 5)
    print(f"workload {workload}: generating inputs", file=sys.stderr, flush=True)
    cache = (os.path.join(args.ref_cache, f"reference_w{workload}_s{args.seed}.npy")
             if args.ref_cache and big else None)
    w = make_workload(workload, args.seed, device=dev if big else None, ref_cache=cache)
    img = L.device_image(w.ref, dev)
    ctx = Context(0)
    if args.star_strip:
        L.oss_ctx_set_option(ctx.handle, L.OSS_OPT_STAR_STRIP, args.star_strip)
    if args.star_blocks:
        L.oss_ctx_set_option(ctx.handle, L.OSS_OPT_STAR_BLOCKS_PER_XCD, args.star_blocks)
    if args.star_lds >= 0:
        L.oss_ctx_set_option(ctx.handle, L.OSS_OPT_STAR_LDS, args.star_lds)
    planar = args.planar
    if planar < 0 and workload == 3:
        # loose tolerances (45-80 %): most positions pass the first feature,
        # so staged lookups on planar tables save nothing and one lookup of
        # an interleaved entry beats several plane reads
        planar = 0
    if planar >= 0:
        L.oss_ctx_set_option(ctx.handle, L.OSS_OPT_TABLE_PLANAR, planar)
    if args.table_rec >= 0:
        L.oss_ctx_set_option(ctx.handle, L.OSS_OPT_TABLE_REC, args.table_rec)
    if args.pipe >= 0:
        L.oss_ctx_set_option(ctx.handle, L.OSS_OPT_STAR_PIPE, args.pipe)
    if args.staged >= 0:
        L.oss_ctx_set_option(ctx.handle, L.OSS_OPT_STAR_STAGED, args.staged)
    if args.build_stream >= 0:
        L.oss_ctx_set_option(ctx.handle, L.OSS_OPT_BUILD_STREAM, args.build_stream)
    lanes = args.pipeline if args.pipeline >= 1 else 2
    lane_stream = L.oss_ctx_get_option(ctx.handle, L.OSS_OPT_BUILD_STREAM)
    if args.build_stream < 0:
        # streaming table stores pay off only beside another lane's star
        # pass: the one-lane runs use ordinary stores
        L.oss_ctx_set_option(ctx.handle, L.OSS_OPT_BUILD_STREAM, 0)
    max_r = max(w.radii())
    if args.alg1:
        from fractions import Fraction
        max_r = max(p.r for t, tp in enumerate(w.templates)
                    for p in L.oss_alg1_probes(tp.pixels, t, Fraction(1, 2), Fraction(2),
                                               (1, 1, 1), w.feat_mask, bit_depth=w.depth))
    ref_fm = (L.OSS_F_SUM | L.OSS_F_SQ | L.OSS_F_MOMENTS) if args.moments else w.feat_mask
    ref = ctx.reference(img, ref_fm, w.depth, build=False, max_radius=max_r)
    T = len(w.templates)
    mask = torch.empty((T, w.H, w.W), dtype=torch.uint8, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    tol = (*w.tol_P, w.tol_Q)

    def tfeat():
        return [L.oss_template_features(t.pixels, t.rho, w.feat_mask, bit_depth=w.depth)
                for t in w.templates]

    def tfeat_rings():
        return [L.oss_template_features_rings(t.pixels, t.rho, w.feat_mask, args.rings,
                                              bit_depth=w.depth) for t in w.templates]

    ALG1_Q = (4, 300, 6) if w.depth == 8 else (64, 80000, 90)

    def alg1_probes():
        from fractions import Fraction
        out = []
        for t, tp in enumerate(w.templates):
            out += L.oss_alg1_probes(tp.pixels, t, Fraction(1, 2), Fraction(2), ALG1_Q,
                                     w.feat_mask, bit_depth=w.depth)
        return out

    MOM_TOL = (5, 30, 40, 100)
    state = {"cap": 0}

    def screen_step(ch, r, st, m, cd, cn, batched, gate=None):
        """One step of the chosen variant on context ch, reference r, stream
        st, into mask m, list cd and count cn; with a gate, the screen (not
        the build) waits for the previous lane's screen."""
        cap = state["cap"]
        r.build(st)
        if gate is not None:
            gate.wait(st)
        if args.alg1:
            L.oss_screen_intervals(ch, r.handle, T, alg1_probes(), w.feat_mask, m, cd, cap, cn,
                                   st)
        elif args.moments:
            tm = [L.oss_template_moments(t.pixels, t.rho, bit_depth=w.depth) for t in w.templates]
            L.oss_screen_moments(ch, r.handle, tm, w.probes, MOM_TOL, 7, m, cd, cap, cn, st)
        elif args.rings > 1:
            L.oss_screen_rings(ch, r.handle, tfeat_rings(), w.probes, tol, w.feat_mask, m, cd,
                               cap, cn, st)
        else:
            L.oss_screen(ch, r.handle, tfeat(), w.probes, tol, w.feat_mask, m, cd, cap, cn, st,
                         batched=batched)
        if gate is not None:
            gate.record(st)

    batched_path = big or args.rings > 1
    # list capacity: the count of a first screen (no list), so the list holds
    # every candidate and the sampled check sees a complete list
    screen_step(ctx.handle, ref, stream, mask, None, count, batched_path)
    torch.cuda.synchronize()
    n_probe = int(count.item())
    cap = max(1, n_probe)
    state["cap"] = cap
    cands = torch.empty((cap, 4), dtype=torch.int32, device=dev)

    def make_step(batched):
        return lambda: screen_step(ctx.handle, ref, stream, mask, cands, count, batched)

    extra = {}
    if big:
        if not args.no_autotune:
            tr = L.oss_autotune_batched(ctx.handle, ref.handle, tfeat(), w.probes, tol,
                                        w.feat_mask, stream)
            extra["autotune"] = {
                "strip": tr.strip, "blocks_per_xcd": tr.blocks_per_xcd,
                "bucket_radii": tr.bucket_radii, "ms": tr.ms,
                "tried": [[tr.tried[i][0], tr.tried[i][1], tr.tried[i][2], tr.tried_ms[i]]
                          for i in range(tr.n_tried)]}
        if compare_plain:
            # the per-template launches at their own best shape (strip 512,
            # 32 / 64 / 128 blocks per XCD), then the batched shape again
            print(f"workload {workload}: per-template launches", file=sys.stderr, flush=True)
            tuned = [L.oss_ctx_get_option(ctx.handle, o)
                     for o in (L.OSS_OPT_STAR_STRIP, L.OSS_OPT_STAR_BLOCKS_PER_XCD)]
            best = None
            for blocks in (32, 64, 128):
                L.oss_ctx_set_option(ctx.handle, L.OSS_OPT_STAR_STRIP, 512)
                L.oss_ctx_set_option(ctx.handle, L.OSS_OPT_STAR_BLOCKS_PER_XCD, blocks)
                plain_s, plain_prof = run_steps(make_step(False), max(1, steps // 4), 1, ctx,
                                                L, torch)
                if best is None or plain_s < best[0]:
                    best = (plain_s, plain_prof, blocks)
            for o, v in zip((L.OSS_OPT_STAR_STRIP, L.OSS_OPT_STAR_BLOCKS_PER_XCD), tuned):
                L.oss_ctx_set_option(ctx.handle, o, v)
            plain_s, plain_prof, blocks = best
            extra["plain_ms_per_step"] = plain_s * 1e3
            extra["plain_shape"] = {"strip": 512, "blocks_per_xcd": blocks}
            extra["plain_kernels"] = {k: v[1] / max(v[0], 1) for k, v in plain_prof.items()}
    lanes = args.pipeline if args.pipeline >= 1 else 2
    if args.lanes_only and lanes >= 2:
        # one untimed step fills this context's outputs, which the lanes'
        # results are compared with
        make_step(batched_path)()
        torch.cuda.synchronize()
        sec, prof = None, {}
    else:
        print(f"workload {workload}: timed steps, one lane", file=sys.stderr, flush=True)
        sec, prof = run_steps(make_step(batched_path), steps, warmup, ctx, L, torch)

    if args.alg1:
        # one pixel-scale per (valid position, template, band)
        bands = {(p.template_id, p.scale_id, p.r) for p in alg1_probes()}
        ps = sum(max(0, w.H - 2 * r) * max(0, w.W - 2 * r) for _, _, r in bands)
    else:
        ps = pixel_scales(w.H, w.W, w.probes)
    value = ps / sec / 1e9 if sec else None
    n = int(count.item())
    if n != n_probe:
        raise RuntimeError(f"candidate count changed between runs ({n_probe} -> {n})")
    if big and compare_plain and sec:
        # batched against per-template launches, one lane each
        extra["plain_value"] = ps / (extra["plain_ms_per_step"] / 1e3) / 1e9
        extra["batched_over_plain"] = extra["plain_ms_per_step"] / (sec * 1e3)
    def run_summary(s, pr, build_stream):
        return {"value": ps / s / 1e9, "ms_per_step": s * 1e3, "build_stream": build_stream,
                "kernels": {k: {"launches": v[0], "avg_ms": v[1] / max(v[0], 1)}
                            for k, v in pr.items()}}

    timed_lanes = lanes
    if lanes >= 2 and sec:
        extra["single_lane"] = run_summary(
            sec, prof, L.oss_ctx_get_option(ctx.handle, L.OSS_OPT_BUILD_STREAM))
    if lanes >= 2:
        L.oss_ctx_set_option(ctx.handle, L.OSS_OPT_BUILD_STREAM, lane_stream)
        print(f"workload {workload}: timed steps, {lanes} lanes", file=sys.stderr, flush=True)
        sub = argparse.Namespace(**vars(args))
        sub.steps, sub.warmup = steps, warmup
        sec_l, prof_l, same = pipelined(sub, lanes, w, L, torch, dev, ctx, img, ref_fm, max_r,
                                        cap, batched_path, screen_step, n, mask, cands)
        extra["lanes_identical_to_single_lane"] = same
        extra["lanes_run"] = dict(run_summary(sec_l, prof_l, lane_stream), lanes=lanes)
        if sec is None or sec_l < sec:
            # the lanes' run is the headline (the single lane's figures are kept)
            sec, prof = sec_l, prof_l
        else:
            # a star pass that fills the GPU alone gains nothing from a second
            # lane beside it: the faster one-lane run is the headline
            timed_lanes = 1
        value = ps / sec / 1e9
    eb = sum(b // 8 for _, b in ref.slots)  # table bytes per position, all quantities
    staged = (ref.plane_bytes > 0 and len(ref.slots) > 1 and not args.moments
              and L.oss_ctx_get_option(ctx.handle, L.OSS_OPT_STAR_STAGED) == 1
              and L.oss_ctx_get_option(ctx.handle, L.OSS_OPT_STAR_PIPE) == 0)
    # table bytes per entry as stored, over all planes
    ebs = ref.stored_entry_bytes
    abytes = algorithmic_bytes(w.H, w.W, T, 2 if w.depth > 8 else 1, ebs, n_cand=n)
    kern = {k: {"launches": v[0], "avg_ms": v[1] / max(v[0], 1), "max_ms": v[2]}
            for k, v in prof.items()}
    dom = max(prof, key=lambda k: prof[k][1])
    avg_s = prof[dom][1] / prof[dom][0] / 1e3
    achieved = abytes[dom] / avg_s / 1e9 if dom in abytes else None
    roof = {
        "kernel": dom,
        "bound": "hbm",
        "achieved": achieved,
        "peak": HBM_PEAK_GBPS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBPS if achieved else None,
        "traffic": traffic_for(dom, workload),
        "algorithmic_bytes_per_launch": abytes.get(dom),
        "algorithmic_unit": "tables read once (entry bytes x 3 tables x (H+1)(W+1)) + uint8 "
                            "mask (templates x H x W)",
        "avg_ms": avg_s * 1e3,
        "timed_on": f"{timed_lanes} lanes" if timed_lanes >= 2 else "one lane",
    }
    if timed_lanes >= 2 and "single_lane" in extra and dom in extra["single_lane"]["kernels"]:
        one = extra["single_lane"]["kernels"][dom]["avg_ms"] / 1e3
        roof["one_lane"] = {"avg_ms": one * 1e3, "achieved": abytes[dom] / one / 1e9,
                            "frac": abytes[dom] / one / 1e9 / HBM_PEAK_GBPS}
    if dom in ("star_plain", "star_batch"):
        # the same launch against the vector-memory path that actually bounds it
        # staged lookups read the first quantity everywhere and the others
        # only where it passes: only the first quantity's bytes are counted
        per = ref.entry_bytes if staged else eb
        lookups = lookup_pairs(w, dom == "star_batch", rings=args.rings) * 8 * per
        roof["vector_l1"] = {"achieved": lookups / avg_s / 1e9, "peak": L1_PEAK_GBPS,
                             "unit": "GB/s", "frac": lookups / avg_s / 1e9 / L1_PEAK_GBPS,
                             "lookup_bytes_per_launch": lookups,
                             "counted": ("first quantity only (staged lookups)" if staged
                                         else "every quantity")}
    for k in kern:
        if k in abytes and abytes[k]:
            kern[k]["achieved_GBps"] = abytes[k] / (kern[k]["avg_ms"] / 1e3) / 1e9
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "G pixel-scales/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE,
        "data": "synthetic",
        "config": {
            "workload": WORKLOAD_TEXT[workload],
            "H": w.H, "W": w.W, "radii": w.radii(), "templates": T, "probes": len(w.probes),
            "tolerance_P_over_Q": [p / w.tol_Q for p in w.tol_P], "seed": args.seed,
            "pixel_scales_per_step": ps,
            "table_value_bits": ref.value_bits,
            "table_entry_bytes": ebs,
            "table_layout": "planar" if ref.plane_bytes else "interleaved",
            "star_strip": L.oss_ctx_get_option(ctx.handle, L.OSS_OPT_STAR_STRIP),
            "star_blocks_per_xcd": L.oss_ctx_get_option(ctx.handle,
                                                        L.OSS_OPT_STAR_BLOCKS_PER_XCD),
            "star_lds": L.oss_ctx_get_option(ctx.handle, L.OSS_OPT_STAR_LDS),
            "table_planar": L.oss_ctx_get_option(ctx.handle, L.OSS_OPT_TABLE_PLANAR),
            "table_rec": L.oss_ctx_get_option(ctx.handle, L.OSS_OPT_TABLE_REC),
            "table_slot_bits": [b for _, b in ref.slots],
            "star_pipe": L.oss_ctx_get_option(ctx.handle, L.OSS_OPT_STAR_PIPE),
            "star_staged": L.oss_ctx_get_option(ctx.handle, L.OSS_OPT_STAR_STAGED),
            "build_stream": (extra["single_lane"]["build_stream"] if timed_lanes < lanes
                             else L.oss_ctx_get_option(ctx.handle, L.OSS_OPT_BUILD_STREAM)),
            "batch_bucket": L.oss_ctx_get_option(ctx.handle, L.OSS_OPT_BATCH_BUCKET),
            "launch": "batched" if batched_path else "plain",
            "lanes": timed_lanes,
            "lanes_tried": lanes,
            "serial_screens": bool(args.serial_screens),
            "rings": args.rings,
            "alg1": bool(args.alg1),
            "moments": bool(args.moments),
            "list_cap": cap,
        },
        "roofline": roof,
        "kernels": kern,
        "candidates": n,
        "pruned_patch_pct": 100.0 * (1 - n / float(T * w.H * w.W)),
    }
    out.update(extra)
    if evaluate:
        out["evaluation"] = evaluate_regions(w, ctx, L, torch, dev, cands, count, cap)
    if cpu_baseline and not args.no_cpu_baseline and not args.alg1 and not args.moments:
        print(f"workload {workload}: CPU oracle on a sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = sampled_check(w, cands, n, cap, mask, cpu_seconds, args.rings)
    ref.release()
    ctx.close()
    del mask, cands, count, img
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def nested(res, keys):
    return {k: res[k] for k in keys if k in res}


def parse_args(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--workload", type=int, default=0, choices=[0, 2, 3, 4, 5],
                    help="0 (default): the headline line, workload 5 with workload 2 and the "
                         "serving loop nested; 2: the rotation+scale screen alone; 3, 5: batched "
                         "workloads alone (batched launch against per-template launches); "
                         "4: serving loop alone")
    ap.add_argument("--evaluate", type=int, default=-1,
                    help="1: preserved region, overlap with the planted ground truth and the 90%% "
                         "success criterion after the timed steps (default: on for workload 2)")
    ap.add_argument("--moments", type=int, default=0,
                    help="1: screen with the paper's own features (mean, variance, first-moment "
                         "gradient magnitude) instead of sum / squares / gradient sum")
    ap.add_argument("--alg1", type=int, default=0,
                    help="1: screen with Algorithm 1 taken literally (sqrt 2 scale bands over "
                         "[1/2, 2], quantised membership) instead of the probe radii")
    ap.add_argument("--rings", type=int, default=1,
                    help="central-star rings per probe (multi-central-area screen); 1 = off")
    ap.add_argument("--requests", type=int, default=100, help="workload 4: requests")
    ap.add_argument("--lanes", type=int, default=2, help="workload 4: server lanes")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-plain", action="store_true",
                    help="batched workloads: skip the per-template comparison")
    ap.add_argument("--lanes-only", action="store_true",
                    help="time only the multi-lane run (no one-lane steps; for traces whose "
                         "launches should all be the timed configuration's)")
    ap.add_argument("--star-strip", type=int, default=0,
                    help="star kernel strip width (threads per block); 0 = library default")
    ap.add_argument("--star-blocks", type=int, default=0,
                    help="star kernel persistent blocks per XCD; 0 = library default")
    ap.add_argument("--pipe", type=int, default=-1,
                    help="1/0: software-pipelined / one-radius-at-a-time star pass; -1 = default")
    ap.add_argument("--pipeline", type=int, default=-1,
                    help="time the steps round-robin over this many lanes (a context, stream, "
                         "tables and outputs each: consecutive batches overlap); 1 = one lane; "
                         "-1 = 2")
    ap.add_argument("--staged", type=int, default=-1,
                    help="1/0: staged lookups (first quantity alone, the rest where it passes) / "
                         "every quantity at every lookup; -1 = library default")
    ap.add_argument("--serial-screens", type=int, default=0,
                    help="1: on two or more lanes a lane's screen waits for the previous "
                         "lane's screen (builds still overlap screens)")
    ap.add_argument("--build-stream", type=int, default=-1,
                    help="1/0: table entries stored with / without non-temporal (streaming) "
                         "stores; -1 = library default for the lanes, ordinary stores for the "
                         "one-lane runs")
    ap.add_argument("--planar", type=int, default=-1,
                    help="1/0: planar / interleaved tables; -1 = library default "
                         "(interleaved for workload 3, whose tolerances are loose)")
    ap.add_argument("--table-rec", type=int, default=-1,
                    help="1/0: record tables (squares' low words and gradients in 8-byte "
                         "records, the squares' bits 32..39 in a byte plane) where they apply, "
                         "or four 32-bit planes; -1 = library default (record)")
    ap.add_argument("--star-lds", type=int, default=-1,
                    help="1/0: star kernel with / without LDS staging; -1 = library default")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="run one plain device-to-device copy of this many MiB first "
                         "(a reference kernel of known size for HBM byte counters)")
    ap.add_argument("--ref-cache", default="",
                    help="directory for the rendered reference of the batched workloads (loaded "
                         "when present, written otherwise): a profiled run can skip rendering")
    ap.add_argument("--gen-only", action="store_true",
                    help="render (and cache) the workload's inputs, then exit")
    ap.add_argument("--copy-peak-mb", type=int, default=4096,
                    help="size of the timed device copy that gives the achievable HBM rate "
                         "(0: skip)")
    return ap.parse_args(argv)


def main(argv=None):
    args = parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the screen shards "
              "by row bands with no exchange on the hot path, but multi-GPU runs are not "
              "implemented.", file=sys.stderr)
        sys.exit(2)
    import torch
    dev = torch.device("cuda", 0)
    if args.copy_probe_mb:
        src = torch.ones(args.copy_probe_mb << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload == 4:
        print(json.dumps(run_serving(args)), flush=True)
        return
    if args.gen_only:
        from synth import make_workload
        for wl in ((args.workload,) if args.workload in (2, 3, 5) else (5,)):
            cache = (os.path.join(args.ref_cache, f"reference_w{wl}_s{args.seed}.npy")
                     if args.ref_cache and wl in (3, 5) else None)
            make_workload(wl, args.seed, device=dev if wl in (3, 5) else None, ref_cache=cache)
        return
    if args.workload in (2, 3, 5):
        out = run_fixed(args, args.workload, steps=args.steps, warmup=args.warmup,
                        cpu_seconds=args.cpu_seconds,
                        evaluate=args.evaluate == 1 or (args.evaluate < 0 and args.workload == 2),
                        compare_plain=not args.no_plain)
    else:
        # the headline: workload 5 (the largest single-GPU configuration),
        # then workload 2 and the serving loop, nested in the same line
        out = run_fixed(args, 5, steps=args.steps, warmup=args.warmup,
                        cpu_seconds=args.cpu_seconds, evaluate=args.evaluate == 1,
                        compare_plain=not args.no_plain)
        w2 = run_fixed(args, 2, steps=max(args.steps, 20), warmup=args.warmup,
                       cpu_seconds=min(args.cpu_seconds, 5.0), evaluate=args.evaluate != 0)
        out["workload_2"] = nested(w2, ("value", "unit", "ms_per_step", "config", "roofline",
                                        "kernels", "single_lane", "lanes_run", "candidates",
                                        "pruned_patch_pct", "evaluation", "cpu_baseline",
                                        "lanes_identical_to_single_lane"))
        print("serving loop", file=sys.stderr, flush=True)
        sv = run_serving(args)
        out["serving"] = nested(sv, ("value", "unit", "ms_per_step", "config", "served",
                                     "per_request_scheme", "offered_requests_per_s"))
    if args.copy_peak_mb:
        cp = copy_peak(torch, dev, args.copy_peak_mb)
        out["copy_peak_GBps"] = cp["GBps"]
        out["roofline"]["achievable_peak"] = cp
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
