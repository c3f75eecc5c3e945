"""GPU parity: the HIP tables and the screen, bit for bit against the numpy
definitions and the CPU oracle, through the C ABI."""
import numpy as np
import pytest

import oracle.core as oc
from gpu_util import Runner, bits_from_list, say, tables_numpy
from synth import blob_image, cut_patch, make_rng, make_workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def runner():
    r = Runner()
    yield r
    r.close()


TABLE_CASES = [
    # (H, W, depth, feature mask, pitch padding, max radius)
    (37, 53, 8, 7, 0, -1),
    (37, 53, 8, 7, 0, 1 << 20),     # forced 64-bit storage
    (1, 1, 8, 7, 0, -1),
    (5, 700, 8, 3, 0, -1),          # two final-pass tiles across
    (129, 100, 12, 7, 0, -1),       # a partial last band
    (129, 100, 12, 7, 0, 8),        # 32-bit storage, 12-bit squares
    (33, 1000, 8, 5, 13, -1),       # three tiles across, pitch > width
    (33, 1000, 8, 5, 13, 1 << 20),
    (70, 450, 8, 4, 0, -1),
    (64, 64, 16, 2, 0, -1),         # full 16-bit squares (64-bit storage)
    (91, 931, 16, 1, 0, 3),         # 16-bit sums, 32-bit storage
    (129, 100, 12, 7, 0, 40),       # mixed entries: 64-bit squares, 32-bit sums and gradients
    (61, 530, 8, 3, 7, 200),        # mixed entries, sums and squares
    (45, 300, 12, 6, 0, 60),        # mixed entries, squares and gradients
    (70, 90, 8, 27, 0, -1),         # first moments i I, j I, 32-bit
    (61, 97, 12, 25, 3, 1 << 20),   # first moments, 64-bit
    (45, 300, 12, 27, 0, 60),       # first moments with 12-bit squares, 64-bit
]


@pytest.mark.parametrize("stream", [1, 0], ids=["streamed", "ordinary"])
@pytest.mark.parametrize("planar", [0, 1], ids=["interleaved", "planar"])
@pytest.mark.parametrize("case", TABLE_CASES, ids=lambda c: "x".join(map(str, c)))
def test_tables_match_definitions(runner, case, planar, stream):
    """Every table entry equals its definition, for every storage width and
    layout, with the entries written by streaming (non-temporal, the
    default) and by ordinary stores."""
    H, W, depth, fm, pad, max_r = case
    rng = np.random.default_rng(H * 1000 + W)
    dt = np.uint8 if depth == 8 else np.uint16
    img = rng.integers(0, 2 ** depth, (H, W)).astype(dt)
    torch = runner.torch
    say(f"tables {case} planar={planar} stream={stream}")
    if pad:
        wide = np.zeros((H, W + pad), dt)
        wide[:, :W] = img
        t_img = runner.L.device_image(wide, runner.dev)[:, :W]
    else:
        t_img = runner.L.device_image(img, runner.dev)
    L = runner.L
    h = runner.ctx.handle
    assert L.oss_ctx_get_option(h, L.OSS_OPT_BUILD_STREAM) == 1
    L.oss_ctx_set_option(h, L.OSS_OPT_TABLE_PLANAR, planar)
    L.oss_ctx_set_option(h, L.OSS_OPT_BUILD_STREAM, stream)
    try:
        ref = runner.ctx.reference(t_img, fm, depth, max_radius=max_r)
    finally:
        L.oss_ctx_set_option(h, L.OSS_OPT_TABLE_PLANAR, 1)
        L.oss_ctx_set_option(h, L.OSS_OPT_BUILD_STREAM, 1)
    torch.cuda.synchronize()
    assert len(ref.slots) == bin(fm).count("1")
    if planar:
        assert ref.plane_bytes > 0
        widths = {b for _, b in ref.slots}
        # 32-bit planes, also when the squares alone take two of them
        assert ref.entry_bytes == (8 if widths == {64} else 4)
    else:
        assert ref.plane_bytes == 0
    got = ref.tables_host()
    slots = ref.slots
    ref.release()
    want = tables_numpy(img, fm)
    for w_ in want:
        for q, (_, b) in enumerate(slots):
            if b < 64:
                w_[..., q] %= 1 << b
    bad = []
    for name, g, w in zip(("L", "R", "R'"), got, want):
        diff = np.argwhere(g.astype(np.int64) != w)
        if len(diff):
            bad.append(f"{name}: {len(diff)} wrong entries of {g.size}, first (row, col, q) "
                       f"{diff[:6].tolist()} (table row = y+1, col = x+1)")
    assert not bad, f"tables with slots {slots}: " + "; ".join(bad)


@pytest.mark.parametrize("rec", [1, 0], ids=["record", "split"])
@pytest.mark.parametrize("case", [(129, 100, 12, 40), (61, 530, 8, 200), (20, 400, 12, 180),
                                  (20, 400, 12, 181)], ids=lambda c: "x".join(map(str, c)))
def test_record_tables(runner, case, rec):
    """Planar sum/squares/gradient tables with 64-bit squares: the record
    layout (squares' low words and the gradient in 8-byte records, the
    squares' bits 32..39 in a byte plane) wherever every square and diamond
    sum of the squares stays below 2^40 (12-bit pixels up to radius 180,
    not 181), else four 32-bit planes; either way every entry equals its
    definition (modulo 2^40 for recorded squares)."""
    H, W, depth, max_r = case
    L = runner.L
    h = runner.ctx.handle
    rng = np.random.default_rng(H + 7 * W)
    dt = np.uint8 if depth == 8 else np.uint16
    img = rng.integers(0, 2 ** depth, (H, W)).astype(dt)
    say(f"record tables {case} rec={rec}")
    assert L.oss_ctx_get_option(h, L.OSS_OPT_TABLE_REC) == 1
    L.oss_ctx_set_option(h, L.OSS_OPT_TABLE_REC, rec)
    try:
        ref = runner.ctx.reference(L.device_image(img, runner.dev), 7, depth, max_radius=max_r)
    finally:
        L.oss_ctx_set_option(h, L.OSS_OPT_TABLE_REC, 1)
    runner.torch.cuda.synchronize()
    sq40 = (2 ** depth - 1) ** 2 * max(2 * max_r * max_r + 2 * max_r + 1,
                                        (2 * oc.square_half(max_r) + 1) ** 2) < 2 ** 40
    widths = [b for _, b in ref.slots]
    if rec and sq40:
        assert widths == [32, 40, 32] and ref.stored_entry_bytes == 13
        with pytest.raises(L.OssError):
            L.oss_ref_layout(ref.handle)  # one stride for all slots cannot describe it
    else:
        assert widths == [32, 64, 32] and ref.stored_entry_bytes == 16
    got = ref.tables_host()
    ref.release()
    want = tables_numpy(img, 7)
    for g, w_ in zip(got, want):
        for q, b in enumerate(widths):
            if b < 64:
                w_[..., q] %= 1 << b
        assert np.array_equal(g, w_)


# max radius -> storage: the probes' own maximum (32-bit entries unless the
# sums need more), 200 (64-bit squares beside 32-bit sums and gradients for 8- and
# 12-bit pixels), 2^20 (64-bit entries)
WIDTHS = pytest.mark.parametrize("max_r", [-2, 200, 1 << 20], ids=["w32", "wmix", "w64"])


def _screen_and_compare(runner, w, max_r=-1, **kw):
    if max_r == -2:  # the largest probe radius: the narrowest exact storage
        max_r = max(p[2] for p in w.probes)
    tm = [(t.pixels, t.rho) for t in w.templates]
    P, Q = w.tol_P, w.tol_Q
    say(f"screen workload {w.cfg_id} {w.H}x{w.W} T={len(tm)} probes={len(w.probes)} {kw}")
    mask, cands, n = runner.screen(w.ref, tm, w.probes, w.feat_mask, P, Q,
                                   bit_depth=w.depth, max_radius=max_r, **kw)
    say(f"  storage {runner.last_value_bits}-bit, {runner.last_entry_bytes} B entries, "
        f"{n} candidates")
    want = oc.screen_full(w.ref, tm, w.probes, w.feat_mask, P, Q)
    wmask, wlist = oc.mask_and_list(want)
    assert n == len(wlist)
    assert np.array_equal(mask, wmask)
    assert np.array_equal(cands, wlist)
    return want


@WIDTHS
def test_cfg1_full(runner, max_r):
    w = make_workload(1, 0)
    want = _screen_and_compare(runner, w, max_r)
    t = w.templates[0]
    assert want[0, t.cy, t.cx] == 1  # exact cut: always survives


@WIDTHS
def test_cfg2_small_full(runner, max_r):
    w = make_workload(2, 0, H=256, blobs_per_512sq=800, sig_hi=24)
    _screen_and_compare(runner, w, max_r)


@WIDTHS
def test_cfg2_ragged_pitch(runner, max_r):
    w = make_workload(2, 1, H=211, W=333, blobs_per_512sq=800, sig_hi=24)
    _screen_and_compare(runner, w, max_r, pitch_pad=7)


@WIDTHS
def test_cfg3_small_full(runner, max_r):
    w = make_workload(3, 0, H=200, W=260, n_templates=5, blobs_per_512sq=1200, sig_hi=20)
    _screen_and_compare(runner, w, max_r)


@WIDTHS
def test_cfg5_small_full(runner, max_r):
    w = make_workload(5, 0, H=224, W=240, n_templates=3, blobs_per_512sq=1200, sig_hi=20)
    _screen_and_compare(runner, w, max_r)


def test_single_valid_position_and_empty(runner):
    rng = make_rng(7, 0)
    img = blob_image(21, 21, rng, blobs_per_512sq=4000, sig_hi=6)
    tm = [(cut_patch(img, 10, 10, 10), 9)]
    probes = [(0, 0, 10), (0, 1, 11), (0, 2, 3)]
    mask, cands, n = runner.screen(img, tm, probes, 7, (100, 100, 100), 100, max_radius=16)
    want = oc.screen_full(img, tm, probes, 7, (100, 100, 100), 100)
    assert np.array_equal(cands, oc.mask_and_list(want)[1])
    assert not (want & 2).any()
    # no valid position at all
    mask, cands, n = runner.screen(img, tm, [(0, 0, 11)], 7, (100, 100, 100), 100,
                                   max_radius=16)
    assert n == 0 and not mask.any()
    # a probe beyond the reference's declared maximum radius is an argument error
    with pytest.raises(runner.L.OssError):
        runner.screen(img, tm, [(0, 0, 11)], 7, (100, 100, 100), 100)


def test_list_truncation(runner):
    w = make_workload(2, 2, H=128, blobs_per_512sq=800, sig_hi=24)
    tm = [(t.pixels, t.rho) for t in w.templates]
    P = (100, 100, 100)
    mask, cands, n = runner.screen(w.ref, tm, w.probes, w.feat_mask, P, 100)
    assert n > 100
    m2, c2, n2 = runner.screen(w.ref, tm, w.probes, w.feat_mask, P, 100, list_cap=100)
    assert n2 == n and np.array_equal(c2, cands[:100]) and np.array_equal(m2, mask)


@pytest.mark.parametrize("max_r", [64, 1 << 20], ids=["rmax64", "w64"])
@pytest.mark.parametrize("depth", [8, 12, 16])
def test_overflow_edge_constant_max(runner, depth, max_r):
    """All pixels at the maximum value, largest radius: exact sums c*A(r),
    c^2*A(r), 0 pass at P = 0 everywhere the star fits."""
    H = W = 129
    c = 2 ** depth - 1
    img = np.full((H, W), c, np.uint8 if depth == 8 else np.uint16)
    tm = [(np.full((131, 131), c, img.dtype), 64)]
    probes = [(0, 0, 64), (0, 1, 63)]
    mask, cands, n = runner.screen(img, tm, probes, 7, (0, 0, 0), 1, bit_depth=depth,
                                   max_radius=max_r)
    want = oc.screen_full(img, tm, probes, 7, (0, 0, 0), 1)
    assert np.array_equal(cands, oc.mask_and_list(want)[1])
    assert want[0, 64, 64] == 3 and n == 9


def test_32bit_storage_near_its_limit(runner):
    """12-bit pixels, radius 10: square sums of squares reach 3.77e9 < 2^32,
    so the reference is stored in 32-bit words; at radius 11 the squares
    need more than 32 bits while sums and gradients still fit: 64-bit
    accumulation, the squares stored in 40 bits (record tables, the planar
    default: their sums stay below 2^40)."""
    rng = np.random.default_rng(4)
    img = rng.integers(3900, 4096, (64, 80)).astype(np.uint16)
    img[20:40, 30:50] = 4095
    tm = [(np.ascontiguousarray(img[20:43, 28:51]), 10)]
    probes = [(0, 0, 10), (0, 1, 7)]
    P, Q = (2, 3, 100), 1000
    mask, cands, n = runner.screen(img, tm, probes, 7, P, Q, bit_depth=12, max_radius=10)
    assert runner.last_value_bits == 32
    want = oc.screen_full(img, tm, probes, 7, P, Q)
    assert np.array_equal(cands, oc.mask_and_list(want)[1]) and n > 0
    mask, cands, n = runner.screen(img, tm, probes, 7, P, Q, bit_depth=12, max_radius=11)
    assert runner.last_value_bits == 64  # 64-bit squares only
    assert [b for _, b in runner.last_slots] == [32, 40, 32]
    assert np.array_equal(cands, oc.mask_and_list(want)[1])


@pytest.mark.parametrize("strip,blocks,lds", [(64, 1, 1), (512, 3, 1), (128, 500, 1),
                                               (256, 64, 0), (64, 7, 0)])
def test_launch_shapes_do_not_change_results(runner, strip, blocks, lds):
    w = make_workload(2, 3, H=300, W=700, blobs_per_512sq=800, sig_hi=24)
    tm = [(t.pixels, t.rho) for t in w.templates]
    base = runner.screen(w.ref, tm, w.probes, w.feat_mask, w.tol_P, w.tol_Q)
    L = runner.L
    opts = (L.OSS_OPT_STAR_STRIP, L.OSS_OPT_STAR_BLOCKS_PER_XCD, L.OSS_OPT_STAR_LDS)
    old = [L.oss_ctx_get_option(runner.ctx.handle, o) for o in opts]
    for o, v in zip(opts, (strip, blocks, lds)):
        L.oss_ctx_set_option(runner.ctx.handle, o, v)
    try:
        got = runner.screen(w.ref, tm, w.probes, w.feat_mask, w.tol_P, w.tol_Q)
    finally:
        for o, v in zip(opts, old):
            L.oss_ctx_set_option(runner.ctx.handle, o, v)
    assert got[2] == base[2] and np.array_equal(got[1], base[1])
    with pytest.raises(L.OssError):
        L.oss_ctx_set_option(runner.ctx.handle, L.OSS_OPT_STAR_STRIP, 100)


def test_deterministic(runner):
    w = make_workload(3, 3, H=160, n_templates=3, blobs_per_512sq=1200, sig_hi=20)
    tm = [(t.pixels, t.rho) for t in w.templates]
    a = runner.screen(w.ref, tm, w.probes, w.feat_mask, w.tol_P, w.tol_Q)
    b = runner.screen(w.ref, tm, w.probes, w.feat_mask, w.tol_P, w.tol_Q)
    assert a[2] == b[2] and np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_cfg2_full_size_sampled(runner):
    """The benchmark workload at full size (4096^2, 7 radii): every sampled
    position bit-exact against the oracle; properties that hold everywhere."""
    w = make_workload(2, 0)
    tm = [(t.pixels, t.rho) for t in w.templates]
    say("cfg2 full size: screening 4096^2")
    mask, cands, n = runner.screen(w.ref, tm, w.probes, w.feat_mask, w.tol_P, w.tol_Q,
                                   list_cap=4 << 20, max_radius=64)
    assert runner.last_value_bits == 32
    assert n == len(cands) == int(mask.sum())
    key = (cands[:, 0] * w.H + cands[:, 1]) * w.W + cands[:, 2]
    assert (np.diff(key) > 0).all()
    assert (mask[0, cands[:, 1], cands[:, 2]] == 1).all() and (cands[:, 3] != 0).all()
    bits = bits_from_list(cands, 1, w.H, w.W)
    rng = np.random.default_rng(0)
    t = w.templates[0]
    xs = np.concatenate([rng.integers(0, w.W, 3000), [t.cx, 16, w.W - 17, 64, w.W - 65, 0]])
    ys = np.concatenate([rng.integers(0, w.H, 3000), [t.cy, 16, w.H - 17, 64, w.H - 65, 0]])
    # plus a band of candidates
    sel = cands[:: max(1, len(cands) // 500)]
    xs = np.concatenate([xs, sel[:, 2]]).astype(np.int32)
    ys = np.concatenate([ys, sel[:, 1]]).astype(np.int32)
    say(f"cfg2 full size: oracle on {len(xs)} sampled positions")
    want = oc.screen_positions(w.ref, tm, w.probes, w.feat_mask, w.tol_P, w.tol_Q, xs, ys)
    assert np.array_equal(bits[0, ys, xs], want[0])
    # the planted template survives at its true radius (32 = scale id 2)
    assert bits[0, t.cy, t.cx] & (1 << 2)


@pytest.mark.parametrize("cfg", [1, 2, 3, 5])
@WIDTHS
def test_interleaved_tables_same_results(runner, cfg, max_r):
    """Interleaved tables (OSS_OPT_TABLE_PLANAR = 0: the quantities of an
    entry side by side, 32-bit, mixed 16-byte or 64-bit entries): plain and
    batched screens equal the oracle."""
    kw = {1: {},
          2: dict(H=230, W=270, blobs_per_512sq=800, sig_hi=24),
          3: dict(H=200, W=260, n_templates=5, blobs_per_512sq=1200, sig_hi=20),
          5: dict(H=224, W=240, n_templates=3, blobs_per_512sq=1200, sig_hi=20)}[cfg]
    w = make_workload(cfg, 1, **kw)
    L = runner.L
    assert L.oss_ctx_get_option(runner.ctx.handle, L.OSS_OPT_TABLE_PLANAR) == 1
    L.oss_ctx_set_option(runner.ctx.handle, L.OSS_OPT_TABLE_PLANAR, 0)
    try:
        _screen_and_compare(runner, w, max_r)
        assert runner.last_plane_bytes == 0
        _screen_and_compare(runner, w, max_r, batched=True)
    finally:
        L.oss_ctx_set_option(runner.ctx.handle, L.OSS_OPT_TABLE_PLANAR, 1)


def test_default_tables_are_planar(runner):
    """The default layout is planar for 32-bit storage, for wide squares
    beside 32-bit sums and gradients (record tables: the squares' sums stay
    below 2^40 at radius 200 for 8-bit pixels), and for 64-bit storage."""
    w = make_workload(2, 0, H=200, W=230, blobs_per_512sq=800, sig_hi=24)
    want = {-2: [32, 32, 32], 200: [32, 40, 32], 1 << 20: [64, 64, 64]}
    for max_r, bits in want.items():
        _screen_and_compare(runner, w, max_r)
        assert runner.last_plane_bytes > 0
        assert [b for _, b in runner.last_slots] == bits
        assert runner.last_entry_bytes == (8 if bits == [64, 64, 64] else 4)


@pytest.mark.parametrize("cfg", [1, 2, 3, 5])
@WIDTHS
def test_pipelined_star_same_results(runner, cfg, max_r):
    """The software-pipelined star pass (OSS_OPT_STAR_PIPE) equals the oracle
    on every workload shape and entry layout, also with narrow strips."""
    kw = {1: {},
          2: dict(H=230, W=270, blobs_per_512sq=800, sig_hi=24),
          3: dict(H=200, W=260, n_templates=5, blobs_per_512sq=1200, sig_hi=20),
          5: dict(H=224, W=240, n_templates=3, blobs_per_512sq=1200, sig_hi=20)}[cfg]
    w = make_workload(cfg, 5, **kw)
    L = runner.L
    h = runner.ctx.handle
    L.oss_ctx_set_option(h, L.OSS_OPT_STAR_PIPE, 1)
    try:
        _screen_and_compare(runner, w, max_r)
        L.oss_ctx_set_option(h, L.OSS_OPT_STAR_STRIP, 64)
        _screen_and_compare(runner, w, max_r, pitch_pad=5)
    finally:
        L.oss_ctx_set_option(h, L.OSS_OPT_STAR_PIPE, 0)
        L.oss_ctx_set_option(h, L.OSS_OPT_STAR_STRIP, 512)


@pytest.mark.parametrize("cfg", [1, 2, 3, 5])
@WIDTHS
def test_unstaged_star_same_results(runner, cfg, max_r):
    """With staged lookups off (OSS_OPT_STAR_STAGED = 0: every quantity at
    every lookup) the plain and the batched star passes equal the oracle on
    every workload shape and entry layout, also with narrow strips."""
    kw = {1: {},
          2: dict(H=230, W=270, blobs_per_512sq=800, sig_hi=24),
          3: dict(H=200, W=260, n_templates=5, blobs_per_512sq=1200, sig_hi=20),
          5: dict(H=224, W=240, n_templates=3, blobs_per_512sq=1200, sig_hi=20)}[cfg]
    w = make_workload(cfg, 6, **kw)
    L = runner.L
    h = runner.ctx.handle
    assert L.oss_ctx_get_option(h, L.OSS_OPT_STAR_STAGED) == 1
    L.oss_ctx_set_option(h, L.OSS_OPT_STAR_STAGED, 0)
    try:
        _screen_and_compare(runner, w, max_r)
        _screen_and_compare(runner, w, max_r, batched=True)
        L.oss_ctx_set_option(h, L.OSS_OPT_STAR_STRIP, 64)
        _screen_and_compare(runner, w, max_r, pitch_pad=5)
    finally:
        L.oss_ctx_set_option(h, L.OSS_OPT_STAR_STAGED, 1)
        L.oss_ctx_set_option(h, L.OSS_OPT_STAR_STRIP, 512)
