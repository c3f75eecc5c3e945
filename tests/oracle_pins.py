"""Pins of the C oracle against facts fixed outside it.

Each ``check_*`` function raises AssertionError when the oracle library
``lib`` disagrees with the paper, a closed form, a library routine or an
independent enumerator.  ``test_oracle_pins.py`` runs them on the real
oracle; ``test_oracle_mutants.py`` runs them on deliberately broken copies
of the oracle to show that each plausible mistake is caught.
"""
from __future__ import annotations

import os

import itertools

import numpy as np
from scipy.signal import correlate2d

import oracle.core as oc
from oracle import enum_star as en

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

# s(r) = round(r / sqrt(2)), evaluated by hand for the radii the workloads use
S_TABLE = {0: 0, 1: 1, 2: 1, 3: 2, 8: 6, 16: 11, 24: 17, 32: 23, 48: 34, 64: 45, 96: 68,
           128: 91}


def _rand_img(shape, seed, hi=255):
    rng = np.random.default_rng(seed)
    dt = np.uint8 if hi <= 255 else np.uint16
    return rng.integers(0, hi + 1, shape).astype(dt)


def check_half_width_and_area(lib):
    for r, s in S_TABLE.items():
        assert oc.square_half(r, lib) == s, (r, oc.square_half(r, lib), s)
    for r in range(0, 131):
        s = en.nearest_half_width(r)
        # closed form: (2s+1)^2 square pixels + 2r^2+2r+1 diamond pixels
        assert oc.star_area(r, lib) == (2 * s + 1) ** 2 + 2 * r * r + 2 * r + 1, r


def read_golden_star():
    rows = []
    with open(os.path.join(GOLDEN, "star_r3.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([int(v) for v in line.split()])
    return np.array(rows)


def check_golden_7x7(lib):
    want = read_golden_star()
    got = np.array([[oc.star_weight(dx, dy, 3, lib) for dx in range(-3, 4)]
                    for dy in range(-3, 4)])
    assert (got == want).all(), got
    # the weight seen through the feature sum of a unit impulse
    img = np.zeros((7, 7), np.uint8)
    for dy in range(-3, 4):
        for dx in range(-3, 4):
            img[:] = 0
            img[3 + dy, 3 + dx] = 1
            F = oc.star_features(img, [3], [3], 3, lib)[0]
            assert F[0] == want[dy + 3, dx + 3] and F[1] == want[dy + 3, dx + 3]


def check_enumerator(lib, sizes=((13, 11), (9, 16)), radii=(1, 2, 3, 4, 5)):
    for seed, (H, W) in enumerate(sizes):
        for hi in (255, 4095):
            img = _rand_img((H, W), 10 + seed, hi)
            rows = img.tolist()
            for r in radii:
                if 2 * r + 1 > min(H, W):
                    continue
                ys, xs = np.mgrid[0:H, 0:W]
                F = oc.star_features(img, xs.ravel(), ys.ravel(), r, lib)
                for i, (x, y) in enumerate(zip(xs.ravel(), ys.ravel())):
                    e = en.star_features(rows, int(x), int(y), r)
                    if e is None:
                        assert (F[i] == -1).all()
                    else:
                        assert tuple(int(v) for v in F[i]) == e, (r, x, y, F[i], e)


def _kernel(r):
    """Integer star kernel built from the enumerator's pixel sets."""
    w = np.zeros((2 * r + 1, 2 * r + 1), np.int64)
    for dx, dy in en.square_pixels(r) + en.diamond_pixels(r):
        w[dy + r, dx + r] += 1
    return w


def check_correlate(lib, H=24, W=21, radii=(1, 2, 4, 6)):
    img = _rand_img((H, W), 3)
    q_all = [img.astype(np.int64), img.astype(np.int64) ** 2,
             np.array([[en.gradient_at(img.tolist(), x, y) for x in range(W)]
                       for y in range(H)], np.int64)]
    for r in radii:
        ys, xs = np.mgrid[r:H - r, r:W - r]
        F = oc.star_features(img, xs.ravel(), ys.ravel(), r, lib)
        for q, qa in enumerate(q_all):
            want = correlate2d(qa, _kernel(r), mode="valid")
            assert (F[:, q].reshape(want.shape) == want).all(), (r, q)


def check_closed_forms(lib):
    # constant image: F = (c A, c^2 A, 0)
    for c in (0, 7, 255):
        img = np.full((15, 17), c, np.uint8)
        for r in (1, 3, 5):
            A = (2 * en.nearest_half_width(r) + 1) ** 2 + 2 * r * r + 2 * r + 1
            ys, xs = np.mgrid[r:15 - r, r:17 - r]
            F = oc.star_features(img, xs.ravel(), ys.ravel(), r, lib)
            assert (F[:, 0] == c * A).all() and (F[:, 1] == c * c * A).all()
            assert (F[:, 2] == 0).all()
    # linear ramp I = a x + b y + c: the symmetric star returns A * I at the
    # centre; away from the border G = 2|a| + 2|b| everywhere in the star
    a, b, c0 = 2, 3, 5
    H, W = 30, 36
    yy, xx = np.mgrid[0:H, 0:W]
    img = (a * xx + b * yy + c0).astype(np.uint8)
    for r in (2, 4, 7):
        A = (2 * en.nearest_half_width(r) + 1) ** 2 + 2 * r * r + 2 * r + 1
        ys, xs = np.mgrid[r + 1:H - 1 - r, r + 1:W - 1 - r]
        F = oc.star_features(img, xs.ravel(), ys.ravel(), r, lib)
        assert (F[:, 0] == A * img[ys.ravel(), xs.ravel()].astype(np.int64)).all()
        assert (F[:, 2] == A * (2 * abs(a) + 2 * abs(b))).all()


_D4 = [
    ("rot90", lambda a: np.rot90(a, 1)),
    ("rot180", lambda a: np.rot90(a, 2)),
    ("rot270", lambda a: np.rot90(a, 3)),
    ("transpose", lambda a: a.T),
    ("fliplr", lambda a: a[:, ::-1]),
    ("flipud", lambda a: a[::-1, :]),
]


def check_d4(lib, H=19, W=23, radii=(2, 4, 7)):
    img = _rand_img((H, W), 5)
    idx = np.arange(H * W).reshape(H, W)
    for name, T in _D4:
        timg = np.ascontiguousarray(T(img))
        tidx = T(idx)
        th, tw = timg.shape
        ys, xs = np.mgrid[0:th, 0:tw]
        src = tidx[ys, xs].ravel()
        oy, ox = np.divmod(src, W)
        for r in radii:
            Ft = oc.star_features(timg, xs.ravel(), ys.ravel(), r, lib)
            Fo = oc.star_features(img, ox, oy, r, lib)
            assert (Ft == Fo).all(), (name, r)


def check_compare(lib):
    # r = rho: the area and gradient factors cancel, |F - FT| Q <= P FT
    for f in (0, 1, 2):
        for F, ok in ((949, False), (950, True), (1000, True), (1050, True), (1051, False)):
            assert oc.feature_pass(f, F, 1000, 16, 16, 1, 20, lib) == ok, (f, F)
    # r = 16 (A = 1074) against rho = 8 (A = 314), exact equality at P = 0:
    # sums and squares compare F * 314 with FT * 1074 ...
    assert oc.feature_pass(0, 537, 157, 16, 8, 0, 1, lib)
    assert not oc.feature_pass(0, 538, 157, 16, 8, 0, 1, lib)
    assert not oc.feature_pass(1, 536, 157, 16, 8, 0, 1, lib)
    # ... and gradients F * 314 * 16 with FT * 1074 * 8
    assert oc.feature_pass(2, 537, 314, 16, 8, 0, 1, lib)
    assert not oc.feature_pass(2, 537, 157, 16, 8, 0, 1, lib)
    # monotone in the tolerance
    rng = np.random.default_rng(9)
    for _ in range(300):
        f = int(rng.integers(0, 3))
        r, rho = int(rng.integers(1, 40)), int(rng.integers(1, 40))
        FT = int(rng.integers(0, 10 ** 6))
        F = int(rng.integers(0, 10 ** 6))
        prev = False
        for P in (0, 1, 3, 10, 40, 200):
            cur = oc.feature_pass(f, F, FT, r, rho, P, 100, lib)
            assert cur or not prev
            prev = cur


def check_planted_exact(lib):
    """An exact cut, and its quarter turns / transpose / mirror, survives at
    its centre for every tolerance (P = 0 included), with all features."""
    from synth import blob_image, make_rng, cut_patch
    img = blob_image(96, 96, make_rng(99, 0), blobs_per_512sq=400)
    cx, cy, rho = 50, 41, 9
    probes = [(0, 0, rho)]
    for kw in ({}, {"quarter_turns": 1}, {"quarter_turns": 2}, {"quarter_turns": 3},
               {"transpose": True}, {"flip": True}):
        tm = cut_patch(img, cx, cy, rho + 1, **kw)
        bits = oc.screen_positions(img, [(tm, rho)], probes, 7, (0, 0, 0), 1, [cx], [cy], lib)
        assert bits[0, 0] == 1, kw
    # and a wrong location does not survive at P = 0
    tm = cut_patch(img, cx, cy, rho + 1)
    bits = oc.screen_positions(img, [(tm, rho)], probes, 7, (0, 0, 0), 1, [cx + 3], [cy], lib)
    assert bits[0, 0] == 0
    # an even-width, odd-height cut: its centre pixel is (floor((w-1)/2),
    # floor((h-1)/2)), so the copy survives at the image pixel that lands
    # there, and not one column further (a one-pixel apron around the star
    # keeps the gradients of the cut equal to the image's)
    w, h = 2 * rho + 4, 2 * rho + 5
    x0, y0 = cx - (w - 1) // 2, cy - (h - 1) // 2
    tm = img[y0:y0 + h, x0:x0 + w].copy()
    bits = oc.screen_positions(img, [(tm, rho)], probes, 7, (0, 0, 0), 1, [cx, cx + 1],
                               [cy, cy], lib)
    assert bits[0, 0] == 1 and bits[0, 1] == 0


def _py_pass(f, F, FT, r, rho, P, Q):
    """The feature test in Python integers, with the weighted areas from the
    enumerator's pixel sets (an implementation independent of the oracle)."""
    def area(rr):
        return len(en.square_pixels(rr)) + len(en.diamond_pixels(rr))
    c_ref, c_t = (r, rho) if f == 2 else (1, 1)
    x_ref = F * area(rho) * c_ref
    x_t = FT * area(r) * c_t
    return (Q - P) * x_t <= Q * x_ref <= (Q + P) * x_t


def _ring_chain(r, n):
    out = [r]
    for _ in range(n - 1):
        out.append(en.nearest_half_width(out[-1]))
    return out


def check_rings_brute_force(lib):
    """Multi-central-area screen (Sec. "Scale Invariance", central areas of
    sizes n, n/lambda, n/lambda^2 with lambda = sqrt 2): at every position of
    a small image, probe (t, k, r) passes iff for every ring j the star of
    radius r_j (r_0 = r, r_{j+1} = round(r_j / sqrt 2)) matches the
    template's central star of radius rho_j the same way; enumerated in
    Python from the star's pixel sets."""
    img = _rand_img((21, 24), 31)
    rng = np.random.default_rng(32)
    templates = []
    for rho in (5, 4):
        cx, cy = int(rng.integers(rho + 1, 24 - rho - 1)), int(rng.integers(rho + 1, 21 - rho - 1))
        tm = img[cy - rho - 1:cy + rho + 2, cx - rho - 1:cx + rho + 2].copy()
        tm = np.clip(tm.astype(np.int64) + rng.integers(-6, 7, tm.shape), 0, 255).astype(np.uint8)
        templates.append((tm, rho))
    probes = [(0, 0, 4), (0, 1, 5), (0, 2, 6), (1, 0, 3), (1, 3, 4)]
    P, Q = (25, 45, 60), 100
    ys, xs = np.mgrid[0:21, 0:24]
    rows = img.tolist()
    seen = set()
    for n_rings in (1, 2, 3):
        got = oc.screen_rings_positions(img, templates, probes, 7, P, Q, n_rings, xs.ravel(),
                                        ys.ravel(), lib)
        for t, (tm, rho) in enumerate(templates):
            trows = tm.tolist()
            c = ((tm.shape[1] - 1) // 2, (tm.shape[0] - 1) // 2)
            rho_c = _ring_chain(rho, n_rings)
            FT = [en.star_features(trows, c[0], c[1], rj) for rj in rho_c]
            for i, (x, y) in enumerate(zip(xs.ravel(), ys.ravel())):
                want = 0
                for tt, k, r in probes:
                    if tt != t:
                        continue
                    ok = True
                    for j, rj in enumerate(_ring_chain(r, n_rings)):
                        F = en.star_features(rows, int(x), int(y), rj)
                        if F is None:
                            ok = False
                            break
                        ok = all(_py_pass(f, F[f], FT[j][f], rj, rho_c[j], P[f], Q)
                                 for f in range(3))
                        if not ok:
                            break
                    want |= (1 << k) if ok else 0
                assert int(got[t, i]) == want, (n_rings, t, x, y, int(got[t, i]), want)
                seen.add(want != 0)
    assert seen == {True, False}  # the case mixes passing and failing positions


def check_rings_consistency(lib):
    """One ring is the plain screen; more rings never add candidates; an
    exact cut survives at its centre at P = 0 with every ring."""
    from synth import blob_image, make_rng, cut_patch
    img = blob_image(80, 90, make_rng(98, 0), blobs_per_512sq=1500, sig_hi=10)
    cx, cy, rho = 44, 37, 10
    tm = cut_patch(img, cx, cy, rho + 1)
    tms = [(tm, rho)]
    probes = [(0, 0, 8), (0, 1, 10), (0, 2, 13)]
    P, Q = (8, 12, 40), 100
    plain = oc.screen_full(img, tms, probes, 7, P, Q, lib)
    prev = None
    for n_rings in (1, 2, 3, 4):
        b = oc.screen_rings_full(img, tms, probes, 7, P, Q, n_rings, lib)
        if n_rings == 1:
            assert np.array_equal(b, plain)
        else:
            assert not (b & ~prev).any()
        prev = b
        exact = oc.screen_rings_positions(img, tms, [(0, 0, rho)], 7, (0, 0, 0), 1, n_rings,
                                          [cx], [cy], lib)
        assert exact[0, 0] == 1, n_rings
    assert (prev != plain).any()  # the rings do prune


def check_region(lib):
    """Preserved region: one candidate covers exactly its star's pixels (the
    7x7 example of Fig. os for r = 3, the enumerator's square and diamond
    pixel sets otherwise); several candidates and scales give the union."""
    golden = read_golden_star() > 0
    reg = oc.region_full(9, 9, 1, [(0, 4, 4, 1)], {(0, 0): 3}, lib)
    assert (reg[0, 1:8, 1:8].astype(bool) == golden).all() and reg.sum() == golden.sum()
    for r in (1, 2, 5, 8, 13):
        n = 2 * r + 5
        reg = oc.region_full(n, n, 1, [(0, r + 2, r + 2, 1)], {(0, 0): r}, lib)
        want = np.zeros((n, n), bool)
        for dx, dy in en.square_pixels(r) + en.diamond_pixels(r):
            want[r + 2 + dy, r + 2 + dx] = True
        assert (reg[0].astype(bool) == want).all(), r
    # two scales on one candidate, two candidates, two templates
    radius_of = {(0, 0): 2, (0, 3): 4, (1, 1): 3}
    cands = [(0, 6, 5, 0b1001), (0, 9, 12, 0b1), (1, 7, 7, 0b10)]
    reg = oc.region_full(16, 18, 2, cands, radius_of, lib)
    want = np.zeros((2, 16, 18), bool)
    for t, y, x, bits in cands:
        for k in range(4):
            if (bits >> k) & 1:
                r = radius_of[(t, k)]
                for dx, dy in en.square_pixels(r) + en.diamond_pixels(r):
                    want[t, y + dy, x + dx] = True
    assert (reg.astype(bool) == want).all()


def check_alg1(lib):
    """Algorithm 1's pieces: the scale bands for [1/2, 2] (four bands; sizes
    from exact integer square roots), the bilinear resize on a textbook
    example (pixel-centre aligned, edges replicated, half up), the
    quantiser's marking guarantee (Sec. "Scale Invariance": marking Q(f-q/2),
    Q(f), Q(f+q/2) admits every g with |f - g| < q/2), and the exact-copy
    guarantee at unit scale."""
    from fractions import Fraction as Fr

    from oracle import alg1
    assert alg1.band_count(Fr(1, 2), Fr(2)) == 4
    assert alg1.band_count(Fr(1), Fr(1)) == 0 and alg1.band_count(Fr(3, 4), Fr(1)) == 1
    assert alg1.bands(64, Fr(1, 2), Fr(2)) == [(91, 91, 128), (64, 64, 90), (46, 46, 64),
                                               (32, 32, 45)]
    assert alg1.bands(33, Fr(1, 2), Fr(2)) == [(47, 47, 66), (33, 33, 46), (24, 24, 33),
                                               (17, 17, 23)]
    # resize: 2x2 -> 4x4 and back, identity, constants
    up = alg1.resize(np.array([[0, 100], [0, 100]], np.uint16), 4)
    assert (up == np.array([[0, 25, 75, 100]] * 4)).all(), up
    down = alg1.resize(up, 2)
    assert (down == np.array([[13, 88]] * 2)).all(), down
    rng = np.random.default_rng(5)
    t = rng.integers(0, 256, (9, 9)).astype(np.uint16)
    assert (alg1.resize(t, 9) == t).all()
    assert (alg1.resize(np.full((7, 7), 200, np.uint16), 12) == 200).all()
    # marking guarantee, on random rationals
    for _ in range(2000):
        q = int(rng.integers(1, 50))
        f = Fr(int(rng.integers(0, 10 ** 6)), int(rng.integers(1, 7)))
        g = f + Fr(int(rng.integers(-10 ** 4, 10 ** 4)), 10 ** 4) * Fr(q, 2)
        if abs(f - g) >= Fr(q, 2):
            continue
        marked = {alg1.quantise(f - Fr(q, 2), q), alg1.quantise(f, q),
                  alg1.quantise(f + Fr(q, 2), q)}
        assert alg1.quantise(g, q) in marked
    assert [alg1.quantise(v, 10) for v in (4, 5, 14, 15, Fr(29, 2))] == [0, 1, 1, 2, 1]
    # the guarantee on the membership array itself: for every crop's feature
    # vector F, every g with |g_f - F_f| < q_f / 2 in each feature is marked
    tm = rng.integers(0, 256, (17, 17)).astype(np.uint16)
    qbar = (1, 40, 2)
    mem = alg1.membership(tm, Fr(1, 2), Fr(2), qbar, 7, lib)
    for (m, lo, hi), (r, q, marked) in zip(alg1.bands(17, Fr(1, 2), Fr(2)), mem):
        for k in range(lo, hi + 1):
            F, _ = alg1.crop_features(tm, k, m, lib)
            for u in itertools.product((-1, 0, 1), repeat=3):
                g = [F[f] + u[f] * (Fr(q[f], 2) - Fr(1, 1000)) for f in range(3)]
                assert tuple(alg1.quantise(g[f], q[f]) for f in range(3)) in marked, (k, m, u)
    # the step is per pixel of star area: a flat template of value c against
    # a flat reference of value c + d, d < qbar/2, is marked in every band
    # (its star sums differ by d A(r) < q/2); d = 2 qbar is marked in none
    # (Q(f + 2q) = Q(f) + 2, while the marked cells reach Q(f) + 1 at most)
    for d, want in ((2, 1), (10, 0)):
        ref = np.full((70, 70), 100 + d, np.uint16)
        flat = np.full((25, 25), 100, np.uint16)
        bits = alg1.screen(ref, [flat], Fr(1, 2), Fr(2), (5, 1, 1), 1, lib)
        nb = len(alg1.bands(25, Fr(1, 2), Fr(2)))
        assert int(bits[0, 35, 35]) == (want * ((1 << nb) - 1)), (d, int(bits[0, 35, 35]))
    # an exact cut survives at its centre in the band holding k = n
    from synth import blob_image, make_rng, cut_patch
    img = blob_image(120, 130, make_rng(97, 0), blobs_per_512sq=1500, sig_hi=10)
    cx, cy, half = 64, 58, 12
    tm = cut_patch(img, cx, cy, half)                          # n = 25
    n = 2 * half + 1
    bits = alg1.screen(img, [tm], Fr(1, 2), Fr(2), (1, 60, 1), 3, lib)
    b = [i for i, (_, lo, hi) in enumerate(alg1.bands(n, Fr(1, 2), Fr(2))) if lo <= n <= hi][0]
    assert (int(bits[0, cy, cx]) >> b) & 1
    # fine steps keep few patches
    assert bits[0].astype(bool).sum() < 0.2 * bits[0].size


def _star_pixels(r):
    """(dx, dy, weight) over the enumerator's square and diamond sets."""
    w = {}
    for dx, dy in en.square_pixels(r) + en.diamond_pixels(r):
        w[(dx, dy)] = w.get((dx, dy), 0) + 1
    return [(dx, dy, v) for (dx, dy), v in w.items()]


def check_moments(lib):
    """The paper's features over the star: first moments against the extended
    Prewitt ramps (correlation with the weighted ramp kernels and a linear
    ramp's closed form), their magnitude under quarter turns, and the three
    tests on hand cases and exact cuts."""
    from oracle import moments as om
    # closed form on a linear ramp I = a x + b y + c: Sx = a sum w dx^2, Sy = b sum w dy^2
    H, W, a, b, c = 40, 44, 3, 2, 7
    yy, xx = np.mgrid[0:H, 0:W]
    img = (a * xx + b * yy + c).astype(np.uint16)
    for r in (2, 5, 9):
        pix = _star_pixels(r)
        sxx = sum(v * dx * dx for dx, dy, v in pix)
        syy = sum(v * dy * dy for dx, dy, v in pix)
        A = sum(v for _, _, v in pix)
        F = om.moments(img, [20], [19], r, lib)[0]
        assert F[0] == A * (a * 20 + b * 19 + c)
        assert F[1] == sum(v * (a * (20 + dx) + b * (19 + dy) + c) ** 2 for dx, dy, v in pix)
        assert F[2] == a * sxx and F[3] == b * syy, (r, F)
    # correlation with the weighted ramp kernels (scipy), random image
    img = _rand_img((23, 27), 41)
    for r in (1, 3, 6):
        kx = np.zeros((2 * r + 1, 2 * r + 1), np.int64)
        ky = np.zeros_like(kx)
        for dx, dy, v in _star_pixels(r):
            kx[dy + r, dx + r] = v * dx
            ky[dy + r, dx + r] = v * dy
        ys, xs = np.mgrid[r:23 - r, r:27 - r]
        F = om.moments(img, xs.ravel(), ys.ravel(), r, lib)
        assert (F[:, 2] == correlate2d(img.astype(np.int64), kx, "valid").ravel()).all()
        assert (F[:, 3] == correlate2d(img.astype(np.int64), ky, "valid").ravel()).all()
    # quarter turn: the moment vector turns, its length stays
    rot = np.rot90(img).copy()
    F0 = om.moments(img, [12], [10], 4, lib)[0]
    # pixel (x, y) of img lands at (y, W-1-x) of rot90 (counter-clockwise)
    F1 = om.moments(rot, [10], [27 - 1 - 12], 4, lib)[0]
    assert F0[0] == F1[0] and F0[1] == F1[1]
    assert F0[2] ** 2 + F0[3] ** 2 == F1[2] ** 2 + F1[3] ** 2
    assert (F1[2], F1[3]) == (F0[3], -F0[2])
    # tests at r = rho reduce to relative differences of the raw values
    FT = (1000, 5000, 30, 40)  # V_T = A F2 - F1^2, M_T = 2500
    ok = om.probe_pass((1049, 5000, 30, 40), FT, 4, 4, (5, 100, 100), 100, om.MEAN, lib)
    assert ok and not om.probe_pass((1051, 5000, 30, 40), FT, 4, 4, (5, 100, 100), 100, om.MEAN,
                                    lib)
    assert om.probe_pass((1000, 5000, 30, 40), FT, 4, 4, (0, 0, 0), 1, 7, lib)
    assert om.probe_pass((1000, 5000, 40, 30), FT, 4, 4, (0, 0, 0), 1, om.MAG, lib)
    assert not om.probe_pass((1000, 5000, 41, 30), FT, 4, 4, (0, 0, 0), 1, om.MAG, lib)
    # magnitude 10% tolerance: |m - 50| <= 5 with m^2 = 55^2 passes, 55^2 + 1 fails
    assert om.probe_pass((1000, 5000, 55, 0), FT, 4, 4, (0, 0, 10), 100, om.MAG, lib)
    assert not om.probe_pass((1000, 5000, 55, 1), FT, 4, 4, (0, 0, 10), 100, om.MAG, lib)
    # r != rho: features built from equal normalised values (mean F1 / A,
    # variance F2 / A - mean^2, magnitude |(Sx, Sy)| / (r A)) pass at P = 0,
    # and one unit more in the raw sum fails
    for r, rho in ((4, 8), (9, 5), (3, 16)):
        A_r, A_t = oc.star_area(r, lib), oc.star_area(rho, lib)
        mean, var, g = 10, 9, 3
        F = (mean * A_r, (var + mean * mean) * A_r, g * r * A_r, 0)
        T = (mean * A_t, (var + mean * mean) * A_t, g * rho * A_t, 0)
        for test, bump in ((om.MEAN, (1, 0, 0, 0)), (om.VAR, (0, 1, 0, 0)),
                           (om.MAG, (0, 0, 1, 0))):
            assert om.probe_pass(F, T, r, rho, (0, 0, 0), 1, test, lib), (r, rho, test)
            Fb = tuple(a + b for a, b in zip(F, bump))
            assert not om.probe_pass(Fb, T, r, rho, (0, 0, 0), 1, test, lib), (r, rho, test)
    # exact cuts survive at their centre with every test at P = 0
    from synth import blob_image, make_rng, cut_patch
    img = blob_image(90, 96, make_rng(95, 0), blobs_per_512sq=1500, sig_hi=10)
    tm = cut_patch(img, 45, 40, 12)
    bits = om.screen_full(img[25:56, 30:62], [(tm, 11)], [(0, 0, 11)], (0, 0, 0), 1, 7, lib)
    assert bits[0, 40 - 25, 45 - 30] == 1 and bits.sum() < 5


ALL_CHECKS = [check_half_width_and_area, check_golden_7x7, check_enumerator, check_correlate,
              check_closed_forms, check_d4, check_compare, check_planted_exact,
              check_rings_brute_force, check_rings_consistency, check_region, check_alg1,
              check_moments]
