"""The C-ABI library on the CPU: it loads, exports every declared entry point,
and its host-only calls (status names, footprints, template features, exact
feature bounds, argument errors) agree with the oracle.  No GPU call is made."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle.core as oc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_1707_05647_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        from paper_1707_05647_amd import build
        build.build()
    return L


def declared_functions():
    src = open(os.path.join(ROOT, "include", "oss.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+char\s*\*|int)\s*(oss_\w+)\s*\(", src, re.M)))


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 11, names
    raw = C.CDLL(lib.LIB_PATH)
    for n in names:
        assert hasattr(raw, n), n
    assert set(names) == set(lib.EXPORTED)


def test_status_strings(lib):
    assert lib.status_string(0) == "OSS_OK"
    assert lib.status_string(-1) == "OSS_E_ARG"
    assert lib.status_string(-3) == "OSS_E_OVERFLOW"
    assert lib.status_string(lib.OSS_E_LIMIT) == "OSS_E_LIMIT"
    assert lib.status_string(lib.OSS_E_CANCELLED) == "OSS_E_CANCELLED"
    assert lib.status_string(lib.OSS_E_TIMEOUT) == "OSS_E_TIMEOUT"


def test_status_codes_match_header(lib):
    hdr = open(os.path.join(ROOT, "include", "oss.h")).read()
    for name, val in re.findall(r"#define (OSS_E_\w+) \((-\d+)\)", hdr):
        assert getattr(lib, name) == int(val), name


def test_server_calls_refuse_a_null_server(lib):
    """Argument errors of the serving calls come back before any device work
    (no GPU needed)."""
    raw = lib.load()
    assert raw.oss_server_cancel(None, 1) == lib.OSS_E_ARG
    assert raw.oss_server_release(None, 1) == lib.OSS_E_ARG
    assert raw.oss_server_pump(None, 0, None) == lib.OSS_E_ARG
    cfg = lib.oss_server_config(1 << 30, 1, 8, -1)  # negative queue timeout
    out = C.c_void_p()
    assert raw.oss_server_create(0, C.byref(cfg), C.byref(out)) == lib.OSS_E_ARG


def test_ref_bytes(lib):
    d = lib.image_desc(4096, 4096)
    # any radius (up to 2047): the squares need 64 bits, the sums (255 A(r))
    # and the gradients (510 A(r) <= 4.28e9) still fit 32: 16-byte entries
    b3 = lib.oss_ref_bytes(d, 7)
    b1 = lib.oss_ref_bytes(d, 1)           # 8-bit sums fit 32 bits at any radius
    b3_64 = lib.oss_ref_bytes(d, 7, 64)    # radius <= 64: every sum below 2^32
    b3_big = lib.oss_ref_bytes(d, 7, 3000)  # gradients past 2^32: 64-bit entries
    tables = 3 * 4097 * 4112
    assert tables * 4 <= b1 < tables * 4 * 1.2
    assert tables * 16 <= b3 < tables * 16 * 1.2
    assert 3 * tables * 8 <= b3_big < 3 * tables * 8 * 1.2
    assert 3 * tables * 4 <= b3_64 < 3 * tables * 4 * 1.2
    # 12-bit squares at radius 96 do not fit 32 bits; sums alone do
    d12 = lib.image_desc(1024, 1024, lib.OSS_U16, 12)
    assert lib.oss_ref_bytes(d12, 2, 96) > 1.9 * lib.oss_ref_bytes(d12, 1, 96)
    with pytest.raises(lib.OssError):
        lib.oss_ref_bytes(lib.image_desc(0, 10), 7)
    with pytest.raises(lib.OssError):
        lib.oss_ref_bytes(d, 8)


@pytest.mark.parametrize("seed", range(6))
def test_template_features_match_oracle(lib, seed):
    rng = np.random.default_rng(seed)
    h, w = int(rng.integers(3, 40)), int(rng.integers(3, 40))
    depth = 8 if seed % 2 == 0 else 12
    img = rng.integers(0, 2 ** depth, (h, w)).astype(np.uint8 if depth == 8 else np.uint16)
    rmax = min((w - 1) // 2, w - 1 - (w - 1) // 2, (h - 1) // 2, h - 1 - (h - 1) // 2)
    for rho in range(0, rmax + 1):
        want = oc.template_features(img, rho)
        for fm in (1, 2, 3, 4, 7):
            if fm & 4 and rho == rmax:
                # the gradient at the border is clamped: the star must stay inside
                with pytest.raises(lib.OssError):
                    lib.oss_template_features(img, rho, fm, bit_depth=depth)
                continue
            got = lib.oss_template_features(img, rho, fm, bit_depth=depth)
            for f in range(3):
                assert got.F[f] == (want[f] if fm & (1 << f) else 0), (rho, fm, f)
            assert got.rho == rho
    # rho < 0 picks the largest fitting radius, one less with the gradient
    assert lib.oss_template_features(img, -1, 3).rho == rmax
    if rmax >= 1:
        assert lib.oss_template_features(img, -1, 7).rho == rmax - 1
    with pytest.raises(lib.OssError):
        lib.oss_template_features(img, rmax + 1, 7)


def test_template_features_strided(lib):
    rng = np.random.default_rng(3)
    big = rng.integers(0, 256, (40, 64)).astype(np.uint8)
    view = big[3:38, 5:40]  # non-contiguous rows; rho 16 with its 1-pixel apron
    got = lib.oss_template_features(np.ascontiguousarray(view), 16, 7)
    want = oc.template_features(view, 16)
    assert list(got.F) == list(want)


def test_feature_bounds_match_cross_multiplied_compare(lib):
    """lo <= F <= hi holds exactly when the oracle's cross-multiplied test passes."""
    rng = np.random.default_rng(11)
    for _ in range(400):
        f = int(rng.integers(0, 3))
        r, rho = int(rng.integers(0, 200)), int(rng.integers(0, 200))
        FT = int(rng.integers(0, 10 ** int(rng.integers(1, 12))))
        P, Q = int(rng.integers(0, 150)), int(rng.integers(1, 101))
        Pv = [0, 0, 0]
        Pv[f] = P
        lo, hi = lib.oss_feature_bounds(f, FT, r, rho, Pv, Q)
        cands = {lo - 1, lo, lo + 1, hi - 1, hi, hi + 1, 0, FT}
        for F in cands:
            if F < 0 or F >= 2 ** 62:
                continue
            want = oc.feature_pass(f, F, FT, r, rho, P, Q)
            assert (lo <= F <= hi) == want, (f, F, FT, r, rho, P, Q, lo, hi)


def test_screen_argument_errors_before_any_launch(lib):
    L = lib.load()
    tol = lib.tolerance((1, 1, 1), 20)
    tm = (lib.oss_template_feat * 1)()
    pr = (lib.oss_probe * 1)(lib.oss_probe(0, 0, 4))
    # null context / reference / count
    assert L.oss_screen(None, None, tm, 1, pr, 1, C.byref(tol), 7, None, None, 0, None,
                        None) == lib.OSS_E_ARG
    bad = lib.tolerance((1, 1, 1), 0)
    assert L.oss_screen(None, None, tm, 1, pr, 1, C.byref(bad), 7, None, None, 0, None,
                        None) == lib.OSS_E_ARG
    assert L.oss_ref_create(None, None, 7, -1, None) == lib.OSS_E_ARG
    assert L.oss_ref_build(None, None, None) == lib.OSS_E_ARG
    # table layout queries need a reference and every output
    out = (lib.oss_quantity_layout * lib.OSS_MAX_QUANTITIES)()
    nq, plane = C.c_int32(), C.c_int64()
    assert L.oss_ref_layout_q(None, out, C.byref(nq), C.byref(plane)) == lib.OSS_E_ARG
    es = C.c_int32()
    off = (C.c_int64 * lib.OSS_MAX_QUANTITIES)()
    bits = (C.c_int32 * lib.OSS_MAX_QUANTITIES)()
    assert L.oss_ref_layout(None, C.byref(es), off, bits, C.byref(plane)) == lib.OSS_E_ARG


def test_server_argument_errors(lib):
    """Config and null-handle errors are reported before any device work."""
    L = lib.load()
    h = C.c_void_p()
    for budget, lanes, mb in ((0, 1, 1), (1 << 30, 0, 1), (1 << 30, 9, 1), (1 << 30, 1, 0)):
        cfg = lib.oss_server_config(budget, lanes, mb)
        assert L.oss_server_create(0, C.byref(cfg), C.byref(h)) == lib.OSS_E_ARG
    assert L.oss_server_create(0, None, C.byref(h)) == lib.OSS_E_ARG
    rid = C.c_int64()
    assert L.oss_server_submit(None, None, C.byref(rid)) == lib.OSS_E_ARG
    assert L.oss_server_pump(None, 0, None) == lib.OSS_E_ARG
    assert L.oss_server_drain(None) == lib.OSS_E_ARG
    assert L.oss_server_release(None, 1) == lib.OSS_E_ARG
    assert L.oss_server_destroy(None) == lib.OSS_E_ARG
    out = lib.oss_result()
    assert L.oss_server_result(None, 1, C.byref(out)) == lib.OSS_E_ARG


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_template_ring_features_match_oracle(lib, seed):
    rng = np.random.default_rng(40 + seed)
    h, w = int(rng.integers(9, 60)), int(rng.integers(9, 60))
    img = rng.integers(0, 256, (h, w)).astype(np.uint8)
    rho = min((w - 1) // 2, (h - 1) // 2) - 1
    for n_rings in (1, 2, 3, 4):
        got = lib.oss_template_features_rings(img, rho, 7, n_rings)
        want, radii = oc.template_ring_features(img, rho, n_rings)
        assert [g.rho for g in got] == radii
        assert [list(g.F) for g in got] == want.tolist()
    for bad in (0, 5):
        with pytest.raises(lib.OssError):
            lib.oss_template_features_rings(img, rho, 7, bad)


def test_region_argument_errors(lib):
    L = lib.load()
    pr = (lib.oss_probe * 1)(lib.oss_probe(0, 0, 3))
    dummy = C.c_void_p(1)
    assert L.oss_region(None, 8, 8, 1, pr, 1, dummy, 1, dummy, dummy, None) == lib.OSS_E_ARG


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_alg1_probes_match_oracle_membership(lib, seed):
    """The library's Algorithm 1 template side (resize, crop, star features,
    quantiser, marking) gives, band by band, exactly the oracle's marked
    cells: each probe box is the product of two cells per feature."""
    from fractions import Fraction as Fr
    from itertools import product

    from oracle import alg1
    rng = np.random.default_rng(60 + seed)
    n = int(rng.integers(9, 30))
    depth = 8 if seed != 2 else 12
    img = rng.integers(0, 2 ** depth, (n, n)).astype(np.uint8 if depth == 8 else np.uint16)
    fm = (7, 3, 5)[seed]
    qbar = (3, 150, 4) if depth == 8 else (40, 40000, 60)
    alpha, beta = (Fr(1, 2), Fr(2)) if seed != 1 else (Fr(3, 4), Fr(3, 2))
    probes = lib.oss_alg1_probes(img, 5, alpha, beta, qbar, fm, bit_depth=depth)
    want = alg1.membership(img, alpha, beta, qbar, fm)
    feats = [f for f in range(3) if fm & (1 << f)]
    assert {p.scale_id for p in probes} <= set(range(len(want)))
    for b, (r, q, marked) in enumerate(want):
        got = set()
        for p in probes:
            if p.scale_id != b:
                continue
            assert p.template_id == 5 and p.r == r
            cells = []
            for f in feats:
                lo_c, hi_c = alg1.quantise(p.lo[f], q[f]), alg1.quantise(p.hi[f], q[f])
                assert hi_c == lo_c + 1
                # the bounds are the box's exact edges
                assert alg1.quantise(p.lo[f] - 1, q[f]) == lo_c - 1
                assert alg1.quantise(p.hi[f] + 1, q[f]) == hi_c + 1
                cells.append((lo_c, hi_c))
            got.update(product(*cells))
        assert got == marked, (b, len(got), len(marked))


def test_alg1_argument_errors(lib):
    from fractions import Fraction as Fr
    img = np.zeros((9, 9), np.uint8)
    for kw in (dict(alpha=Fr(2), beta=Fr(1, 2), q=(1, 1, 1)),
               dict(alpha=Fr(1, 2), beta=Fr(2), q=(0, 1, 1))):
        with pytest.raises(lib.OssError):
            lib.oss_alg1_probes(img, 0, kw["alpha"], kw["beta"], kw["q"], 7)
    with pytest.raises(lib.OssError):
        lib.oss_alg1_probes(np.zeros((9, 8), np.uint8), 0, Fr(1, 2), Fr(2), (1, 1, 1), 7)


@pytest.mark.parametrize("seed", [0, 1])
def test_template_moments_match_oracle(lib, seed):
    from oracle import moments as om
    rng = np.random.default_rng(70 + seed)
    h, w = int(rng.integers(5, 40)), int(rng.integers(5, 40))
    depth = (8, 12)[seed]
    img = rng.integers(0, 2 ** depth, (h, w)).astype(np.uint8 if depth == 8 else np.uint16)
    rmax = min((w - 1) // 2, w - 1 - (w - 1) // 2, (h - 1) // 2, h - 1 - (h - 1) // 2)
    for rho in range(rmax + 1):
        got = lib.oss_template_moments(img, rho, bit_depth=depth)
        assert (got.F1, got.F2, got.Sx, got.Sy) == om.template_moments(img, rho)
        assert got.rho == rho


def test_moment_feature_sets(lib):
    d = lib.image_desc(256, 256)
    for fm in (25, 27):
        assert lib.oss_ref_bytes(d, fm, 20) > 0
    for fm in (8, 16, 24, 9, 17, 29, 31, 32):
        with pytest.raises(lib.OssError):
            lib.oss_ref_bytes(d, fm, 20)
