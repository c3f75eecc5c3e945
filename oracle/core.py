"""ctypes wrapper of the C oracle (``oss_oracle.c``).

TEST INFRASTRUCTURE ONLY: see the package docstring.  The shared library
is compiled with gcc on first use (or by ``build()``) next to the source.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import tempfile

import numpy as np

F_SUM, F_SQ, F_GRAD = 1, 2, 4

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oss_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboss_oracle.so")
_lib = None


def build(force: bool = False, src: str = _SRC, out: str = _LIB_PATH) -> str:
    """Compile the oracle with gcc (-O2, OpenMP).  Returns the library path."""
    if (not force and os.path.exists(out)
            and os.path.getmtime(out) >= os.path.getmtime(src)):
        return out
    fd, tmp = tempfile.mkstemp(suffix=".so", dir=os.path.dirname(out))
    os.close(fd)
    try:
        subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, src],
                       check=True, capture_output=True, text=True)
        os.chmod(tmp, 0o755)
        os.replace(tmp, out)
    finally:
        if os.path.exists(tmp):
            os.unlink(tmp)
    return out


def _declare(lib):
    i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
    i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
    u16p = np.ctypeslib.ndpointer(np.uint16, flags="C_CONTIGUOUS")
    u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
    lib.oracle_threads.argtypes = []
    lib.oracle_threads.restype = C.c_int
    lib.oracle_square_half.argtypes = [C.c_int]
    lib.oracle_square_half.restype = C.c_int
    lib.oracle_star_weight.argtypes = [C.c_int, C.c_int, C.c_int]
    lib.oracle_star_weight.restype = C.c_int
    lib.oracle_star_area.argtypes = [C.c_int]
    lib.oracle_star_area.restype = C.c_int64
    lib.oracle_gradient.argtypes = [u16p, C.c_int, C.c_int, C.c_int64, i32p]
    lib.oracle_gradient.restype = None
    lib.oracle_features.argtypes = [u16p, i32p, C.c_int, C.c_int, C.c_int64, i32p, i32p,
                                    C.c_int64, C.c_int, i64p]
    lib.oracle_features.restype = None
    lib.oracle_feature_pass.argtypes = [C.c_int, C.c_int64, C.c_int64, C.c_int, C.c_int,
                                        C.c_int, C.c_int]
    lib.oracle_feature_pass.restype = C.c_int
    lib.oracle_screen.argtypes = [u16p, i32p, C.c_int, C.c_int, C.c_int64, i32p, i32p, C.c_int64,
                                  i32p, C.c_int, i64p, i32p, C.c_int, C.c_int, i32p, C.c_int, u32p]
    lib.oracle_screen.restype = C.c_int
    lib.oracle_screen_rings.argtypes = [u16p, i32p, C.c_int, C.c_int, C.c_int64, i32p, i32p,
                                        C.c_int64, i32p, C.c_int, i64p, i32p, C.c_int, C.c_int,
                                        C.c_int, i32p, C.c_int, u32p]
    lib.oracle_screen_rings.restype = C.c_int
    lib.oracle_moments.argtypes = [u16p, C.c_int, C.c_int, C.c_int64, i32p, i32p, C.c_int64,
                                   C.c_int, i64p]
    lib.oracle_moments.restype = None
    return lib


def load(path: str | None = None):
    """Load the oracle library (building it if needed).  ``path`` selects an
    alternative build of the same source (used by the mutation tests)."""
    global _lib
    if path is not None:
        return _declare(C.CDLL(path))
    if _lib is None:
        _lib = _declare(C.CDLL(build()))
    return _lib


def _img16(img) -> np.ndarray:
    a = np.asarray(img)
    if a.ndim != 2 or a.dtype not in (np.uint8, np.uint16):
        raise ValueError("image must be a 2-D uint8 or uint16 array")
    return np.ascontiguousarray(a, dtype=np.uint16)


def threads(lib=None) -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int((lib or load()).oracle_threads())


def square_half(r: int, lib=None) -> int:
    return (lib or load()).oracle_square_half(int(r))


def star_weight(dx: int, dy: int, r: int, lib=None) -> int:
    return (lib or load()).oracle_star_weight(int(dx), int(dy), int(r))


def star_area(r: int, lib=None) -> int:
    return int((lib or load()).oracle_star_area(int(r)))


def gradient(img, lib=None) -> np.ndarray:
    lib = lib or load()
    a = _img16(img)
    H, W = a.shape
    G = np.empty((H, W), np.int32)
    lib.oracle_gradient(a, H, W, W, G)
    return G


def star_features(img, xs, ys, r: int, lib=None, G=None) -> np.ndarray:
    """[n, 3] int64: star sums of I, I^2 and G at (xs[i], ys[i]) for radius r.
    Positions where the star does not fit give -1."""
    lib = lib or load()
    a = _img16(img)
    H, W = a.shape
    if G is None:
        G = gradient(a, lib)
    xs = np.ascontiguousarray(xs, np.int32)
    ys = np.ascontiguousarray(ys, np.int32)
    F = np.empty((len(xs), 3), np.int64)
    lib.oracle_features(a, np.ascontiguousarray(G, np.int32), H, W, W, xs, ys, len(xs), int(r), F)
    return F


def template_features(tmpl, rho: int, lib=None) -> np.ndarray:
    """Features of the radius-rho star at the template centre
    (floor((w-1)/2), floor((h-1)/2)), with the gradient taken on the template."""
    a = _img16(tmpl)
    h, w = a.shape
    cx, cy = (w - 1) // 2, (h - 1) // 2
    F = star_features(a, [cx], [cy], rho, lib)[0]
    if F[0] < 0:
        raise ValueError("template star does not fit")
    return F


def feature_pass(f: int, F: int, FT: int, r: int, rho: int, P: int, Q: int, lib=None) -> bool:
    return bool((lib or load()).oracle_feature_pass(f, int(F), int(FT), int(r), int(rho),
                                                    int(P), int(Q)))


def _probe_arrays(templates, probes, lib):
    FT = np.ascontiguousarray(
        np.stack([template_features(px, rho, lib) for px, rho in templates]), np.int64)
    rho = np.ascontiguousarray([rho for _, rho in templates], np.int32)
    pr = sorted((int(t), int(k), int(r)) for t, k, r in probes)
    pr.sort(key=lambda p: p[2])
    parr = np.ascontiguousarray(np.array(pr, np.int32).reshape(-1, 3))
    return FT, rho, parr


def screen_positions(img, templates, probes, feat_mask: int, P, Q: int, xs, ys,
                     lib=None, G=None) -> np.ndarray:
    """bits[n_tmpl, n]: bit k of entry (t, i) is set iff probe (t, k) passes
    at (xs[i], ys[i]).  ``templates`` is a list of (pixels, rho)."""
    lib = lib or load()
    a = _img16(img)
    H, W = a.shape
    if G is None:
        G = gradient(a, lib)
    FT, rho, parr = _probe_arrays(templates, probes, lib)
    xs = np.ascontiguousarray(xs, np.int32)
    ys = np.ascontiguousarray(ys, np.int32)
    bits = np.zeros((len(templates), len(xs)), np.uint32)
    Pa = np.ascontiguousarray(list(P) + [0] * (3 - len(P)), np.int32)
    rc = lib.oracle_screen(a, np.ascontiguousarray(G, np.int32), H, W, W, xs, ys, len(xs),
                           parr, len(parr), FT, rho, len(templates), int(feat_mask), Pa, int(Q),
                           bits)
    if rc != 0:
        raise ValueError("oracle_screen rejected its arguments")
    return bits


def screen_full(img, templates, probes, feat_mask: int, P, Q: int, lib=None) -> np.ndarray:
    """bits[n_tmpl, H, W] over every position of the image."""
    a = _img16(img)
    H, W = a.shape
    ys, xs = np.meshgrid(np.arange(H, dtype=np.int32), np.arange(W, dtype=np.int32),
                         indexing="ij")
    bits = screen_positions(a, templates, probes, feat_mask, P, Q, xs.ravel(), ys.ravel(), lib)
    return bits.reshape(len(templates), H, W)


def ring_radii(r: int, n_rings: int, lib=None) -> list:
    """r, s(r), s(s(r)), ...: the radii of the n_rings concentric central
    stars, each a factor sqrt 2 smaller (rounded as the square half-width)."""
    out = [int(r)]
    for _ in range(n_rings - 1):
        out.append(square_half(out[-1], lib))
    return out


def template_ring_features(tmpl, rho: int, n_rings: int, lib=None):
    """([n_rings][3] features, [n_rings] radii) of the template's central
    stars of radii rho, s(rho), s(s(rho)), ..."""
    radii = ring_radii(rho, n_rings, lib)
    return np.stack([template_features(tmpl, rj, lib) for rj in radii]), radii


def screen_rings_positions(img, templates, probes, feat_mask: int, P, Q: int, n_rings: int,
                           xs, ys, lib=None, G=None) -> np.ndarray:
    """bits[n_tmpl, n] of the multi-central-area screen: probe (t, k, r)
    passes where the stars of radii r, s(r), ... all match the template's
    central stars of radii rho, s(rho), ...  (n_rings of them)."""
    lib = lib or load()
    a = _img16(img)
    H, W = a.shape
    if G is None:
        G = gradient(a, lib)
    FT = np.zeros((len(templates), n_rings, 3), np.int64)
    rho = np.zeros((len(templates), n_rings), np.int32)
    for t, (px, r0) in enumerate(templates):
        FT[t], rho[t] = template_ring_features(px, r0, n_rings, lib)
    parr = np.ascontiguousarray(np.array(sorted(probes), np.int32).reshape(-1, 3))
    xs = np.ascontiguousarray(xs, np.int32)
    ys = np.ascontiguousarray(ys, np.int32)
    bits = np.zeros((len(templates), len(xs)), np.uint32)
    Pa = np.ascontiguousarray(list(P) + [0] * (3 - len(P)), np.int32)
    rc = lib.oracle_screen_rings(a, np.ascontiguousarray(G, np.int32), H, W, W, xs, ys, len(xs),
                                 parr, len(parr), np.ascontiguousarray(FT), rho, len(templates),
                                 int(n_rings), int(feat_mask), Pa, int(Q), bits)
    if rc != 0:
        raise ValueError("oracle_screen_rings rejected its arguments")
    return bits


def screen_rings_full(img, templates, probes, feat_mask: int, P, Q: int, n_rings: int,
                      lib=None) -> np.ndarray:
    """bits[n_tmpl, H, W] of the multi-central-area screen."""
    a = _img16(img)
    H, W = a.shape
    ys, xs = np.meshgrid(np.arange(H, dtype=np.int32), np.arange(W, dtype=np.int32),
                         indexing="ij")
    bits = screen_rings_positions(a, templates, probes, feat_mask, P, Q, n_rings, xs.ravel(),
                                  ys.ravel(), lib)
    return bits.reshape(len(templates), H, W)


def star_support(r: int, lib=None) -> np.ndarray:
    """[2r+1, 2r+1] bool: the pixels the radius-r star covers (weight > 0)."""
    lib = lib or load()
    return np.array([[lib.oracle_star_weight(dx, dy, r) > 0 for dx in range(-r, r + 1)]
                     for dy in range(-r, r + 1)], bool)


def region_full(H: int, W: int, n_tmpl: int, cands, radius_of: dict, lib=None) -> np.ndarray:
    """Preserved region [n_tmpl, H, W] (uint8): the union, over every
    candidate (t, y, x, scale_bits) and every scale bit k it carries, of the
    pixels covered by the star of radius radius_of[(t, k)] centred on it
    (Sec. "Experimental Results", Exp. I: the regions the pre-processor
    preserves, whose complement is the pruned region)."""
    lib = lib or load()
    out = np.zeros((n_tmpl, H, W), np.uint8)
    sup = {}
    for t, y, x, bits in np.asarray(cands, np.int64).reshape(-1, 4):
        for k in range(32):
            if not (int(bits) >> k) & 1:
                continue
            r = radius_of[(int(t), k)]
            if r not in sup:
                sup[r] = star_support(r, lib)
            out[t, y - r:y + r + 1, x - r:x + r + 1] |= sup[r]
    return out


def mask_and_list(bits: np.ndarray):
    """Candidate mask (uint8, 1 = survives at some scale) and the candidate
    list as an [n, 4] int64 array of (t, y, x, scale_bits) in (t, y, x) order."""
    mask = (bits != 0).astype(np.uint8)
    t, y, x = np.nonzero(bits)
    lst = np.stack([t, y, x, bits[t, y, x].astype(np.int64)], axis=1).astype(np.int64)
    return mask, lst
