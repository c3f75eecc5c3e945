"""Algorithm 1 taken literally: the scale-invariant screening pre-processor
with quantised feature-set membership (Sec. "Scale Invariance",
Algorithm 1, Eq. F_n).

TEST INFRASTRUCTURE.  Only the test suite and the benchmark's CPU baseline
use this module; the product path never imports it.

Steps, in the paper's order:
  * lambda = sqrt 2, n = template width; scale bands m_b = beta n / lambda^(b+1)
    for b = 0 .. B-1 with B = ceil(log_lambda(beta / alpha)) (reading of the
    paper's loop, whose literal form runs one band more than its text
    states);
  * for every integer size k with ceil(m_b) <= k <= floor(lambda m_b): the
    template resized to k x k (bilinear, pixel centres aligned, edge pixels
    replicated, rounded half up, all in exact integer arithmetic), its
    central m x m crop with m = ceil(m_b), and the features of that crop:
    the star of radius (m-1)//2 at the crop's centre pixel, gradients taken
    on the resized template;
  * the quantiser Q(f) = floor(f / q + 1/2) per feature, q = the per-pixel
    quantisation step times the star's weighted area A(r), and the
    membership array: Q(f - q/2), Q(f) and Q(f + q/2) are marked, per
    feature, for every crop feature vector (all combinations across
    features);
  * every reference position whose radius-r star fits is a candidate of
    band b when the quantised features of its star are marked.
The membership array is a Python set of marked cells, looked up per
position; no interval arithmetic is used here.
"""
from __future__ import annotations

import itertools
from fractions import Fraction
from math import floor, isqrt

import numpy as np

from . import core as oc


def band_count(alpha: Fraction, beta: Fraction) -> int:
    """Smallest B with lambda^B >= beta / alpha (lambda = sqrt 2), i.e.
    2^B >= (beta / alpha)^2."""
    ratio2 = (Fraction(beta) / Fraction(alpha)) ** 2
    B = 0
    while Fraction(2) ** B < ratio2:
        B += 1
    return B


def _floor_over_sqrt2_pow(v: Fraction, e: int) -> int:
    """floor(v / sqrt2^e) for rational v >= 0, exactly."""
    v = Fraction(v)
    if e % 2 == 0:
        return floor(v / 2 ** (e // 2))
    # v / sqrt2^e = sqrt(2 a^2) / (d 2^((e+1)/2)) with v = a / d
    a, d = v.numerator, v.denominator
    return isqrt(2 * a * a) // (d * 2 ** ((e + 1) // 2))


def _ceil_over_sqrt2_pow(v: Fraction, e: int) -> int:
    v = Fraction(v)
    if e % 2 == 0:
        q = v / 2 ** (e // 2)
        return -floor(-q)
    if v == 0:
        return 0
    return _floor_over_sqrt2_pow(v, e) + 1  # an irrational value is never an integer


def bands(n: int, alpha, beta):
    """[(m, k_lo, k_hi)] per band: m = ceil(m_b) is the patch size, the
    template sizes are k_lo..k_hi."""
    alpha, beta = Fraction(alpha), Fraction(beta)
    v = beta * n
    out = []
    for b in range(band_count(alpha, beta)):
        k_lo = _ceil_over_sqrt2_pow(v, b + 1)
        k_hi = _floor_over_sqrt2_pow(v, b)
        out.append((k_lo, k_lo, k_hi))
    return out


def resize(img: np.ndarray, k: int) -> np.ndarray:
    """Bilinear resize of a square n x n image to k x k: destination pixel i
    samples source coordinate (i + 1/2) n / k - 1/2, edges replicated, the
    result rounded half up.  Exact integers: weights in units of 1/(2k)."""
    a = np.asarray(img).astype(np.int64)
    n = a.shape[0]
    assert a.shape == (n, n)

    def axis():
        idx0 = np.zeros(k, np.int64)
        idx1 = np.zeros(k, np.int64)
        w = np.zeros(k, np.int64)
        for i in range(k):
            num = (2 * i + 1) * n - k  # source coordinate times 2k
            if num < 0:
                x0, wx = 0, 0
            else:
                x0, wx = num // (2 * k), num % (2 * k)
            if x0 >= n - 1:
                x0, wx = n - 1, 0
            idx0[i], idx1[i], w[i] = x0, min(x0 + 1, n - 1), wx
        return idx0, idx1, w

    i0, i1, w = axis()
    D = 2 * k
    top = (D - w)[None, :] * a[:, i0] + w[None, :] * a[:, i1]        # rows of the source
    val = (D - w)[:, None] * top[i0, :] + w[:, None] * top[i1, :]     # over (2k)^2
    den = D * D
    return ((2 * val + den) // (2 * den)).astype(a.dtype)


def crop_features(tmpl: np.ndarray, k: int, m: int, lib=None):
    """Features of the central m x m crop of the k x k resized template: the
    star of radius (m-1)//2 at the crop's centre pixel (gradient of the
    resized template)."""
    Y = resize(tmpl, k).astype(np.uint16)
    off = (k - m) // 2
    c = off + (m - 1) // 2
    r = (m - 1) // 2
    return oc.star_features(Y, [c], [c], r, lib)[0], r


def quantise(f, q) -> int:
    """Q(f) = floor(f / q + 1/2) for rational f."""
    return floor(Fraction(f) / q + Fraction(1, 2))


def membership(tmpl: np.ndarray, alpha, beta, qbar, feat_mask: int, lib=None):
    """Per band: (star radius r, quantisation steps q[3], set of marked
    cells (tuples over the enabled features))."""
    n = tmpl.shape[1]
    feats = [f for f in range(3) if feat_mask & (1 << f)]
    out = []
    for m, k_lo, k_hi in bands(n, alpha, beta):
        r = (m - 1) // 2
        A = oc.star_area(r, lib)
        q = [qbar[f] * A for f in range(3)]
        marked = set()
        for k in range(k_lo, k_hi + 1):
            F, _ = crop_features(tmpl, k, m, lib)
            cells = []
            for f in feats:
                h = Fraction(q[f], 2)
                cells.append(sorted({quantise(F[f] - h, q[f]), quantise(F[f], q[f]),
                                     quantise(F[f] + h, q[f])}))
            marked.update(itertools.product(*cells))
        out.append((r, q, marked))
    return out


def screen(img, templates, alpha, beta, qbar, feat_mask: int, lib=None) -> np.ndarray:
    """bits[n_tmpl, H, W]: bit b set where the band-b star of the position
    fits and its quantised features are marked for that template."""
    a = np.asarray(img)
    H, W = a.shape
    ys, xs = np.meshgrid(np.arange(H, dtype=np.int32), np.arange(W, dtype=np.int32),
                         indexing="ij")
    xs, ys = xs.ravel(), ys.ravel()
    feats = [f for f in range(3) if feat_mask & (1 << f)]
    bits = np.zeros((len(templates), H * W), np.uint32)
    G = oc.gradient(a, lib)
    cache = {}
    for t, tmpl in enumerate(templates):
        for b, (r, q, marked) in enumerate(membership(tmpl, alpha, beta, qbar, feat_mask, lib)):
            if r not in cache:
                cache[r] = oc.star_features(a, xs, ys, r, lib, G=G)
            F = cache[r]
            for i in range(H * W):
                if F[i, 0] < 0:
                    continue
                key = tuple(quantise(int(F[i, f]), q[f]) for f in feats)
                if key in marked:
                    bits[t, i] |= 1 << b
    return bits.reshape(len(templates), H, W)
