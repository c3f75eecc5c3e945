"""Seeded reference images and template cuts.

The reference image recipe follows the synthetic stand-in for the paper's
natural-image test sets (Sec. "Exp. I: Image Matching"): a flat grey base,
a few hundred Gaussian blobs per 512x512 area and uniform noise, rounded to
integers and clipped to the pixel range.  Templates are cut from the
reference around a seeded centre, either exactly, by an exact quarter turn
or transpose, or by bilinear resampling after a rotation and a scale
(the paper extracts its templates at random locations with random
rotations and scales, Sec. "Exp. I").  A template is rejected when its
standard deviation is below a threshold, as the paper requires of its test
templates.

Everything here is input generation; none of it is screening arithmetic.
"""
from __future__ import annotations

import math

import numpy as np


def make_rng(cfg_id: int, seed: int) -> np.random.Generator:
    """Counter-free seeded generator: one stream per (workload id, seed)."""
    return np.random.default_rng(np.random.SeedSequence([int(cfg_id), int(seed)]))


def _round_clip(v: np.ndarray, hi: int, dtype) -> np.ndarray:
    out = np.floor(v + 0.5)
    np.clip(out, 0, hi, out=out)
    return out.astype(dtype)


def blob_image(H: int, W: int, rng: np.random.Generator, *, depth: int = 8,
               blobs_per_512sq: float = 200.0, n_blobs: int | None = None,
               base: float = 128.0, amp: float = 80.0, sig_lo: float = 4.0,
               sig_hi: float = 64.0, noise: float = 8.0, device=None,
               render: bool = True) -> np.ndarray | None:
    """Base + Gaussian blobs + iid uniform noise, rounded and clipped.

    * ``n_blobs`` defaults to ``blobs_per_512sq`` per 512x512 of area.
    * Each blob has amplitude U[-amp, amp], sigma U[sig_lo, sig_hi] px and a
      centre uniform over the image; it is truncated at 4 sigma (below half
      a grey level).
    * Noise is real-valued U[-noise, noise].
    * depth 8 -> uint8 ``floor(v+1/2)`` clipped to [0, 255];
      depth 12 -> uint16 ``floor(16 v + 1/2)`` clipped to [0, 4095].

    ``device`` (a torch device) renders the same blob parameters there in
    float64 (fast for very large images); the noise then comes from a torch
    generator seeded from ``rng``, so the image is a deterministic function
    of the seed but not bit-identical to the host rendering.  The result is
    returned as a host array either way.  With ``render=False`` (device
    rendering only) the same numbers are drawn from ``rng`` and nothing is
    rendered (None is returned): the generator is left exactly where a
    rendering would leave it, for callers that hold the image already.
    """
    if device is not None:
        return _blob_image_torch(H, W, rng, depth, blobs_per_512sq, n_blobs, base, amp, sig_lo,
                                 sig_hi, noise, device, render)
    if not render:
        raise ValueError("render=False needs device rendering (its noise is one seed)")
    if n_blobs is None:
        n_blobs = max(1, int(round(blobs_per_512sq * H * W / (512.0 * 512.0))))
    img = np.full((H, W), base, dtype=np.float64)
    amps = rng.uniform(-amp, amp, n_blobs)
    sigs = rng.uniform(sig_lo, sig_hi, n_blobs)
    cxs = rng.uniform(0.0, W, n_blobs)
    cys = rng.uniform(0.0, H, n_blobs)
    for a, sg, cx, cy in zip(amps, sigs, cxs, cys):
        rad = 4.0 * sg
        x0 = max(0, int(math.floor(cx - rad)))
        x1 = min(W, int(math.ceil(cx + rad)) + 1)
        y0 = max(0, int(math.floor(cy - rad)))
        y1 = min(H, int(math.ceil(cy + rad)) + 1)
        if x0 >= x1 or y0 >= y1:
            continue
        inv = -0.5 / (sg * sg)
        gx = np.exp(inv * (np.arange(x0, x1, dtype=np.float64) - cx) ** 2)
        gy = np.exp(inv * (np.arange(y0, y1, dtype=np.float64) - cy) ** 2)
        img[y0:y1, x0:x1] += np.outer(a * gy, gx)
    img += rng.uniform(-noise, noise, (H, W))
    if depth == 8:
        return _round_clip(img, 255, np.uint8)
    if depth == 12:
        return _round_clip(16.0 * img, 4095, np.uint16)
    raise ValueError(f"unsupported depth {depth}")


def _blob_image_torch(H, W, rng, depth, blobs_per_512sq, n_blobs, base, amp, sig_lo, sig_hi,
                      noise, device, render=True):
    if n_blobs is None:
        n_blobs = max(1, int(round(blobs_per_512sq * H * W / (512.0 * 512.0))))
    amps = rng.uniform(-amp, amp, n_blobs)
    sigs = rng.uniform(sig_lo, sig_hi, n_blobs)
    cxs = rng.uniform(0.0, W, n_blobs)
    cys = rng.uniform(0.0, H, n_blobs)
    nseed = int(rng.integers(0, 2 ** 62))
    if not render:
        return None
    import torch
    img = torch.full((H, W), base, dtype=torch.float64, device=device)
    xs_all = torch.arange(W, dtype=torch.float64, device=device)
    ys_all = torch.arange(H, dtype=torch.float64, device=device)
    for a, sg, cx, cy in zip(amps, sigs, cxs, cys):
        rad = 4.0 * sg
        x0 = max(0, int(math.floor(cx - rad)))
        x1 = min(W, int(math.ceil(cx + rad)) + 1)
        y0 = max(0, int(math.floor(cy - rad)))
        y1 = min(H, int(math.ceil(cy + rad)) + 1)
        if x0 >= x1 or y0 >= y1:
            continue
        inv = -0.5 / (sg * sg)
        gx = torch.exp(inv * (xs_all[x0:x1] - cx) ** 2)
        gy = torch.exp(inv * (ys_all[y0:y1] - cy) ** 2) * a
        img[y0:y1, x0:x1] += gy[:, None] * gx[None, :]
    gen = torch.Generator(device=device)
    gen.manual_seed(nseed)
    img += (torch.rand((H, W), dtype=torch.float64, device=device, generator=gen) * 2 - 1) * noise
    if depth == 8:
        out = torch.clamp(torch.floor(img + 0.5), 0, 255).to(torch.uint8)
        return out.cpu().numpy()
    if depth == 12:
        out = torch.clamp(torch.floor(16.0 * img + 0.5), 0, 4095).to(torch.int16)
        return out.cpu().numpy().view(np.uint16)
    raise ValueError(f"unsupported depth {depth}")


def patch_std(img: np.ndarray, cx: int, cy: int, half: int) -> float:
    p = img[cy - half:cy + half + 1, cx - half:cx + half + 1].astype(np.float64)
    return float(p.std())


def pick_centre(rng: np.random.Generator, img: np.ndarray, margin: int, *,
                std_half: int, std_min: float, tries: int = 1000) -> tuple[int, int]:
    """Uniform integer centre at least ``margin`` px from every border whose
    (2*std_half+1)^2 neighbourhood has a standard deviation >= std_min.
    Rejected draws are retried deterministically from the same stream."""
    H, W = img.shape
    if 2 * margin >= min(H, W):
        raise ValueError("margin too large for the image")
    for _ in range(tries):
        cx = int(rng.integers(margin, W - margin))
        cy = int(rng.integers(margin, H - margin))
        if patch_std(img, cx, cy, std_half) >= std_min:
            return cx, cy
    raise RuntimeError("no textured centre found")


def cut_patch(img: np.ndarray, cx: int, cy: int, half: int, quarter_turns: int = 0,
              transpose: bool = False, flip: bool = False) -> np.ndarray:
    """Exact (2*half+1)^2 cut centred on (cx, cy), optionally turned by a
    multiple of 90 degrees, transposed or mirrored (all exact)."""
    p = img[cy - half:cy + half + 1, cx - half:cx + half + 1].copy()
    if p.shape != (2 * half + 1, 2 * half + 1):
        raise ValueError("cut leaves the image")
    if transpose:
        p = p.T.copy()
    if flip:
        p = p[:, ::-1].copy()
    if quarter_turns % 4:
        p = np.rot90(p, quarter_turns % 4).copy()
    return p


def rotate_scale_patch(img: np.ndarray, cx: float, cy: float, theta_deg: float,
                       scale: float, half: int, hi: int) -> np.ndarray:
    """Template of size (2*half+1)^2 whose pixel at offset (u, v) from its
    centre samples the reference at (cx, cy) + Rot(theta) (u, v) / scale by
    bilinear interpolation, then rounds and clips to [0, hi].

    ``scale`` > 1 magnifies: the reference object of radius R appears in the
    template with radius about R * scale.  Quarter turns at unit scale are
    cut exactly instead of resampled."""
    if scale == 1.0 and float(theta_deg) % 90.0 == 0.0:
        return cut_patch(img, int(cx), int(cy), half, int(round(theta_deg / 90.0)))
    H, W = img.shape
    t = math.radians(theta_deg)
    c, s = math.cos(t), math.sin(t)
    off = np.arange(-half, half + 1, dtype=np.float64)
    u, v = np.meshgrid(off, off)  # u: column offset, v: row offset
    xs = cx + (c * u - s * v) / scale
    ys = cy + (s * u + c * v) / scale
    if xs.min() < 0 or ys.min() < 0 or xs.max() > W - 1 or ys.max() > H - 1:
        raise ValueError("resampled template leaves the image")
    x0 = np.floor(xs).astype(np.int64)
    y0 = np.floor(ys).astype(np.int64)
    x0 = np.minimum(x0, W - 2)
    y0 = np.minimum(y0, H - 2)
    fx = xs - x0
    fy = ys - y0
    f = img.astype(np.float64)
    v00 = f[y0, x0]
    v01 = f[y0, x0 + 1]
    v10 = f[y0 + 1, x0]
    v11 = f[y0 + 1, x0 + 1]
    val = (v00 * (1 - fx) * (1 - fy) + v01 * fx * (1 - fy)
           + v10 * (1 - fx) * fy + v11 * fx * fy)
    return _round_clip(val, hi, img.dtype)
