"""Helpers for the GPU tests: numpy definitions of the integral tables and a
runner that screens a synthetic workload through the C ABI."""
from __future__ import annotations

import sys

import numpy as np

import oracle.core as oc


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def quantities(img: np.ndarray, fm: int):
    """q arrays in feature-bit order: I, I^2, G (G from the pinned oracle)."""
    a = img.astype(np.int64)
    out = []
    if fm & 1:
        out.append(a)
    if fm & 2:
        out.append(a * a)
    if fm & 4:
        out.append(oc.gradient(img).astype(np.int64))
    H, W = img.shape
    yy, xx = np.mgrid[0:H, 0:W]
    if fm & 8:
        out.append(xx.astype(np.int64) * a)   # first-moment quantity i I
    if fm & 16:
        out.append(yy.astype(np.int64) * a)   # j I
    return out


def tables_numpy(img: np.ndarray, fm: int):
    """(L, R, R') as [H+1, W+1, nq] int64 for x, y in [-1, W-1] x [-1, H-1],
    straight from the definitions through row prefix sums P_j:
      L(x,y)  = sum_{i<=x, j<=y} q
      R(x,y)  = sum_{j<=y} P_j(x+(y-j)) - P_j(x-(y-j)-1)
      R'(x,y) = sum_{j<=y} P_j(x+1+(y-j)) - P_j(x-(y-j)-1)
    with P_j(c) clamped (0 left of the image, the row total right of it)."""
    H, W = img.shape
    qs = quantities(img, fm)
    nq = len(qs)
    L = np.zeros((H + 1, W + 1, nq), np.int64)
    R = np.zeros_like(L)
    Rp = np.zeros_like(L)
    xs = np.arange(-1, W)
    for qi, q in enumerate(qs):
        L[1:, 1:, qi] = np.cumsum(np.cumsum(q, 0), 1)
        pre = np.zeros((H, W + 1), np.int64)
        pre[:, 1:] = np.cumsum(q, 1)          # P_j(c) = pre[j, clip(c,-1,W-1)+1]

        def P(rows, cols):
            return pre[rows, np.clip(cols, -1, W - 1) + 1]
        for y in range(H):
            js = np.arange(y + 1)[:, None]
            d = y - js
            R[y + 1, :, qi] = (P(js, xs[None, :] + d) - P(js, xs[None, :] - d - 1)).sum(0)
            Rp[y + 1, :, qi] = (P(js, xs[None, :] + 1 + d) - P(js, xs[None, :] - d - 1)).sum(0)
    return L, R, Rp


def bits_from_list(cands: np.ndarray, T: int, H: int, W: int) -> np.ndarray:
    bits = np.zeros((T, H, W), np.uint32)
    if len(cands):
        bits[cands[:, 0], cands[:, 1], cands[:, 2]] = cands[:, 3].astype(np.uint32)
    return bits


class Runner:
    """Screens workloads through the library on cuda:0."""

    def __init__(self):
        import torch
        from paper_1707_05647_amd import _lib as L
        from paper_1707_05647_amd.screen import Context
        self.torch = torch
        self.L = L
        self.dev = torch.device("cuda", 0)
        self.ctx = Context(0)

    def screen(self, img: np.ndarray, templates, probes, fm: int, P, Q: int, *,
               bit_depth=None, list_cap=None, pitch_pad: int = 0, tm_fm=None,
               max_radius: int = -1, batched: bool = False):
        torch = self.torch
        if pitch_pad:
            wide = np.zeros((img.shape[0], img.shape[1] + pitch_pad), img.dtype)
            wide[:, :img.shape[1]] = img
            t_img = self.L.device_image(wide, self.dev)[:, :img.shape[1]]
        else:
            t_img = self.L.device_image(img, self.dev)
        if bit_depth is None:
            bit_depth = 8 if img.dtype == np.uint8 else 16
        ref = self.ctx.reference(t_img, fm, bit_depth, max_radius=max_radius)
        self.last_value_bits = ref.value_bits
        self.last_entry_bytes = ref.entry_bytes
        self.last_slots = ref.slots
        self.last_plane_bytes = ref.plane_bytes
        tm = [self.L.oss_template_features(px, rho, tm_fm or fm, bit_depth=bit_depth)
              for px, rho in templates]
        H, W = img.shape
        cap = list_cap if list_cap is not None else len(templates) * H * W
        res = self.ctx.screen(ref, tm, probes, (*P, Q), fm, list_cap=cap, batched=batched)
        torch.cuda.synchronize()
        mask, cands, n = res.host()
        ref.release()
        return mask, cands, n

    def close(self):
        self.ctx.close()
