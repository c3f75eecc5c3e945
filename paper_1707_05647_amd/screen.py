"""Convenience layer over the C ABI: owns the handles and the torch output
tensors.  All computation happens in liboss.so."""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import _lib as L


@dataclass
class ScreenResult:
    mask: "object"        # torch uint8 [T, H, W] on the device
    cands: "object"       # torch int32 [cap, 4] (t, y, x, scale_bits as int32)
    count: "object"       # torch int64 [1] on the device

    def host(self):
        """(mask ndarray, candidate ndarray [n, 4] int64, total count)."""
        n = int(self.count.item())
        c = self.cands[:min(n, self.cands.shape[0])].cpu().numpy().astype(np.int64)
        if len(c):
            c[:, 3] &= 0xFFFFFFFF
        return self.mask.cpu().numpy(), c, n


class Reference:
    """Integral tables of one device-resident reference image."""

    def __init__(self, ctx: "Context", image, feat_mask: int, bit_depth: int | None = None,
                 stream=None, build: bool = True, max_radius: int = -1):
        self.ctx = ctx
        self.image = image
        self.desc = L.desc_of(image, bit_depth)
        self.feat_mask = int(feat_mask)
        self.handle = L.oss_ref_create(ctx.handle, self.desc, self.feat_mask, max_radius)
        info = L.oss_ref_tables(self.handle)
        self.value_bits, self.max_radius = info[5], info[6]
        # per quantity slot: where its (low) value and its high part sit
        self.layout, self.plane_bytes = L.oss_ref_layout_q(self.handle)
        # (offset, stored width in bits) per slot; values narrower than 64
        # bits are the sums modulo 2^width
        self.slots = [(o, b + hb) for o, _, b, _, _, hb in self.layout]
        self.entry_bytes = self.layout[0][1] if self.layout else 0  # first slot's stride
        # bytes one table entry takes over all planes
        self.stored_entry_bytes = sum((b + hb) // 8 for _, _, b, _, _, hb in self.layout)
        if build:
            self.build(stream)

    @property
    def H(self):
        return self.desc.H

    @property
    def W(self):
        return self.desc.W

    def build(self, stream=None, image=None):
        if image is not None:
            self.image = image
        L.oss_ref_build(self.handle, self.image, stream)

    def release(self):
        if self.handle:
            L.oss_ref_release(self.handle)
            self.handle = None

    def tables_host(self):
        """Copy (L, R, R') to host int64 arrays [H+1, W+1, nq]: each slot's
        stored value (``self.slots[q][1]`` bits wide: the sums modulo
        2^width, zero-extended; 64 = exact); synchronous; for tests and
        inspection."""
        Lp, Rp_, Rpp, pitch, nq, vb, _ = L.oss_ref_tables(self.handle)
        H1 = self.H + 1
        n = H1 * pitch
        # the byte span of one table: every quantity's low and high parts
        parts = []
        for off, st, b, hoff, hst, hb in self.layout:
            parts.append((off, st, b // 8))
            if hb:
                parts.append((hoff, hst, hb // 8))
        span = max(o + (n - 1) * st + nb for o, st, nb in parts)
        out = []
        for p in (Lp, Rp_, Rpp):
            raw = np.zeros(span + 8, np.uint8)
            _hip_memcpy_d2h(raw[:span], p)

            def values(off, st, nb):
                idx = off + np.arange(n, dtype=np.int64).reshape(H1, pitch)[:, :self.W + 1] * st
                v = np.zeros(idx.shape, np.uint64)
                for k in range(nb):  # little-endian bytes
                    v |= raw[idx + k].astype(np.uint64) << np.uint64(8 * k)
                return v
            t = np.empty((H1, self.W + 1, nq), np.int64)
            for q, (off, st, b, hoff, hst, hb) in enumerate(self.layout):
                v = values(off, st, b // 8)
                if hb:
                    v |= values(hoff, hst, hb // 8) << np.uint64(b)
                t[..., q] = v.view(np.int64)
            out.append(t)
        return out


class Context:
    def __init__(self, device: int = 0):
        self.device = device
        self.handle = L.oss_ctx_create(device)

    def reference(self, image, feat_mask: int = L.OSS_F_ALL, bit_depth: int | None = None,
                  stream=None, build: bool = True, max_radius: int = -1) -> Reference:
        return Reference(self, image, feat_mask, bit_depth, stream, build, max_radius)

    def template_features(self, pixels, rho: int, feat_mask: int, bit_depth: int | None = None):
        return L.oss_template_features(pixels, rho, feat_mask, bit_depth)

    def screen(self, ref: Reference, templates, probes, tol, feat_mask: int,
               list_cap: int | None = None, stream=None, out: ScreenResult | None = None,
               with_mask: bool = True, batched: bool = False) -> ScreenResult:
        """templates: list of oss_template_feat; probes: (t, k, r) triples;
        tol: (P0, P1, P2, Q)."""
        import torch
        dev = torch.device("cuda", self.device)
        T = len(templates)
        if out is None:
            cap = list_cap if list_cap is not None else max(1024, T * ref.H * ref.W // 50)
            mask = (torch.empty((T, ref.H, ref.W), dtype=torch.uint8, device=dev)
                    if with_mask else None)
            cands = torch.empty((max(cap, 1), 4), dtype=torch.int32, device=dev)
            count = torch.zeros(1, dtype=torch.int64, device=dev)
            out = ScreenResult(mask, cands, count)
        cap = out.cands.shape[0] if list_cap is None else list_cap
        L.oss_screen(self.handle, ref.handle, templates, probes, tol, feat_mask, out.mask,
                     out.cands, cap, out.count, stream, batched=batched)
        return out

    def close(self):
        if self.handle:
            L.oss_ctx_destroy(self.handle)
            self.handle = None


_hip = None


def _hip_memcpy_d2h(dst: np.ndarray, src_ptr: int):
    """hipMemcpy device -> host of dst.nbytes bytes (blocking)."""
    global _hip
    import ctypes as C
    if _hip is None:
        import torch  # noqa: F401  (binds to torch's runtime by soname)
        _hip = C.CDLL("libamdhip64.so.7")
        _hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        _hip.hipMemcpy.restype = C.c_int
        _hip.hipDeviceSynchronize.restype = C.c_int
    if _hip.hipDeviceSynchronize() != 0:
        raise RuntimeError("hipDeviceSynchronize failed")
    rc = _hip.hipMemcpy(dst.ctypes.data, src_ptr, dst.nbytes, 2)  # hipMemcpyDeviceToHost
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed ({rc})")


class Server:
    """Serving loop over the C ABI (oss_server_*): queued requests, admission
    by device-memory footprint, resident-reference cache, merged launches."""

    def __init__(self, device: int = 0, memory_budget: int = 64 << 30, lanes: int = 2,
                 max_batch_templates: int = 64, queue_timeout_ns: int = 0):
        self.handle = L.oss_server_create(device, memory_budget, lanes, max_batch_templates,
                                          queue_timeout_ns)
        self._pixels = {}  # request id -> device pixels kept alive until release

    def submit(self, ref_key: int, pixels, templates, probes, tol, feat_mask: int,
               list_cap: int, bit_depth: int | None = None, arrival_ns: int = 0) -> int:
        rid = L.oss_server_submit(self.handle, ref_key, pixels, templates, probes, tol, feat_mask,
                                  list_cap, bit_depth, arrival_ns)
        self._pixels[rid] = pixels
        return rid

    def pump(self, wait_us: int = 0) -> int:
        return L.oss_server_pump(self.handle, wait_us)

    def drain(self):
        L.oss_server_drain(self.handle)

    def result(self, rid: int):
        return L.oss_server_result(self.handle, rid)

    def host_result(self, rid: int):
        """(mask ndarray [T, H, W], candidates [n, 4] int64, total count) of a
        completed request (synchronous copies)."""
        r = self.result(rid)
        if r.status != L.OSS_OK:
            raise L.OssError(r.status, f"request {rid}")
        mask = np.empty((r.n_tmpl, r.H, r.W), np.uint8)
        _hip_memcpy_d2h(mask, r.dev_mask)
        n = min(r.count, r.list_cap)
        c = np.empty((n, 4), np.int32)
        if n:
            _hip_memcpy_d2h(c, r.dev_list)
        c = c.astype(np.int64)
        if n:
            c[:, 3] &= 0xFFFFFFFF
        return mask, c, r.count

    def cancel(self, rid: int):
        """Cancel a queued request (it completes with OSS_E_CANCELLED)."""
        L.oss_server_cancel(self.handle, rid)

    def release(self, rid: int):
        L.oss_server_release(self.handle, rid)
        self._pixels.pop(rid, None)

    def stats(self) -> dict:
        return L.oss_server_stats_read(self.handle)

    def close(self):
        if self.handle:
            L.oss_server_destroy(self.handle)
            self.handle = None
            self._pixels.clear()
