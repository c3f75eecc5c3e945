"""ctypes binding of liboss.so (include/oss.h): argument marshalling only.

Every function here has the name of the C entry point it calls.  Device
buffers are torch tensors (only their data pointers cross the boundary);
streams are torch streams or raw hipStream_t integers.  Nothing is computed
in Python: a missing library is an error, never a fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboss.so")

OSS_OK, OSS_E_ARG, OSS_E_NOMEM, OSS_E_OVERFLOW, OSS_E_DEVICE, OSS_E_STATE = 0, -1, -2, -3, -4, -5
OSS_E_LIMIT, OSS_E_CANCELLED, OSS_E_TIMEOUT = -6, -7, -8
OSS_U8, OSS_U16 = 0, 1
OSS_F_SUM, OSS_F_SQ, OSS_F_GRAD, OSS_F_ALL = 1, 2, 4, 7
OSS_F_XMOM, OSS_F_YMOM, OSS_F_MOMENTS = 8, 16, 24
OSS_MAX_QUANTITIES = 5
OSS_T_MEAN, OSS_T_VAR, OSS_T_MAG = 1, 2, 4
OSS_MAX_SCALES = 32
OSS_NOALLOC_SCRATCH_BYTES = 160 << 20

EXPORTED = [
    "oss_ctx_create", "oss_ctx_destroy", "oss_status_string", "oss_ref_bytes", "oss_ref_create",
    "oss_ref_build", "oss_ref_release", "oss_ref_tables", "oss_template_features",
    "oss_feature_bounds", "oss_screen", "oss_ctx_profile", "oss_ctx_profile_read",
    "oss_ctx_set_option", "oss_ctx_get_option", "oss_screen_batched", "oss_autotune_batched",
    "oss_ref_layout", "oss_region", "oss_template_moments", "oss_screen_moments", "oss_screen_intervals", "oss_alg1_probes", "oss_template_features_rings", "oss_screen_rings", "oss_server_create", "oss_server_destroy", "oss_server_submit", "oss_server_pump",
    "oss_server_drain", "oss_server_result", "oss_server_release", "oss_server_stats_read",
    "oss_screen_noalloc", "oss_server_cancel", "oss_ref_layout_q",
]
OSS_OPT_STAR_STRIP, OSS_OPT_STAR_BLOCKS_PER_XCD, OSS_OPT_STAR_LDS, OSS_OPT_BATCH_BUCKET = 1, 2, 3, 4
OSS_OPT_TABLE_PLANAR = 5
OSS_OPT_STAR_PIPE = 6
OSS_OPT_STAR_STAGED = 7
OSS_OPT_TABLE_REC = 9
OSS_OPT_BUILD_STREAM = 8
OSS_MAX_RINGS = 4
OSS_TUNE_MAX = 64


class oss_image_desc(C.Structure):
    _fields_ = [("H", C.c_int32), ("W", C.c_int32), ("pitch_bytes", C.c_int64),
                ("dtype", C.c_int32), ("bit_depth", C.c_int32)]


class oss_template_feat(C.Structure):
    _fields_ = [("F", C.c_int64 * 3), ("rho", C.c_int32), ("feat_mask", C.c_uint32)]


class oss_probe(C.Structure):
    _fields_ = [("template_id", C.c_int32), ("scale_id", C.c_int32), ("r", C.c_int32)]


class oss_tolerance(C.Structure):
    _fields_ = [("P", C.c_int32 * 3), ("Q", C.c_int32)]


class oss_quantity_layout(C.Structure):
    _fields_ = [("offset", C.c_int64), ("stride", C.c_int32), ("bits", C.c_int32),
                ("hi_offset", C.c_int64), ("hi_stride", C.c_int32), ("hi_bits", C.c_int32)]


class oss_candidate(C.Structure):
    _fields_ = [("t", C.c_int32), ("y", C.c_int32), ("x", C.c_int32), ("scale_bits", C.c_uint32)]


class oss_kernel_stat(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int64), ("total_ms", C.c_double),
                ("max_ms", C.c_double)]


class oss_tune_result(C.Structure):
    _fields_ = [("strip", C.c_int32), ("blocks_per_xcd", C.c_int32), ("bucket_radii", C.c_int32),
                ("ms", C.c_float), ("n_tried", C.c_int32),
                ("tried", (C.c_int32 * 3) * OSS_TUNE_MAX), ("tried_ms", C.c_float * OSS_TUNE_MAX)]


class oss_interval_probe(C.Structure):
    _fields_ = [("template_id", C.c_int32), ("scale_id", C.c_int32), ("r", C.c_int32),
                ("pad", C.c_int32), ("lo", C.c_int64 * 3), ("hi", C.c_int64 * 3)]


class oss_alg1_params(C.Structure):
    _fields_ = [("alpha_num", C.c_int32), ("alpha_den", C.c_int32), ("beta_num", C.c_int32),
                ("beta_den", C.c_int32), ("q", C.c_int32 * 3), ("feat_mask", C.c_uint32)]


class oss_template_mom(C.Structure):
    _fields_ = [("F1", C.c_int64), ("F2", C.c_int64), ("Sx", C.c_int64), ("Sy", C.c_int64),
                ("rho", C.c_int32), ("pad", C.c_int32)]


class oss_server_config(C.Structure):
    _fields_ = [("memory_budget", C.c_int64), ("lanes", C.c_int32),
                ("max_batch_templates", C.c_int32), ("queue_timeout_ns", C.c_int64)]


class oss_request(C.Structure):
    _fields_ = [("ref_key", C.c_uint64), ("dev_pixels", C.c_void_p), ("desc", oss_image_desc),
                ("tmpl", C.POINTER(oss_template_feat)), ("n_tmpl", C.c_int32),
                ("probes", C.POINTER(oss_probe)), ("n_probes", C.c_int32),
                ("tol", oss_tolerance), ("feat_mask", C.c_uint32), ("list_cap", C.c_int64),
                ("arrival_ns", C.c_int64)]


class oss_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("n_tmpl", C.c_int32), ("H", C.c_int32), ("W", C.c_int32),
                ("dev_mask", C.c_void_p), ("dev_list", C.c_void_p), ("list_cap", C.c_int64),
                ("count", C.c_int64), ("latency_ms", C.c_double), ("queue_ms", C.c_double),
                ("batch_requests", C.c_int32), ("resident_hit", C.c_int32), ("lane", C.c_int32),
                ("pad", C.c_int32)]


class oss_server_stats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("submitted", "completed", "failed", "launches",
                                         "resident_hits", "builds", "evictions", "bytes_in_use",
                                         "bytes_peak", "memory_budget")] + \
               [("queued", C.c_int32), ("running", C.c_int32)]


class OssError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {status_string(status)} ({status})")
        self.status = status


_lib = None


def load(path: str | None = None):
    """Load liboss.so (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    # torch first: its bundled HIP runtime carries the soname liboss.so needs
    # (libamdhip64.so.7), so the library binds to the one runtime torch uses
    import torch  # noqa: F401
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is missing: build it with `python -m paper_1707_05647_amd.build`")
    lib = C.CDLL(p)
    vp, i32, i64, u32 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32
    lib.oss_ctx_create.argtypes = [C.c_int, C.POINTER(vp)]
    lib.oss_ctx_destroy.argtypes = [vp]
    lib.oss_status_string.argtypes = [C.c_int]
    lib.oss_status_string.restype = C.c_char_p
    lib.oss_ref_bytes.argtypes = [C.POINTER(oss_image_desc), u32, i32, C.POINTER(C.c_size_t)]
    lib.oss_ref_create.argtypes = [vp, C.POINTER(oss_image_desc), u32, i32, C.POINTER(vp)]
    lib.oss_ref_build.argtypes = [vp, vp, vp]
    lib.oss_ref_release.argtypes = [vp]
    lib.oss_ref_tables.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp),
                                   C.POINTER(i64), C.POINTER(i32), C.POINTER(i32),
                                   C.POINTER(i32)]
    lib.oss_ref_layout.argtypes = [vp, C.POINTER(i32), C.POINTER(i64), C.POINTER(i32),
                                   C.POINTER(i64)]
    lib.oss_ref_layout_q.argtypes = [vp, C.POINTER(oss_quantity_layout), C.POINTER(i32),
                                     C.POINTER(i64)]
    lib.oss_template_features.argtypes = [vp, C.POINTER(oss_image_desc), i32, u32,
                                          C.POINTER(oss_template_feat)]
    lib.oss_feature_bounds.argtypes = [i32, i64, i32, i32, C.POINTER(oss_tolerance),
                                       C.POINTER(i64), C.POINTER(i64)]
    lib.oss_ctx_set_option.argtypes = [vp, i32, i32]
    lib.oss_ctx_get_option.argtypes = [vp, i32, C.POINTER(i32)]
    lib.oss_ctx_profile.argtypes = [vp, C.c_int]
    lib.oss_ctx_profile_read.argtypes = [vp, C.POINTER(oss_kernel_stat), i32, C.POINTER(i32)]
    lib.oss_screen.argtypes = [vp, vp, C.POINTER(oss_template_feat), i32, C.POINTER(oss_probe), i32,
                               C.POINTER(oss_tolerance), u32, vp, vp, i64, vp, vp]
    lib.oss_screen_batched.argtypes = lib.oss_screen.argtypes
    lib.oss_screen_noalloc.argtypes = lib.oss_screen.argtypes
    lib.oss_screen_intervals.argtypes = [vp, vp, i32, C.POINTER(oss_interval_probe), i32, u32,
                                         vp, vp, i64, vp, vp]
    lib.oss_alg1_probes.argtypes = [vp, C.POINTER(oss_image_desc), i32,
                                    C.POINTER(oss_alg1_params), C.POINTER(oss_interval_probe),
                                    i32, C.POINTER(i32)]
    lib.oss_template_moments.argtypes = [vp, C.POINTER(oss_image_desc), i32,
                                         C.POINTER(oss_template_mom)]
    lib.oss_screen_moments.argtypes = [vp, vp, C.POINTER(oss_template_mom), i32,
                                       C.POINTER(oss_probe), i32, C.POINTER(oss_tolerance), u32,
                                       vp, vp, i64, vp, vp]
    lib.oss_region.argtypes = [vp, i32, i32, i32, C.POINTER(oss_probe), i32, vp, i64, vp, vp, vp]
    lib.oss_template_features_rings.argtypes = [vp, C.POINTER(oss_image_desc), i32, u32, i32,
                                                C.POINTER(oss_template_feat)]
    lib.oss_screen_rings.argtypes = [vp, vp, C.POINTER(oss_template_feat), i32, i32,
                                     C.POINTER(oss_probe), i32, C.POINTER(oss_tolerance), u32, vp,
                                     vp, i64, vp, vp]
    lib.oss_autotune_batched.argtypes = [vp, vp, C.POINTER(oss_template_feat), i32,
                                         C.POINTER(oss_probe), i32, C.POINTER(oss_tolerance), u32,
                                         vp, C.POINTER(oss_tune_result)]
    lib.oss_server_create.argtypes = [C.c_int, C.POINTER(oss_server_config), C.POINTER(vp)]
    lib.oss_server_destroy.argtypes = [vp]
    lib.oss_server_submit.argtypes = [vp, C.POINTER(oss_request), C.POINTER(i64)]
    lib.oss_server_pump.argtypes = [vp, i64, C.POINTER(i32)]
    lib.oss_server_drain.argtypes = [vp]
    lib.oss_server_result.argtypes = [vp, i64, C.POINTER(oss_result)]
    lib.oss_server_release.argtypes = [vp, i64]
    lib.oss_server_cancel.argtypes = [vp, i64]
    lib.oss_server_stats_read.argtypes = [vp, C.POINTER(oss_server_stats)]
    for name in EXPORTED:
        if name != "oss_status_string":
            getattr(lib, name).restype = C.c_int
    if path is None:
        _lib = lib
    return lib


def status_string(status: int) -> str:
    return load().oss_status_string(int(status)).decode()


def _check(status: int, what: str):
    if status != OSS_OK:
        raise OssError(status, what)


def _ptr(t) -> int | None:
    if t is None:
        return None
    return int(t.data_ptr())


def _stream(stream) -> int | None:
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def image_desc(H: int, W: int, dtype: int = OSS_U8, bit_depth: int | None = None,
               pitch_bytes: int | None = None) -> oss_image_desc:
    px = 1 if dtype == OSS_U8 else 2
    return oss_image_desc(int(H), int(W), int(pitch_bytes if pitch_bytes is not None else W * px),
                          int(dtype), int(bit_depth if bit_depth is not None else 8 * px))


def device_image(arr, device):
    """Copy a 2-D uint8/uint16 numpy image to a torch device tensor (16-bit
    pixels travel as int16 storage, the same bytes)."""
    import torch
    a = np.ascontiguousarray(arr)
    if a.dtype == np.uint16:
        a = a.view(np.int16)
    return torch.from_numpy(a).to(device)


def desc_of(arr, bit_depth: int | None = None) -> oss_image_desc:
    """Descriptor of a 2-D uint8/uint16 numpy array or torch tensor."""
    import torch
    if isinstance(arr, torch.Tensor):
        # int16 tensors are accepted as the storage of 16-bit unsigned pixels
        if (arr.dtype not in (torch.uint8, torch.uint16, torch.int16) or arr.dim() != 2
                or arr.stride(1) != 1):
            raise ValueError("need a 2-D uint8/uint16 tensor with unit column stride")
        dt = OSS_U8 if arr.dtype == torch.uint8 else OSS_U16
        return image_desc(arr.shape[0], arr.shape[1], dt, bit_depth,
                          arr.stride(0) * arr.element_size())
    a = np.asarray(arr)
    if a.dtype not in (np.uint8, np.uint16) or a.ndim != 2 or a.strides[1] != a.itemsize:
        raise ValueError("need a 2-D uint8/uint16 array with unit column stride")
    dt = OSS_U8 if a.dtype == np.uint8 else OSS_U16
    return image_desc(a.shape[0], a.shape[1], dt, bit_depth, a.strides[0])


def oss_ctx_create(device: int = 0) -> int:
    h = C.c_void_p()
    _check(load().oss_ctx_create(int(device), C.byref(h)), "oss_ctx_create")
    return h.value


def oss_ctx_destroy(ctx: int):
    _check(load().oss_ctx_destroy(ctx), "oss_ctx_destroy")


def oss_ctx_set_option(ctx: int, option: int, value: int):
    _check(load().oss_ctx_set_option(ctx, int(option), int(value)), "oss_ctx_set_option")


def oss_ctx_get_option(ctx: int, option: int) -> int:
    v = C.c_int32()
    _check(load().oss_ctx_get_option(ctx, int(option), C.byref(v)), "oss_ctx_get_option")
    return v.value


def oss_ctx_profile(ctx: int, enable: bool):
    _check(load().oss_ctx_profile(ctx, 1 if enable else 0), "oss_ctx_profile")


def oss_ctx_profile_read(ctx: int) -> dict:
    """{kernel name: (launches, total_ms, max_ms)} (waits for the events)."""
    arr = (oss_kernel_stat * 32)()
    n = C.c_int32()
    _check(load().oss_ctx_profile_read(ctx, arr, 32, C.byref(n)), "oss_ctx_profile_read")
    return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms, arr[i].max_ms)
            for i in range(n.value)}


def oss_ref_bytes(desc: oss_image_desc, feat_mask: int, max_radius: int = -1) -> int:
    out = C.c_size_t()
    _check(load().oss_ref_bytes(C.byref(desc), int(feat_mask), int(max_radius), C.byref(out)),
           "oss_ref_bytes")
    return out.value


def oss_ref_create(ctx: int, desc: oss_image_desc, feat_mask: int, max_radius: int = -1) -> int:
    h = C.c_void_p()
    _check(load().oss_ref_create(ctx, C.byref(desc), int(feat_mask), int(max_radius),
                                 C.byref(h)), "oss_ref_create")
    return h.value


def oss_ref_build(ref: int, pixels, stream=None):
    _check(load().oss_ref_build(ref, _ptr(pixels), _stream(stream)), "oss_ref_build")


def oss_ref_release(ref: int):
    _check(load().oss_ref_release(ref), "oss_ref_release")


def oss_ref_layout(ref: int):
    """(entry_stride, [(offset, bits) per quantity slot], plane_bytes)."""
    eb = C.c_int32()
    off = (C.c_int64 * OSS_MAX_QUANTITIES)()
    bits = (C.c_int32 * OSS_MAX_QUANTITIES)()
    plane = C.c_int64()
    _check(load().oss_ref_layout(ref, C.byref(eb), off, bits, C.byref(plane)), "oss_ref_layout")
    return (eb.value, [(off[q], bits[q]) for q in range(OSS_MAX_QUANTITIES) if bits[q]],
            plane.value)


def oss_ref_layout_q(ref: int):
    """([(offset, stride, bits, hi_offset, hi_stride, hi_bits) per quantity
    slot], plane_bytes): hi_offset -1 means no high part; a value is stored
    modulo 2^(bits + hi_bits)."""
    out = (oss_quantity_layout * OSS_MAX_QUANTITIES)()
    nq = C.c_int32()
    plane = C.c_int64()
    _check(load().oss_ref_layout_q(ref, out, C.byref(nq), C.byref(plane)), "oss_ref_layout_q")
    return ([(o.offset, o.stride, o.bits, o.hi_offset, o.hi_stride, o.hi_bits)
             for o in out[:nq.value]], plane.value)


def oss_ref_tables(ref: int):
    """(L, R, Rp) device pointers, pitch in entries, number of quantities,
    value width in bits (32: sums modulo 2^32, or 64), maximum radius."""
    L, R, Rp = C.c_void_p(), C.c_void_p(), C.c_void_p()
    pitch, nq, vb, mr = C.c_int64(), C.c_int32(), C.c_int32(), C.c_int32()
    _check(load().oss_ref_tables(ref, C.byref(L), C.byref(R), C.byref(Rp), C.byref(pitch),
                                 C.byref(nq), C.byref(vb), C.byref(mr)), "oss_ref_tables")
    return L.value, R.value, Rp.value, pitch.value, nq.value, vb.value, mr.value


def oss_template_features(pixels, rho: int, feat_mask: int,
                          bit_depth: int | None = None) -> oss_template_feat:
    a = np.ascontiguousarray(pixels)
    out = oss_template_feat()
    d = desc_of(a, bit_depth)
    _check(load().oss_template_features(a.ctypes.data, C.byref(d), int(rho), int(feat_mask),
                                        C.byref(out)), "oss_template_features")
    return out


def tolerance(P, Q: int) -> oss_tolerance:
    P = list(P) + [0] * (3 - len(P))
    return oss_tolerance((C.c_int32 * 3)(*[int(v) for v in P[:3]]), int(Q))


def oss_feature_bounds(feature: int, FT: int, r: int, rho: int, P, Q: int):
    """(lo, hi): the feature sums F that pass are exactly lo <= F <= hi."""
    lo, hi = C.c_int64(), C.c_int64()
    _check(load().oss_feature_bounds(int(feature), int(FT), int(r), int(rho),
                                     C.byref(tolerance(P, Q)), C.byref(lo), C.byref(hi)),
           "oss_feature_bounds")
    return lo.value, hi.value


def _screen_args(tmpl, probes, tol):
    nt = len(tmpl)
    ta = (oss_template_feat * nt)(*tmpl)
    npb = len(probes)
    pa = (oss_probe * max(1, npb))(*[oss_probe(int(t), int(k), int(r)) for t, k, r in probes])
    if not isinstance(tol, oss_tolerance):
        P0, P1, P2, Q = tol
        tol = oss_tolerance((C.c_int32 * 3)(int(P0), int(P1), int(P2)), int(Q))
    return ta, nt, pa, npb, tol


def oss_screen(ctx: int, ref: int, tmpl, probes, tol, feat_mask: int, mask=None, cand_list=None,
               list_cap: int = 0, count=None, stream=None, batched: bool = False):
    """tmpl: sequence of oss_template_feat; probes: sequence of (t, k, r);
    tol: (P0, P1, P2, Q) or oss_tolerance; mask/cand_list/count: torch
    device tensors (uint8 [T,H,W], int32 [cap,4], int64 [1]).  batched=True
    calls oss_screen_batched."""
    ta, nt, pa, npb, tol = _screen_args(tmpl, probes, tol)
    if count is None:
        raise ValueError("count tensor required")
    fn = load().oss_screen_batched if batched else load().oss_screen
    _check(fn(ctx, ref, ta, nt, pa, npb, C.byref(tol), int(feat_mask), _ptr(mask),
              _ptr(cand_list), int(list_cap), _ptr(count), _stream(stream)),
           "oss_screen_batched" if batched else "oss_screen")


def oss_screen_noalloc(ctx: int, ref: int, tmpl, probes, tol, feat_mask: int, mask=None,
                       cand_list=None, list_cap: int = 0, count=None, stream=None):
    """oss_screen with its scratch in the library's fixed device array (no
    allocation; OSS_E_LIMIT past OSS_NOALLOC_SCRATCH_BYTES)."""
    ta, nt, pa, npb, tol = _screen_args(tmpl, probes, tol)
    if count is None:
        raise ValueError("count tensor required")
    _check(load().oss_screen_noalloc(ctx, ref, ta, nt, pa, npb, C.byref(tol), int(feat_mask),
                                     _ptr(mask), _ptr(cand_list), int(list_cap), _ptr(count),
                                     _stream(stream)), "oss_screen_noalloc")


def oss_screen_batched(ctx: int, ref: int, tmpl, probes, tol, feat_mask: int, mask=None,
                       cand_list=None, list_cap: int = 0, count=None, stream=None):
    oss_screen(ctx, ref, tmpl, probes, tol, feat_mask, mask, cand_list, list_cap, count, stream,
               batched=True)


def oss_autotune_batched(ctx: int, ref: int, tmpl, probes, tol, feat_mask: int,
                         stream=None) -> oss_tune_result:
    ta, nt, pa, npb, tol = _screen_args(tmpl, probes, tol)
    out = oss_tune_result()
    _check(load().oss_autotune_batched(ctx, ref, ta, nt, pa, npb, C.byref(tol), int(feat_mask),
                                       _stream(stream), C.byref(out)), "oss_autotune_batched")
    return out


# --- serving loop -----------------------------------------------------------

def oss_server_create(device: int, memory_budget: int, lanes: int = 2,
                      max_batch_templates: int = 64, queue_timeout_ns: int = 0) -> int:
    h = C.c_void_p()
    cfg = oss_server_config(int(memory_budget), int(lanes), int(max_batch_templates),
                            int(queue_timeout_ns))
    _check(load().oss_server_create(int(device), C.byref(cfg), C.byref(h)), "oss_server_create")
    return h.value


def oss_server_destroy(srv: int):
    _check(load().oss_server_destroy(srv), "oss_server_destroy")


def oss_server_submit(srv: int, ref_key: int, pixels, tmpl, probes, tol, feat_mask: int,
                      list_cap: int, bit_depth: int | None = None, arrival_ns: int = 0) -> int:
    """pixels: torch device tensor [H, W] (uint8, or int16 holding uint16);
    it must stay alive until the request completes."""
    ta, nt, pa, npb, tl = _screen_args(tmpl, probes, tol)
    rq = oss_request(int(ref_key), _ptr(pixels), desc_of(pixels, bit_depth), ta, nt, pa, npb, tl,
                     int(feat_mask), int(list_cap), int(arrival_ns))
    rid = C.c_int64()
    _check(load().oss_server_submit(srv, C.byref(rq), C.byref(rid)), "oss_server_submit")
    return rid.value


def oss_server_pump(srv: int, wait_us: int = 0) -> int:
    n = C.c_int32()
    _check(load().oss_server_pump(srv, int(wait_us), C.byref(n)), "oss_server_pump")
    return n.value


def oss_server_drain(srv: int):
    _check(load().oss_server_drain(srv), "oss_server_drain")


def oss_server_result(srv: int, rid: int) -> oss_result:
    out = oss_result()
    _check(load().oss_server_result(srv, int(rid), C.byref(out)), "oss_server_result")
    return out


def oss_server_cancel(srv: int, rid: int):
    _check(load().oss_server_cancel(srv, int(rid)), "oss_server_cancel")


def oss_server_release(srv: int, rid: int):
    _check(load().oss_server_release(srv, int(rid)), "oss_server_release")


def oss_server_stats_read(srv: int) -> dict:
    out = oss_server_stats()
    _check(load().oss_server_stats_read(srv, C.byref(out)), "oss_server_stats_read")
    return {n: getattr(out, n) for n, _ in oss_server_stats._fields_}


# --- multi-central-area screen -------------------------------------------------

def oss_template_features_rings(pixels, rho: int, feat_mask: int, n_rings: int,
                                bit_depth: int | None = None) -> list:
    a = np.ascontiguousarray(pixels)
    d = desc_of(a, bit_depth)
    out = (oss_template_feat * n_rings)()
    _check(load().oss_template_features_rings(a.ctypes.data, C.byref(d), int(rho),
                                              int(feat_mask), int(n_rings), out),
           "oss_template_features_rings")
    return list(out)


def oss_screen_rings(ctx: int, ref: int, tmpl_rings, probes, tol, feat_mask: int, mask=None,
                     cand_list=None, list_cap: int = 0, count=None, stream=None):
    """tmpl_rings: one list of n_rings oss_template_feat per template (as from
    oss_template_features_rings)."""
    n_rings = len(tmpl_rings[0])
    if any(len(r) != n_rings for r in tmpl_rings):
        raise ValueError("every template needs the same number of rings")
    flat = [f for rings in tmpl_rings for f in rings]
    ta, _, pa, npb, tl = _screen_args(flat, probes, tol)
    if count is None:
        raise ValueError("count tensor required")
    _check(load().oss_screen_rings(ctx, ref, ta, len(tmpl_rings), n_rings, pa, npb, C.byref(tl),
                                   int(feat_mask), _ptr(mask), _ptr(cand_list), int(list_cap),
                                   _ptr(count), _stream(stream)), "oss_screen_rings")


def oss_region(ctx: int, H: int, W: int, n_tmpl: int, probes, cand_list, list_cap: int, count,
               region, stream=None):
    """region: torch uint8 [n_tmpl, H, W] on the device (overwritten)."""
    npb = len(probes)
    pa = (oss_probe * max(1, npb))(*[oss_probe(int(t), int(k), int(r)) for t, k, r in probes])
    _check(load().oss_region(ctx, int(H), int(W), int(n_tmpl), pa, npb, _ptr(cand_list),
                             int(list_cap), _ptr(count), _ptr(region), _stream(stream)),
           "oss_region")


# --- interval probes and Algorithm 1 -----------------------------------------------

def oss_alg1_probes(pixels, t: int, alpha, beta, q, feat_mask: int,
                    bit_depth: int | None = None) -> list:
    """Algorithm 1's interval probes of one square template (alpha, beta as
    fractions.Fraction or (num, den))."""
    from fractions import Fraction
    a, b = Fraction(alpha), Fraction(beta)
    a_img = np.ascontiguousarray(pixels)
    d = desc_of(a_img, bit_depth)
    prm = oss_alg1_params(a.numerator, a.denominator, b.numerator, b.denominator,
                          (C.c_int32 * 3)(*[int(v) for v in q]), int(feat_mask))
    n = C.c_int32()
    cap = 256  # one call unless a template has more distinct band probes
    out = (oss_interval_probe * cap)()
    rc = load().oss_alg1_probes(a_img.ctypes.data, C.byref(d), int(t), C.byref(prm), out, cap,
                                C.byref(n))
    if rc == OSS_E_NOMEM:
        out = (oss_interval_probe * n.value)()
        rc = load().oss_alg1_probes(a_img.ctypes.data, C.byref(d), int(t), C.byref(prm), out,
                                    n.value, C.byref(n))
    _check(rc, "oss_alg1_probes")
    return list(out[:n.value])


def oss_screen_intervals(ctx: int, ref: int, n_tmpl: int, probes, feat_mask: int, mask=None,
                         cand_list=None, list_cap: int = 0, count=None, stream=None):
    npb = len(probes)
    pa = (oss_interval_probe * max(1, npb))(*probes)
    if count is None:
        raise ValueError("count tensor required")
    _check(load().oss_screen_intervals(ctx, ref, int(n_tmpl), pa, npb, int(feat_mask),
                                       _ptr(mask), _ptr(cand_list), int(list_cap), _ptr(count),
                                       _stream(stream)), "oss_screen_intervals")


# --- the paper's own features ---------------------------------------------------------

def oss_template_moments(pixels, rho: int, bit_depth: int | None = None) -> oss_template_mom:
    a = np.ascontiguousarray(pixels)
    out = oss_template_mom()
    d = desc_of(a, bit_depth)
    _check(load().oss_template_moments(a.ctypes.data, C.byref(d), int(rho), C.byref(out)),
           "oss_template_moments")
    return out


def oss_screen_moments(ctx: int, ref: int, tmpl, probes, tol, tests: int, mask=None,
                       cand_list=None, list_cap: int = 0, count=None, stream=None):
    nt = len(tmpl)
    ta = (oss_template_mom * nt)(*tmpl)
    npb = len(probes)
    pa = (oss_probe * max(1, npb))(*[oss_probe(int(t), int(k), int(r)) for t, k, r in probes])
    if not isinstance(tol, oss_tolerance):
        P0, P1, P2, Q = tol
        tol = oss_tolerance((C.c_int32 * 3)(int(P0), int(P1), int(P2)), int(Q))
    if count is None:
        raise ValueError("count tensor required")
    _check(load().oss_screen_moments(ctx, ref, ta, nt, pa, npb, C.byref(tol), int(tests),
                                     _ptr(mask), _ptr(cand_list), int(list_cap), _ptr(count),
                                     _stream(stream)), "oss_screen_moments")
