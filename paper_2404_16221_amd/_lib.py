"""ctypes binding of libxl.so (include/xl.h).  Argument marshalling only.

Every function has the name of the C entry point it calls.  Tensors must live
on the GPU, be contiguous and have the documented dtype; the call is enqueued
on torch's current stream.  There is no fallback: if libxl.so is missing or a
call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libxl.so")

XL_OK, XL_PENDING = 0, 1
XL_EINVAL, XL_ENOMEM, XL_EHIP, XL_EAGAIN, XL_EFAULT = -1, -2, -3, -4, -5
XL_F32, XL_BF16, XL_F16 = 0, 1, 2
XL_MERGE_FP64 = 1
XL_MERGE_STAGED = 2
DTYPES = {torch.float32: XL_F32, torch.bfloat16: XL_BF16, torch.float16: XL_F16}
XL_BF16_F16 = 3
# Mixed 16-bit storage: sigma in bfloat16, rgb in float16.
BF16_F16 = (torch.bfloat16, torch.float16)


def storage_code(sigma_dtype, rgb_dtype=None) -> int:
    """The XL_* storage code of (sigma, rgb) dtypes (one dtype: both alike)."""
    rgb_dtype = sigma_dtype if rgb_dtype is None else rgb_dtype
    if (sigma_dtype, rgb_dtype) == BF16_F16:
        return XL_BF16_F16
    if sigma_dtype != rgb_dtype or sigma_dtype not in DTYPES:
        raise ValueError(f"unsupported storage: sigma {sigma_dtype}, rgb {rgb_dtype}")
    return DTYPES[sigma_dtype]


def storage_dtypes(dtype):
    """(sigma dtype, rgb dtype) of a storage given as a torch dtype or a pair."""
    return tuple(dtype) if isinstance(dtype, (tuple, list)) else (dtype, dtype)
TORCH_DTYPES = {v: k for k, v in DTYPES.items()}
TUPLE = 7
TUPLE_STRIDE = 8  # XL_TUPLE_STRIDE: words per segment tuple record

_c = ctypes
_vp, _i64, _i32, _sz = _c.c_void_p, _c.c_int64, _c.c_int32, _c.c_size_t


class XLSamples(_c.Structure):
    _fields_ = [("dtype", _i32), ("sigma", _vp), ("rgb", _vp), ("t_start", _vp),
                ("t_end", _vp), ("n", _i64)]


class XLGenParams(_c.Structure):
    _fields_ = [("n_rays", _i64), ("ray0", _i64), ("n_min", _i32), ("n_max", _i32),
                ("grid", _i32 * 3), ("reserved", _i32), ("sigma_mu", _c.c_double),
                ("sigma_s", _c.c_double), ("zero_frac", _c.c_double), ("width_mean", _c.c_double),
                ("t_far", _c.c_double), ("seed", _c.c_uint64)]


class XLRays(_c.Structure):
    _fields_ = [("origins", _vp), ("dirs", _vp), ("t_start", _vp), ("t_end", _vp),
                ("ray_offsets", _vp), ("n_rays", _i64)]


class XLFeatures(_c.Structure):
    _fields_ = [("dtype", _i32), ("n_feat", _i32), ("sigma", _vp), ("feat", _vp), ("t_start", _vp),
                ("t_end", _vp), ("n", _i64)]


class XLBreakable(_c.Structure):
    _fields_ = [("dtype", _i32), ("source", _i32), ("n_ch", _i32), ("n_pairs", _i32),
                ("pair_a", _i32 * 4), ("pair_b", _i32 * 4), ("sigma", _vp), ("ch", _vp),
                ("t_start", _vp), ("t_end", _vp), ("n", _i64)]


XL_CH_LOADED = 0
XL_CH_MIDPOINT_POWERS = 1


class XLError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libxl error {code}: {msg}")
        self.code = code


_LIB: Optional[ctypes.CDLL] = None

# name -> (restype, argtypes)
SIGNATURES = {
    "xl_version": (_c.c_int, []),
    "xl_last_error": (_c.c_char_p, []),
    "xl_segments_workspace_bytes": (_sz, [_i64]),
    "xl_render_segments_fwd": (_c.c_int, [_c.POINTER(XLSamples), _vp, _i64, _vp, _vp, _sz, _vp]),
    "xl_render_segments_fwd_static": (_c.c_int, [_c.POINTER(XLSamples), _vp, _i64, _vp, _vp]),
    "xl_render_segments_bwd": (_c.c_int, [_c.POINTER(XLSamples), _vp, _i64, _vp, _sz, _vp, _vp,
                                          _vp, _vp]),
    "xl_merge_fwd": (_c.c_int, [_vp, _i64, _vp, _i32, _vp, _vp, _i64, _vp, _i32, _vp]),
    "xl_merge_bwd": (_c.c_int, [_vp, _i64, _vp, _i32, _vp, _vp, _i64, _vp, _vp, _i32, _vp]),
    "xl_check_inputs": (_c.c_int, [_c.POINTER(XLSamples), _vp, _i64, _vp, _vp, _i64, _vp]),
    "xl_gen_workspace_bytes": (_sz, [_c.POINTER(XLGenParams)]),
    "xl_gen_plan": (_c.c_int, [_c.POINTER(XLGenParams), _vp, _sz, _c.POINTER(_i64),
                               _c.POINTER(_i64), _vp]),
    "xl_gen_fill": (_c.c_int, [_c.POINTER(XLGenParams), _i32, _vp, _sz, _i64, _vp, _vp, _vp, _vp,
                               _vp, _vp, _vp, _vp, _vp]),
    "xl_partition_build": (_c.c_int, [_vp, _i64, _i32, _vp, _vp]),
    "xl_render_features_fwd": (_c.c_int, [_c.POINTER(XLFeatures), _vp, _i64, _vp, _vp, _vp]),
    "xl_merge_features_fwd": (_c.c_int, [_vp, _vp, _i32, _i64, _vp, _vp, _i64, _vp, _vp]),
    "xl_merge_features_bwd": (_c.c_int, [_vp, _vp, _i32, _i64, _vp, _vp, _i64, _vp, _vp, _vp, _vp]),
    "xl_render_features_bwd": (_c.c_int, [_c.POINTER(XLFeatures), _vp, _i64, _vp, _vp, _vp, _vp, _vp,
                                          _i32, _vp]),
    "xl_render_breakable_fwd": (_c.c_int, [_c.POINTER(XLBreakable), _vp, _i64, _vp, _vp]),
    "xl_merge_breakable_fwd": (_c.c_int, [_c.POINTER(XLBreakable), _vp, _i64, _vp, _vp, _i64, _vp,
                                          _vp]),
    "xl_merge_breakable_bwd": (_c.c_int, [_c.POINTER(XLBreakable), _vp, _i64, _vp, _vp, _i64, _vp,
                                          _vp, _vp]),
    "xl_render_breakable_bwd": (_c.c_int, [_c.POINTER(XLBreakable), _vp, _i64, _vp, _vp, _vp, _vp,
                                           _i32, _vp]),
    "xl_pack_workspace_bytes": (_sz, [_i64, _i32]),
    "xl_pack_plan": (_c.c_int, [_c.POINTER(XLRays), _vp, _vp, _i32, _vp, _sz, _c.POINTER(_i64),
                                _c.POINTER(_i64), _vp]),
    "xl_pack_fill": (_c.c_int, [_c.POINTER(XLRays), _vp, _vp, _i32, _vp, _sz, _i64, _vp, _vp, _vp,
                                _vp, _vp, _vp, _vp, _vp, _vp]),
}


def lib() -> ctypes.CDLL:
    """The loaded libxl.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2404_16221_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def _check(rc: int) -> None:
    if rc != XL_OK:
        raise XLError(rc, lib().xl_last_error().decode())


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _dev(t: torch.Tensor, name: str, dtype=None) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype not in (dtype if isinstance(dtype, tuple) else (dtype,)):
        raise ValueError(f"{name} has dtype {t.dtype}, expected {dtype}")
    return t.data_ptr() if t.numel() else 0


def tuple_buffer(n_seg: int, device, zero: bool = False) -> torch.Tensor:
    """Segment tuples (or their gradients) as the library stores them, one
    record of TUPLE_STRIDE floats per segment, seen as the [7, n_seg] tensor of
    components (a strided view; the pad word stays out of it)."""
    alloc = torch.zeros if zero else torch.empty
    return alloc((n_seg, TUPLE_STRIDE), dtype=torch.float32, device=device)[:, :TUPLE].t()


def as_tuples(x: torch.Tensor) -> torch.Tensor:
    """A copy of [7, n_seg] components in tuple records (see tuple_buffer)."""
    if x.dim() != 2 or x.shape[0] != TUPLE:
        raise ValueError("expected [7, n_seg] tuple components")
    out = tuple_buffer(x.shape[1], x.device, zero=True)
    out.copy_(x)
    return out


def _tup(t: torch.Tensor, name: str) -> int:
    """Pointer of a tuple array: a [7, n_seg] view made by tuple_buffer (or
    any [7, n_seg] float32 view with strides (1, TUPLE_STRIDE) over
    16-byte-aligned records)."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32:
        raise ValueError(f"{name} must be a float32 CUDA tensor")
    if t.dim() != 2 or t.shape[0] != TUPLE:
        raise ValueError(f"{name} must be [7, n_seg] (see tuple_buffer)")
    n = t.shape[1]
    if n == 0:
        return 0
    records = t.untyped_storage().nbytes() - t.storage_offset() * 4
    if (t.stride(0) != 1 or (n > 1 and t.stride(1) != TUPLE_STRIDE)
            or records < 4 * TUPLE_STRIDE * n or t.data_ptr() % 16):
        raise ValueError(f"{name} must be tuple records: a [7, n_seg] view with strides "
                         f"(1, {TUPLE_STRIDE}) over 16-byte-aligned storage, from tuple_buffer "
                         "or as_tuples")
    return t.data_ptr()


def samples(sigma, rgb, t_start, t_end) -> XLSamples:
    code = storage_code(sigma.dtype, rgb.dtype)
    n = sigma.shape[0]
    if rgb.shape != (n, 3) or t_start.shape != (n,) or t_end.shape != (n,):
        raise ValueError("shapes must be sigma[n], rgb[n,3], t_start[n], t_end[n]")
    return XLSamples(code, _dev(sigma, "sigma"), _dev(rgb, "rgb"),
                     _dev(t_start, "t_start", torch.float32), _dev(t_end, "t_end", torch.float32), n)


def xl_version() -> int:
    return lib().xl_version()


def xl_segments_workspace_bytes(n: int) -> int:
    return lib().xl_segments_workspace_bytes(n)


def xl_render_segments_fwd(sigma, rgb, t_start, t_end, seg_offsets, seg_out=None,
                           workspace=None) -> Tuple[torch.Tensor, torch.Tensor]:
    """seg_out[7, n_seg] (a view of the tuple records, see tuple_buffer) and
    the workspace the backward needs."""
    s = samples(sigma, rgb, t_start, t_end)
    n_seg = seg_offsets.shape[0] - 1
    dev = sigma.device
    if seg_out is None:
        seg_out = tuple_buffer(n_seg, dev)
    wsb = xl_segments_workspace_bytes(s.n)
    if workspace is None:
        workspace = torch.empty(wsb, dtype=torch.uint8, device=dev)
    _check(lib().xl_render_segments_fwd(ctypes.byref(s), _dev(seg_offsets, "seg_offsets", torch.int64),
                                        n_seg, _tup(seg_out, "seg_out"),
                                        _dev(workspace, "workspace"), workspace.numel(), _stream()))
    return seg_out, workspace


def xl_render_segments_fwd_static(sigma, rgb, t_start, t_end, seg_offsets,
                                  seg_out=None) -> torch.Tensor:
    """seg_out[7, n_seg] by the no-allocation entry point (tile records in the
    library's static scratch; forward only)."""
    s = samples(sigma, rgb, t_start, t_end)
    n_seg = seg_offsets.shape[0] - 1
    if seg_out is None:
        seg_out = tuple_buffer(n_seg, sigma.device)
    _check(lib().xl_render_segments_fwd_static(ctypes.byref(s),
                                               _dev(seg_offsets, "seg_offsets", torch.int64), n_seg,
                                               _tup(seg_out, "seg_out"), _stream()))
    return seg_out


def xl_render_segments_bwd(sigma, rgb, t_start, t_end, seg_offsets, workspace, grad_seg,
                           grad_sigma=None, grad_rgb=None) -> Tuple[torch.Tensor, torch.Tensor]:
    """(dl/dsigma [n], dl/drgb [n, 3]) in the storage dtype."""
    s = samples(sigma, rgb, t_start, t_end)
    n_seg = seg_offsets.shape[0] - 1
    if grad_sigma is None:
        grad_sigma = torch.empty_like(sigma)
    if grad_rgb is None:
        grad_rgb = torch.empty_like(rgb)
    _check(lib().xl_render_segments_bwd(ctypes.byref(s), _dev(seg_offsets, "seg_offsets", torch.int64),
                                        n_seg, _dev(workspace, "workspace"), workspace.numel(),
                                        _tup(grad_seg, "grad_seg"),
                                        _dev(grad_sigma, "grad_sigma", sigma.dtype),
                                        _dev(grad_rgb, "grad_rgb", rgb.dtype), _stream()))
    return grad_sigma, grad_rgb


def _check_ids(seg_out, seg_ids):
    if seg_ids.shape != (seg_out.shape[1],):
        raise ValueError("seg_ids must list every segment once: shape (n_seg,)")


def _regions(region_offsets):
    """(pointer, n_regions) of optional region boundaries [K + 1]."""
    if region_offsets is None:
        return None, 0
    return _dev(region_offsets, "region_offsets", torch.int64), region_offsets.shape[0] - 1


def _merge_flags(fp64, staged):
    return (XL_MERGE_FP64 if fp64 else 0) | (XL_MERGE_STAGED if staged else 0)


def xl_merge_fwd(seg_out, ray_offsets, seg_ids, ray_out=None, fp64: bool = False,
                 region_offsets=None, staged: bool = False) -> torch.Tensor:
    """ray_out[7, n_rays] = (T, r, g, b, A, D, L).  region_offsets [K + 1]
    (optional): the tuples' region boundaries, for the LDS-staged form (used
    from 4M segments up, or at any size with staged=True)."""
    _check_ids(seg_out, seg_ids)
    n_seg = seg_out.shape[1]
    n_rays = ray_offsets.shape[0] - 1
    if ray_out is None:
        ray_out = torch.empty((TUPLE, n_rays), dtype=torch.float32, device=seg_out.device)
    _check(lib().xl_merge_fwd(_tup(seg_out, "seg_out"), n_seg,
                              *_regions(region_offsets),
                              _dev(ray_offsets, "ray_offsets", torch.int64),
                              _dev(seg_ids, "seg_ids", torch.int64), n_rays,
                              _dev(ray_out, "ray_out", torch.float32),
                              _merge_flags(fp64, staged), _stream()))
    return ray_out


def xl_merge_bwd(seg_out, ray_offsets, seg_ids, grad_ray, grad_seg=None,
                 fp64: bool = False, region_offsets=None, staged: bool = False) -> torch.Tensor:
    """grad_seg[7, n_seg] = dl/d(tau, r, g, b, A, D, L) of each listed segment
    (tuple records, see tuple_buffer)."""
    _check_ids(seg_out, seg_ids)
    n_seg = seg_out.shape[1]
    n_rays = ray_offsets.shape[0] - 1
    if grad_seg is None:
        grad_seg = tuple_buffer(n_seg, seg_out.device, zero=True)
    _check(lib().xl_merge_bwd(_tup(seg_out, "seg_out"), n_seg,
                              *_regions(region_offsets),
                              _dev(ray_offsets, "ray_offsets", torch.int64),
                              _dev(seg_ids, "seg_ids", torch.int64), n_rays,
                              _dev(grad_ray, "grad_ray", torch.float32),
                              _tup(grad_seg, "grad_seg"),
                              _merge_flags(fp64, staged), _stream()))
    return grad_seg


def xl_check_inputs(sigma, rgb, t_start, t_end, seg_offsets, ray_offsets=None,
                    seg_ids=None) -> None:
    s = samples(sigma, rgb, t_start, t_end)
    n_seg = seg_offsets.shape[0] - 1
    n_rays = 0 if ray_offsets is None else ray_offsets.shape[0] - 1
    _check(lib().xl_check_inputs(ctypes.byref(s), _dev(seg_offsets, "seg_offsets", torch.int64),
                                 n_seg, None if ray_offsets is None else _dev(ray_offsets, "ray_offsets"),
                                 None if seg_ids is None else _dev(seg_ids, "seg_ids"), n_rays,
                                 _stream()))


def gen_params(w, ray0: int = 0, n_rays: Optional[int] = None) -> XLGenParams:
    """Device generator parameters for rays [ray0, ray0 + n_rays) of workload `w`
    (a synth.Workload)."""
    n = w.n_rays - ray0 if n_rays is None else n_rays
    return XLGenParams(n, ray0, w.n_min, w.n_max, (_i32 * 3)(*w.grid), 0, w.sigma_mu, w.sigma_s,
                       w.zero_frac, w.width_mean, w.t_far, w.seed)


def xl_gen(w, dtype=torch.float32, ray0: int = 0, n_rays: Optional[int] = None,
           device="cuda") -> dict:
    """Generate rays of workload `w` on the device, packed region-major.

    dtype: a torch dtype for both sigma and rgb, or the pair BF16_F16.
    Returns device tensors sigma, rgb (storage dtypes), t_start, t_end,
    seg_offsets, ray_offsets, seg_ids, region_offsets."""
    p = gen_params(w, ray0, n_rays)
    L = lib()
    wsb = L.xl_gen_workspace_bytes(ctypes.byref(p))
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=device)
    ns, nseg = _i64(0), _i64(0)
    _check(L.xl_gen_plan(ctypes.byref(p), ws.data_ptr(), wsb, ctypes.byref(ns), ctypes.byref(nseg),
                         _stream()))
    n, n_seg = ns.value, nseg.value
    sdt, cdt = storage_dtypes(dtype)
    out = dict(sigma=torch.empty(n, dtype=sdt, device=device),
               rgb=torch.empty((n, 3), dtype=cdt, device=device),
               t_start=torch.empty(n, dtype=torch.float32, device=device),
               t_end=torch.empty(n, dtype=torch.float32, device=device),
               seg_offsets=torch.empty(n_seg + 1, dtype=torch.int64, device=device),
               ray_offsets=torch.empty(p.n_rays + 1, dtype=torch.int64, device=device),
               seg_ids=torch.empty(n_seg, dtype=torch.int64, device=device),
               region_offsets=torch.empty(w.grid[0] * w.grid[1] * w.grid[2] + 1, dtype=torch.int64,
                                          device=device))
    _check(L.xl_gen_fill(ctypes.byref(p), storage_code(sdt, cdt), ws.data_ptr(), wsb, n_seg,
                         _dev(out["sigma"], "sigma"), _dev(out["rgb"], "rgb"),
                         _dev(out["t_start"], "t_start"), _dev(out["t_end"], "t_end"),
                         _dev(out["seg_offsets"], "seg_offsets"), _dev(out["ray_offsets"], "ray_offsets"),
                         _dev(out["seg_ids"], "seg_ids"),
                         _dev(out["region_offsets"], "region_offsets"), _stream()))
    return out


def xl_partition_build(points, levels: int):
    """(axis int32 [2^levels - 1], plane float32 [...]) of the CDF partition of
    `points` (host array-like [n, 3], float32).  Runs on the host."""
    import numpy as np
    pts = np.ascontiguousarray(np.asarray(points, dtype=np.float32).reshape(-1, 3))
    k1 = max((1 << levels) - 1, 0) if 0 <= levels <= 30 else 0
    axis = np.zeros(max(k1, 1), dtype=np.int32)
    plane = np.zeros(max(k1, 1), dtype=np.float32)
    _check(lib().xl_partition_build(pts.ctypes.data if pts.size else None, pts.shape[0], levels,
                                    axis.ctypes.data, plane.ctypes.data))
    return axis[:k1], plane[:k1]


def _tree(axis, plane, device):
    a = torch.as_tensor(axis, dtype=torch.int32).to(device).contiguous()
    p = torch.as_tensor(plane, dtype=torch.float32).to(device).contiguous()
    if a.numel() == 0:  # the one-box tree: the kernels read nothing
        a = torch.zeros(1, dtype=torch.int32, device=device)
        p = torch.zeros(1, dtype=torch.float32, device=device)
    return a, p


def xl_pack(origins, dirs, t_start, t_end, ray_offsets, axis, plane, levels: int,
            with_src: bool = True, reuse: Optional[dict] = None) -> dict:
    """Cut, tag and pack ray-major samples region-major (xl_pack_plan + xl_pack_fill).

    origins, dirs: device float32 [R, 3]; t_start, t_end: device float32 [n];
    ray_offsets: device int64 [R + 1]; axis, plane: the partition tree (host or
    device).  Returns device tensors t_start, t_end, src (or None),
    seg_offsets, ray_offsets, seg_ids, seg_box, region_offsets, and the
    workspace.  reuse: the result of an earlier call whose tensors (workspace
    included) are written again where their shapes fit, instead of allocating."""
    dev = origins.device
    R = origins.shape[0]
    if origins.shape != (R, 3) or dirs.shape != (R, 3) or ray_offsets.shape != (R + 1,):
        raise ValueError("shapes must be origins[R,3], dirs[R,3], ray_offsets[R+1]")
    if t_start.shape != t_end.shape or t_start.dim() != 1:
        raise ValueError("t_start and t_end must be 1-D of one length")
    a, p = _tree(axis, plane, dev)
    if t_start.numel() == 0:  # rays without samples: any readable address will do
        t_start = t_end = torch.zeros(1, dtype=torch.float32, device=dev)
    rays = XLRays(_dev(origins, "origins", torch.float32), _dev(dirs, "dirs", torch.float32),
                  _dev(t_start, "t_start", torch.float32), _dev(t_end, "t_end", torch.float32),
                  _dev(ray_offsets, "ray_offsets", torch.int64), R)
    L = lib()
    old = reuse or {}

    def buf(key, shape, dtype):
        t = old.get(key)
        if t is not None and tuple(t.shape) == shape and t.dtype == dtype and t.device == dev:
            return t
        return torch.empty(shape, dtype=dtype, device=dev)

    wsb = L.xl_pack_workspace_bytes(R, levels)
    ws = buf("workspace", (max(wsb, 1),), torch.uint8)
    npc, nseg = _i64(0), _i64(0)
    _check(L.xl_pack_plan(ctypes.byref(rays), a.data_ptr(), p.data_ptr(), levels, ws.data_ptr(), wsb,
                          ctypes.byref(npc), ctypes.byref(nseg), _stream()))
    n, n_seg = npc.value, nseg.value
    out = dict(t_start=buf("t_start", (n,), torch.float32),
               t_end=buf("t_end", (n,), torch.float32),
               src=buf("src", (n,), torch.int64) if with_src else None,
               seg_offsets=buf("seg_offsets", (n_seg + 1,), torch.int64),
               ray_offsets=buf("ray_offsets", (R + 1,), torch.int64),
               seg_ids=buf("seg_ids", (n_seg,), torch.int64),
               seg_box=buf("seg_box", (n_seg,), torch.int32),
               region_offsets=buf("region_offsets", ((1 << levels) + 1,), torch.int64),
               workspace=ws)
    _check(L.xl_pack_fill(ctypes.byref(rays), a.data_ptr(), p.data_ptr(), levels, ws.data_ptr(), wsb,
                          n_seg, _dev(out["t_start"], "t_start"), _dev(out["t_end"], "t_end"),
                          _dev(out["src"], "src") if with_src else None,
                          _dev(out["seg_offsets"], "seg_offsets"),
                          _dev(out["ray_offsets"], "ray_offsets"), _dev(out["seg_ids"], "seg_ids"),
                          _dev(out["seg_box"], "seg_box"),
                          _dev(out["region_offsets"], "region_offsets"), _stream()))
    return out


def features(sigma, feat, t_start, t_end) -> XLFeatures:
    if sigma.dtype not in DTYPES or feat.dtype != sigma.dtype:
        raise ValueError("sigma and feat must share a storage dtype (float32, bfloat16, float16)")
    n = sigma.shape[0]
    if feat.dim() != 2 or feat.shape[0] != n or t_start.shape != (n,) or t_end.shape != (n,):
        raise ValueError("shapes must be sigma[n], feat[n, F], t_start[n], t_end[n]")
    return XLFeatures(DTYPES[sigma.dtype], feat.shape[1], _dev(sigma, "sigma"), _dev(feat, "feat"),
                      _dev(t_start, "t_start", torch.float32), _dev(t_end, "t_end", torch.float32), n)


def xl_render_features_fwd(sigma, feat, t_start, t_end, seg_offsets, phi_seg=None, tau_seg=None):
    """(phi_seg [F, n_seg], tau_seg [n_seg]) of every segment."""
    f = features(sigma, feat, t_start, t_end)
    n_seg = seg_offsets.shape[0] - 1
    dev = sigma.device
    if phi_seg is None:
        phi_seg = torch.empty((f.n_feat, n_seg), dtype=torch.float32, device=dev)
    if tau_seg is None:
        tau_seg = torch.empty(n_seg, dtype=torch.float32, device=dev)
    _check(lib().xl_render_features_fwd(ctypes.byref(f), _dev(seg_offsets, "seg_offsets", torch.int64),
                                        n_seg, _dev(phi_seg, "phi_seg", torch.float32),
                                        _dev(tau_seg, "tau_seg", torch.float32), _stream()))
    return phi_seg, tau_seg


def xl_merge_features_fwd(tau_seg, phi_seg, ray_offsets, seg_ids, phi_ray=None) -> torch.Tensor:
    """phi_ray [F, n_rays]."""
    F, n_seg = phi_seg.shape
    n_rays = ray_offsets.shape[0] - 1
    if phi_ray is None:
        phi_ray = torch.empty((F, n_rays), dtype=torch.float32, device=phi_seg.device)
    _check(lib().xl_merge_features_fwd(_dev(tau_seg, "tau_seg", torch.float32),
                                       _dev(phi_seg, "phi_seg", torch.float32), F, n_seg,
                                       _dev(ray_offsets, "ray_offsets", torch.int64),
                                       _dev(seg_ids, "seg_ids", torch.int64), n_rays,
                                       _dev(phi_ray, "phi_ray", torch.float32), _stream()))
    return phi_ray


def xl_merge_features_bwd(tau_seg, phi_seg, ray_offsets, seg_ids, grad_ray):
    """(grad_phi_seg [F, n_seg], grad_tau_seg [n_seg]); unlisted segments get 0."""
    F, n_seg = phi_seg.shape
    n_rays = ray_offsets.shape[0] - 1
    gphi = torch.zeros((F, n_seg), dtype=torch.float32, device=phi_seg.device)
    gtau = torch.zeros(n_seg, dtype=torch.float32, device=phi_seg.device)
    _check(lib().xl_merge_features_bwd(_dev(tau_seg, "tau_seg", torch.float32),
                                       _dev(phi_seg, "phi_seg", torch.float32), F, n_seg,
                                       _dev(ray_offsets, "ray_offsets", torch.int64),
                                       _dev(seg_ids, "seg_ids", torch.int64), n_rays,
                                       _dev(grad_ray, "grad_ray", torch.float32),
                                       _dev(gphi, "grad_phi_seg"), _dev(gtau, "grad_tau_seg"), _stream()))
    return gphi, gtau


def xl_render_features_bwd(sigma, feat, t_start, t_end, seg_offsets, phi_seg, grad_phi_seg,
                           grad_tau_seg=None, grad_sigma=None, grad_feat=None,
                           accumulate_sigma: bool = False):
    """(dl/dsigma [n], dl/dfeat [n, F]) in the storage dtype."""
    f = features(sigma, feat, t_start, t_end)
    n_seg = seg_offsets.shape[0] - 1
    if grad_sigma is None:
        if accumulate_sigma:
            raise ValueError("accumulate_sigma needs grad_sigma")
        grad_sigma = torch.empty_like(sigma)
    if grad_feat is None:
        grad_feat = torch.empty_like(feat)
    _check(lib().xl_render_features_bwd(
        ctypes.byref(f), _dev(seg_offsets, "seg_offsets", torch.int64), n_seg,
        _dev(phi_seg, "phi_seg", torch.float32), _dev(grad_phi_seg, "grad_phi_seg", torch.float32),
        None if grad_tau_seg is None else _dev(grad_tau_seg, "grad_tau_seg", torch.float32),
        _dev(grad_sigma, "grad_sigma", sigma.dtype), _dev(grad_feat, "grad_feat", sigma.dtype),
        1 if accumulate_sigma else 0, _stream()))
    return grad_sigma, grad_feat


def breakable(sigma, t_start, t_end, pairs, ch=None, n_ch=None, dtype=None) -> XLBreakable:
    """Descriptor of a breakable-integral member set: loaded channels ch [n, F]
    (sigma's storage dtype), or with ch None the midpoint powers m^0..m^(n_ch-1)."""
    dt = sigma.dtype if dtype is None else dtype
    if dt not in DTYPES:
        raise ValueError("storage dtype must be float32, bfloat16 or float16")
    n = sigma.shape[0]
    if t_start.shape != (n,) or t_end.shape != (n,):
        raise ValueError("shapes must be sigma[n], t_start[n], t_end[n]")
    if ch is not None:
        if ch.dim() != 2 or ch.shape[0] != n or ch.dtype != sigma.dtype:
            raise ValueError("ch must be [n, F] in sigma's dtype")
        F, src, chp = ch.shape[1], XL_CH_LOADED, _dev(ch, "ch")
    else:
        F, src, chp = int(n_ch), XL_CH_MIDPOINT_POWERS, None
    if len(pairs) > 4:
        raise ValueError("at most 4 pairs")
    pa = [a for a, _ in pairs] + [0] * (4 - len(pairs))
    pb = [b for _, b in pairs] + [0] * (4 - len(pairs))
    return XLBreakable(DTYPES[dt], src, F, len(pairs), (_i32 * 4)(*pa), (_i32 * 4)(*pb),
                       _dev(sigma, "sigma"), chp, _dev(t_start, "t_start", torch.float32),
                       _dev(t_end, "t_end", torch.float32), n)


def _rows(d: XLBreakable) -> int:
    return 1 + d.n_ch + d.n_pairs


def xl_render_breakable_fwd(d: XLBreakable, seg_offsets, seg_out=None) -> torch.Tensor:
    """seg_out [1+F+P, n_seg] = (tau, Phi, Psi) of every segment."""
    n_seg = seg_offsets.shape[0] - 1
    if seg_out is None:
        seg_out = torch.empty((_rows(d), n_seg), dtype=torch.float32, device=seg_offsets.device)
    _check(lib().xl_render_breakable_fwd(ctypes.byref(d), _dev(seg_offsets, "seg_offsets", torch.int64),
                                         n_seg, _dev(seg_out, "seg_out", torch.float32), _stream()))
    return seg_out


def xl_merge_breakable_fwd(d: XLBreakable, seg_out, ray_offsets, seg_ids, ray_out=None) -> torch.Tensor:
    """ray_out [1+F+P, n_rays] = (T, Phi, Psi) of every ray."""
    n_seg = seg_out.shape[1]
    n_rays = ray_offsets.shape[0] - 1
    if ray_out is None:
        ray_out = torch.empty((_rows(d), n_rays), dtype=torch.float32, device=seg_out.device)
    _check(lib().xl_merge_breakable_fwd(ctypes.byref(d), _dev(seg_out, "seg_out", torch.float32), n_seg,
                                        _dev(ray_offsets, "ray_offsets", torch.int64),
                                        _dev(seg_ids, "seg_ids", torch.int64), n_rays,
                                        _dev(ray_out, "ray_out", torch.float32), _stream()))
    return ray_out


def xl_merge_breakable_bwd(d: XLBreakable, seg_out, ray_offsets, seg_ids, grad_ray,
                           grad_seg=None) -> torch.Tensor:
    """grad_seg [1+F+P, n_seg] = dl/d(tau, Phi, Psi) of every listed segment."""
    n_seg = seg_out.shape[1]
    n_rays = ray_offsets.shape[0] - 1
    if grad_seg is None:
        grad_seg = torch.zeros((_rows(d), n_seg), dtype=torch.float32, device=seg_out.device)
    _check(lib().xl_merge_breakable_bwd(ctypes.byref(d), _dev(seg_out, "seg_out", torch.float32), n_seg,
                                        _dev(ray_offsets, "ray_offsets", torch.int64),
                                        _dev(seg_ids, "seg_ids", torch.int64), n_rays,
                                        _dev(grad_ray, "grad_ray", torch.float32),
                                        _dev(grad_seg, "grad_seg", torch.float32), _stream()))
    return grad_seg


def xl_render_breakable_bwd(d: XLBreakable, seg_offsets, seg_out, grad_seg, grad_sigma,
                            grad_ch=None, accumulate_sigma: bool = False):
    """Writes dl/dsigma into grad_sigma [n] and, for loaded channels, dl/dch into
    grad_ch [n, F] (storage dtype); returns (grad_sigma, grad_ch)."""
    n_seg = seg_offsets.shape[0] - 1
    _check(lib().xl_render_breakable_bwd(ctypes.byref(d), _dev(seg_offsets, "seg_offsets", torch.int64),
                                         n_seg, _dev(seg_out, "seg_out", torch.float32),
                                         _dev(grad_seg, "grad_seg", torch.float32),
                                         _dev(grad_sigma, "grad_sigma"),
                                         _dev(grad_ch, "grad_ch") if grad_ch is not None else None,
                                         int(accumulate_sigma), _stream()))
    return grad_sigma, grad_ch
