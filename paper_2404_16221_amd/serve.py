"""ctypes binding of the render server (xl_serve_* in include/xl.h)."""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import torch

from . import _lib
from ._lib import XLError, _check, _stream, lib

_c = ctypes
_i32, _i64, _u64, _dbl, _vp = _c.c_int32, _c.c_int64, _c.c_uint64, _c.c_double, _c.c_void_p


class XLServeConfig(_c.Structure):
    _fields_ = [("hbm_budget_bytes", _u64), ("max_slots", _i32), ("max_queue", _i32),
                ("device", _i32), ("dtype", _i32), ("merge_fp64", _i32), ("reserved", _i32)]


class XLRequest(_c.Structure):
    _fields_ = [("width", _i32), ("height", _i32), ("grid", _i32 * 3), ("n_min", _i32),
                ("n_max", _i32), ("inject_fault", _i32), ("sigma_mu", _dbl), ("sigma_s", _dbl),
                ("zero_frac", _dbl), ("width_mean", _dbl), ("t_far", _dbl), ("seed", _u64)]


class XLResult(_c.Structure):
    _fields_ = [("status", _i32), ("reserved", _i32), ("ray_out", _vp), ("n_rays", _i64),
                ("n_samples", _i64), ("n_segments", _i64), ("footprint_bytes", _u64),
                ("latency_us", _i64), ("queue_us", _i64), ("device_us", _i64),
                ("device_start_us", _i64), ("device_end_us", _i64)]


class XLServeStats(_c.Structure):
    _fields_ = [("completed", _i64), ("failed", _i64), ("queued", _i64), ("samples", _i64),
                ("budget_used_bytes", _u64), ("p50_latency_us", _i64), ("p99_latency_us", _i64),
                ("max_latency_us", _i64), ("span_us", _i64)]


_P = _c.POINTER
SERVE_SIGNATURES = {
    "xl_serve_create": (_c.c_int, [_P(XLServeConfig), _P(_vp)]),
    "xl_serve_submit": (_c.c_int, [_vp, _P(XLRequest), _P(_u64)]),
    "xl_serve_poll": (_c.c_int, [_vp, _u64, _P(XLResult), _i64]),
    "xl_serve_copy_result": (_c.c_int, [_vp, _u64, _vp, _vp]),
    "xl_serve_release": (_c.c_int, [_vp, _u64]),
    "xl_serve_stats_get": (_c.c_int, [_vp, _P(XLServeStats)]),
    "xl_serve_destroy": (_c.c_int, [_vp]),
}
_bound = False


def _bind():
    global _bound
    if not _bound:
        L = lib()
        for name, (res, args) in SERVE_SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _bound = True
    return lib()


def request(width: int, height: int, grid: Sequence[int] = (4, 4, 2), n_min: int = 16,
            n_max: int = 512, sigma_mu: float = 0.0, sigma_s: float = 1.5, zero_frac: float = 0.0,
            seed: int = 0, inject_fault: bool = False, width_mean: float = 0.02,
            t_far: float = 3.0) -> XLRequest:
    return XLRequest(width, height, (_i32 * 3)(*grid), n_min, n_max, int(inject_fault), sigma_mu,
                     sigma_s, zero_frac, width_mean, t_far, seed)


class Server:
    """A render server on one GPU; see xl_serve_create."""

    def __init__(self, hbm_budget_bytes: int = 64 << 30, max_slots: int = 4, max_queue: int = 1024,
                 device: int = 0, dtype=torch.float16, merge_fp64: bool = False):
        L = _bind()
        self.cfg = XLServeConfig(hbm_budget_bytes, max_slots, max_queue, device,
                                 _lib.storage_code(*_lib.storage_dtypes(dtype)), int(merge_fp64), 0)
        h = _vp()
        _check(L.xl_serve_create(ctypes.byref(self.cfg), ctypes.byref(h)))
        self.h = h

    def submit(self, req: XLRequest) -> Optional[int]:
        """Ticket, or None when the queue is full (XL_EAGAIN)."""
        t = _u64()
        rc = lib().xl_serve_submit(self.h, ctypes.byref(req), ctypes.byref(t))
        if rc == _lib.XL_EAGAIN:
            return None
        _check(rc)
        return t.value

    def poll(self, ticket: int, timeout_us: int = -1) -> dict:
        r = XLResult()
        rc = lib().xl_serve_poll(self.h, ticket, ctypes.byref(r), timeout_us)
        out = {k: getattr(r, k) for k, _ in XLResult._fields_ if k not in ("reserved",)}
        out["rc"] = rc
        if rc not in (_lib.XL_OK, _lib.XL_PENDING):
            out["error"] = lib().xl_last_error().decode()
        return out

    def result(self, ticket: int, n_rays: int, device="cuda") -> torch.Tensor:
        dst = torch.empty((7, n_rays), dtype=torch.float32, device=device)
        _check(lib().xl_serve_copy_result(self.h, ticket, dst.data_ptr(), _stream()))
        return dst

    def release(self, ticket: int) -> None:
        _check(lib().xl_serve_release(self.h, ticket))

    def stats(self) -> dict:
        s = XLServeStats()
        _check(lib().xl_serve_stats_get(self.h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in XLServeStats._fields_}

    def close(self) -> None:
        if self.h:
            _check(lib().xl_serve_destroy(self.h))
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
