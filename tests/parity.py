"""Helpers for GPU-vs-oracle parity tests: device upload and tolerance checks.

Tolerances (FP32 path, the 1e-5 relative bar with explicit floors):
  * colour and opacity (values in [0, 1]):  |x - x64| <= 1e-5 |x64| + 1e-8
  * depth and distortion (t <= 3):          |x - x64| <= 1e-5 |x64| + 3e-8
  * transmittance is judged through tau = -log T:
        |tau - tau64| <= 1e-5 tau64 + 1e-7  (1e-7 ~ one FP32 ulp of T near 1);
    where tau64 > 80 (T below FP32's normal range) T must be < 1e-34
  * gradients: |g - g64| <= 1e-5 |g64| + 1e-6 max|g64| per element and
    ||g - g64|| <= 1e-5 ||g64||.  The 1e-6 floor (about 16 FP32 ulps of the
    largest gradient) covers elements that are differences of terms of the
    size of the largest gradient (moving weight between samples), whose FP32
    rounding is absolute, not relative.
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import dataclass

import numpy as np
import torch

RTOL = 1e-5
ATOL = np.array([0.0, 1e-8, 1e-8, 1e-8, 1e-8, 3e-8, 3e-8])
TAU_ATOL = 1e-7


@dataclass
class Dev:
    sigma: torch.Tensor
    rgb: torch.Tensor
    t0: torch.Tensor
    t1: torch.Tensor
    seg_offsets: torch.Tensor
    ray_offsets: torch.Tensor
    seg_ids: torch.Tensor


# Mixed 16-bit storage: densities in bfloat16, colours in float16.
BF16_F16 = (torch.bfloat16, torch.float16)


def dtypes_of(dtype):
    """(sigma dtype, rgb dtype) of a storage given as one dtype or a pair."""
    return tuple(dtype) if isinstance(dtype, (tuple, list)) else (dtype, dtype)


def storage_name(dtype):
    s, c = dtypes_of(dtype)
    return str(s)[6:] if s == c else f"{str(s)[6:]}-sigma/{str(c)[6:]}-rgb"


def grad_ulps(dtype):
    """Unit roundoff of the stored dsigma and drgb (None for float32)."""
    u = {torch.bfloat16: 2.0 ** -8, torch.float16: 2.0 ** -11, torch.float32: None}
    s, c = dtypes_of(dtype)
    return u[s], u[c]


def to_dev(b, dtype=torch.float32, device="cuda") -> Dev:
    sdt, cdt = dtypes_of(dtype)

    def T(a, dt=None):
        t = torch.from_numpy(np.ascontiguousarray(a))
        return t.to(device=device, dtype=dt) if dt is not None else t.to(device)
    return Dev(T(b.sigma, sdt), T(b.rgb, cdt), T(b.t_start), T(b.t_end), T(b.seg_offsets),
               T(b.ray_offsets), T(b.seg_ids))


def quantize(b, dtype):
    """Host copies of sigma, rgb rounded to their storage types (round to
    nearest even) and back."""
    sdt, cdt = dtypes_of(dtype)
    s = torch.from_numpy(b.sigma).to(sdt).to(torch.float32).numpy()
    c = torch.from_numpy(b.rgb).to(cdt).to(torch.float32).numpy()
    return s, c


def tuple_report(got, ref, kind: str, rtol=RTOL, atol=ATOL):
    """Per-component errors of [7, N] tuples.

    kind = "seg": component 0 is tau; kind = "ray": component 0 is T, judged
    through tau = -log T.  Returns worst normalised error (<= 1 passes), the
    largest absolute error, the largest relative error over the elements the
    relative bar governs (rtol |ref| >= floor), and how many elements the floor
    governs instead.
    """
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    rep = {"norm": np.zeros(7), "rel": np.zeros(7), "abs": np.zeros(7), "floored": np.zeros(7, int),
           "n": ref.shape[1]}
    if ref.shape[1] == 0:
        return rep

    def rel_governed(err, r, floor):
        gov = rtol * np.abs(r) >= floor
        return (float((err[gov] / np.abs(r[gov])).max()) if gov.any() else 0.0), int((~gov).sum())

    if kind == "ray":
        with np.errstate(divide="ignore"):
            tau_ref = -np.log(ref[0])
            tau_got = -np.log(np.maximum(got[0], 1e-300))
        deep = tau_ref > 80.0
        lim = rtol * tau_ref + TAU_ATOL
        e = np.where(deep, 0.0, np.abs(tau_got - tau_ref) / np.where(deep, 1.0, lim))
        e = np.where(deep & (got[0] >= 1e-34), np.inf, e)
        rep["norm"][0] = e.max()
        ok = ~deep
        rep["rel"][0], rep["floored"][0] = rel_governed(np.abs(tau_got - tau_ref)[ok], tau_ref[ok],
                                                        TAU_ATOL)
        rep["abs"][0] = np.abs(got[0] - ref[0]).max()
    else:
        err = np.abs(got[0] - ref[0])
        rep["norm"][0] = (err / (rtol * np.abs(ref[0]) + TAU_ATOL)).max()
        rep["rel"][0], rep["floored"][0] = rel_governed(err, ref[0], TAU_ATOL)
        rep["abs"][0] = err.max()
    for k in range(1, 7):
        err = np.abs(got[k] - ref[k])
        rep["norm"][k] = (err / (rtol * np.abs(ref[k]) + atol[k])).max()
        rep["rel"][k], rep["floored"][k] = rel_governed(err, ref[k], atol[k])
        rep["abs"][k] = err.max()
    return rep


def assert_tuples(got, ref, kind, what="", **kw):
    rep = tuple_report(got, ref, kind, **kw)
    names = ["T" if kind == "ray" else "tau", "r", "g", "b", "A", "D", "L"]
    msg = f"{what}: worst normalised error " + ", ".join(
        f"{n}={v:.3g}" for n, v in zip(names, rep["norm"])) + "; max rel " + ", ".join(
        f"{n}={v:.3g}" for n, v in zip(names, rep["rel"]))
    record(what, {n: {"max_abs": float(a), "max_rel": float(r), "floored": int(f)}
                  for n, a, r, f in zip(names, rep["abs"], rep["rel"], rep["floored"])},
           n=int(rep["n"]), worst_normalised=float(rep["norm"].max()))
    assert np.all(rep["norm"] <= 1.0), msg
    return rep


def grad_report(got, ref, rtol=RTOL, floor=1e-6):
    """Worst normalised error (<= 1 passes), norm-wise relative error, and the
    unfloored maxima: largest absolute error, largest relative error over the
    elements the relative bar governs, and how many elements the floor governs
    (floor * max|ref| > rtol * |ref|)."""
    got = np.asarray(got, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    rep = {"norm": 0.0, "normwise": 0.0, "max_abs": 0.0, "max_rel": 0.0, "floored": 0,
           "max_ref": 0.0, "n": int(ref.size)}
    if ref.size == 0:
        return rep
    s = np.abs(ref).max()
    err = np.abs(got - ref)
    lim = rtol * np.abs(ref) + floor * s
    rep["norm"] = float((err / np.where(lim > 0, lim, 1.0)).max()) if s > 0 else float(np.abs(got).max())
    rep["normwise"] = float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))
    rep["max_abs"] = float(err.max())
    rep["max_ref"] = float(s)
    rel_gov = rtol * np.abs(ref) >= floor * s
    rep["floored"] = int((~rel_gov).sum())
    if rel_gov.any():
        rep["max_rel"] = float((err[rel_gov] / np.abs(ref[rel_gov])).max())
    return rep


def assert_grads(got, ref, what="", rtol=RTOL, floor=1e-6, norm_tol=1e-5):
    rep = grad_report(got, ref, rtol, floor)
    record(what, {k: rep[k] for k in ("max_abs", "max_rel", "floored", "normwise", "max_ref")},
           n=rep["n"], worst_normalised=rep["norm"])
    assert rep["norm"] <= 1.0 and rep["normwise"] <= norm_tol, \
        f"{what}: worst normalised {rep['norm']:.3g}, norm-wise rel {rep['normwise']:.3g}"
    return rep


def record(what, errors, **extra):
    """Append one comparison's measured errors to the JSON-lines file named by
    XL_ERRORS_LOG (nothing is written when it is unset)."""
    path = os.environ.get("XL_ERRORS_LOG")
    if not path or not what:
        return
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "a") as f:
        f.write(json.dumps({"what": what, **extra, "errors": errors}) + "\n")


def sample_rays(n_rays, k, seed):
    rng = np.random.default_rng(seed)
    k = min(k, n_rays)
    return np.sort(rng.choice(n_rays, size=k, replace=False))
