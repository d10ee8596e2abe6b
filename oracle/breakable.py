"""FP64 CPU oracle for breakable integrals composited across regions (App. B.2).

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute this module: only the test suite, the smoke check of the build entry
point and the CPU-baseline leg of the benchmark do.  It shares no code with the
HIP library or its Python binding, and none with oracle/render.py.

App. B.2 calls an integral over [t_1, t_{N+1}] breakable when it is a sum of
products of per-segment factors, so that each region can evaluate its own
segment and only per-ray data is combined.  Property 1: sums and products of
breakable integrals are breakable.  Property 2: integrating a breakable F
against any f, A = int F(t_1 -> t) f(t) dt, is breakable again.  The Examples
subsection builds the transmittance, the volume-rendering equation and the
distortion loss from these two rules.  This oracle implements the family the
two rules generate from the transmittance, up to one level of nesting:

* first order (Property 2 once, F = T sigma):
      Phi_c = int T(t_1 -> t) sigma(t) f_c(t) dt,        c = 0 .. F-1
* second order (Property 2 on Property 1's product T * Phi_b, then Property 2
  again), for pairs p = (a_p, b_p) of channels:
      Psi_p = int w(u) f_a(u) [ int_{t_1}^{u} w(v) f_b(v) dv ] du,   w = T sigma.
  The distortion loss of the Examples is 2 (Psi_(m,1) - Psi_(1,m)) with
  channels 1 and m (the sample position), plus the within-sample term of its
  discretisation.

Discretisation (the colour path's quadrature: piecewise-constant density,
and channels constant over each sample interval): w_i = T_i (1 - exp(-tau_i))
with T_i = exp(-sum_{j<i} tau_j), tau_i = sigma_i (t_end - t_start), and
      Phi_c = sum_i w_i f_ci
      Psi_p = sum_i sum_{j<i} w_i a_i w_j b_j  +  1/2 sum_i w_i^2 a_i b_i.
The last term is exact, not a model: over one interval of constant channels,
the part of the double integral with v < u is half the square of the
interval's weight, whatever the weight's shape inside it.

Merge of a ray's segments in order (what the proof of Property 2 does with its
terms S_1 and S_2), with P_k = prod_{j<k} exp(-tau_j):
      T     = prod_k exp(-tau_k)
      Phi_c = sum_k P_k Phi_ck
      Psi_p = sum_k P_k^2 Psi_pk + sum_k P_k Phi_(a_p)k sum_{j<k} P_j Phi_(b_p)j.

Gradients: float64 autodiff (PyTorch, CPU) through these plain definitions.

Channel sources: a loaded [n, F] array, or the powers of the sample midpoint
m^0 .. m^(F-1) (formed from the interval ends; they carry no gradient).
"""
from __future__ import annotations

from typing import Sequence, Tuple

import numpy as np
import torch

F64 = np.float64


def _rows(ch, n) -> np.ndarray:
    """Channels as an [n, F] float64 array."""
    ch = np.asarray(ch, F64)
    return ch.reshape(n, ch.shape[-1] if ch.ndim == 2 else -1)


def midpoint_powers(t0, t1, F: int) -> np.ndarray:
    """Channels m^0 .. m^(F-1) of every sample, m the interval midpoint."""
    m = 0.5 * (np.asarray(t0, F64) + np.asarray(t1, F64))
    return np.stack([m ** c for c in range(F)], axis=1) if F else np.zeros((m.size, 0))


def segment(sigma, ch, t0, t1, pairs) -> np.ndarray:
    """(tau, Phi_0..Phi_{F-1}, Psi_0..Psi_{P-1}) of one run of samples, T from 1."""
    sigma = np.asarray(sigma, F64)
    ch = _rows(ch, sigma.size)
    t0 = np.asarray(t0, F64)
    t1 = np.asarray(t1, F64)
    F, P = ch.shape[1], len(pairs)
    out = np.zeros(1 + F + P, F64)
    n = sigma.size
    tau = sigma * (t1 - t0)
    out[0] = tau.sum()
    T = 1.0
    w = np.zeros(n)
    for i in range(n):
        w[i] = T * -np.expm1(-tau[i])
        T *= np.exp(-tau[i])
    for c in range(F):
        out[1 + c] = (w * ch[:, c]).sum()
    for p, (a, b) in enumerate(pairs):
        s = 0.0
        inner = 0.0  # sum_{j<i} w_j b_j
        for i in range(n):
            s += w[i] * ch[i, a] * inner + 0.5 * w[i] * w[i] * ch[i, a] * ch[i, b]
            inner += w[i] * ch[i, b]
        out[1 + F + p] = s
    return out


def merge(seg_tuples: Sequence[np.ndarray], F: int, pairs) -> np.ndarray:
    """Ray tuple (T, Phi, Psi) from the ray's segment tuples, front to back."""
    P = len(pairs)
    x = np.asarray(seg_tuples, F64).reshape(-1, 1 + F + P)
    K = x.shape[0]
    out = np.zeros(1 + F + P, F64)
    Pk = np.ones(K)
    for k in range(1, K):
        Pk[k] = Pk[k - 1] * np.exp(-x[k - 1, 0])
    out[0] = float(np.prod(np.exp(-x[:, 0]))) if K else 1.0
    for c in range(F):
        out[1 + c] = (Pk * x[:, 1 + c]).sum()
    for p, (a, b) in enumerate(pairs):
        s = 0.0
        for k in range(K):
            s += Pk[k] ** 2 * x[k, 1 + F + p]
            s += Pk[k] * x[k, 1 + a] * sum(Pk[j] * x[j, 1 + b] for j in range(k))
        out[1 + F + p] = s
    return out


def single(sigma, ch, t0, t1, pairs) -> np.ndarray:
    """The ray in one pass: (T, Phi, Psi) of all its samples in t order."""
    out = segment(sigma, ch, t0, t1, pairs)
    out[0] = np.exp(-out[0])
    return out


# ---------------------------------------------------------------- packed batches
def render_rays(sigma, ch, t0, t1, seg_offsets, ray_offsets, seg_ids, pairs,
                rays=None) -> Tuple[np.ndarray, np.ndarray]:
    """(segment tuples [1+F+P, n_seg], ray tuples [1+F+P, R] by the merge)."""
    ch = _rows(ch, np.asarray(sigma).size)
    F = ch.shape[1]
    seg_offsets = np.asarray(seg_offsets, np.int64)
    ray_offsets = np.asarray(ray_offsets, np.int64)
    seg_ids = np.asarray(seg_ids, np.int64)
    n_seg = seg_offsets.size - 1
    seg = np.zeros((1 + F + len(pairs), n_seg))
    for s in range(n_seg):
        a, b = seg_offsets[s], seg_offsets[s + 1]
        seg[:, s] = segment(sigma[a:b], ch[a:b], t0[a:b], t1[a:b], pairs)
    rays = np.arange(ray_offsets.size - 1) if rays is None else np.asarray(rays)
    ray = np.zeros((seg.shape[0], rays.size))
    for j, r in enumerate(rays):
        ray[:, j] = merge([seg[:, s] for s in seg_ids[ray_offsets[r]:ray_offsets[r + 1]]], F, pairs)
    return seg, ray


# ---------------------------------------------------------------- gradients
def _segment_t(sigma, ch, t0, t1, pairs):
    """Torch twin of ``segment`` (same definition, vectorised) for autodiff."""
    tau = sigma * (t1 - t0)
    T = torch.exp(-(torch.cumsum(tau, 0) - tau))
    w = T * -torch.expm1(-tau)
    parts = [tau.sum().reshape(1), w @ ch]
    for a, b in pairs:
        wa, wb = w * ch[:, a], w * ch[:, b]
        excl = torch.cumsum(wb, 0) - wb
        parts.append(((wa * excl).sum() + 0.5 * (wa * wb).sum()).reshape(1))
    return torch.cat(parts)


def _merge_t(x, F, pairs):
    """Torch twin of ``merge`` for autodiff; x is [K, 1+F+P]."""
    e = torch.exp(-x[:, 0])
    Pk = torch.cat([x.new_ones(1), torch.cumprod(e, 0)[:-1]])
    parts = [torch.prod(e).reshape(1), Pk @ x[:, 1:1 + F]]
    for p, (a, b) in enumerate(pairs):
        fb = Pk * x[:, 1 + b]
        excl = torch.cumsum(fb, 0) - fb
        parts.append(((Pk ** 2) @ x[:, 1 + F + p] + (Pk * x[:, 1 + a]) @ excl).reshape(1))
    return torch.cat(parts)


def _t(a):
    return torch.as_tensor(np.asarray(a, F64), dtype=torch.float64)


def backward(sigma, ch, t0, t1, seg_offsets, ray_offsets, seg_ids, pairs, grad_ray,
             channels_have_grad=True):
    """d<grad_ray, ray tuples>/d(sigma, ch) through the partitioned path (each
    segment composited alone, then merged), plus dl/d(segment tuples).

    Returns (grad_seg [1+F+P, n_seg], dsigma [n], dch [n, F] or None).
    """
    s = _t(sigma).requires_grad_(True)
    c = _t(_rows(ch, s.numel())).requires_grad_(channels_have_grad)
    F = c.shape[1]
    a_t, b_t = _t(t0), _t(t1)
    seg_offsets = np.asarray(seg_offsets, np.int64)
    ray_offsets = np.asarray(ray_offsets, np.int64)
    seg_ids = np.asarray(seg_ids, np.int64)
    n_seg = seg_offsets.size - 1
    segs = []
    for k in range(n_seg):
        a, b = int(seg_offsets[k]), int(seg_offsets[k + 1])
        segs.append(_segment_t(s[a:b], c[a:b], a_t[a:b], b_t[a:b], pairs))
    seg = torch.stack(segs, 1) if segs else torch.zeros((1 + F + len(pairs), 0), dtype=torch.float64)
    seg.retain_grad()
    g = _t(grad_ray)
    loss = torch.zeros((), dtype=torch.float64)
    for r in range(ray_offsets.size - 1):
        ids = seg_ids[ray_offsets[r]:ray_offsets[r + 1]]
        if ids.size == 0:
            continue
        loss = loss + (_merge_t(seg[:, torch.as_tensor(ids)].T, F, pairs) * g[:, r]).sum()
    if loss.requires_grad:
        loss.backward()
    gs = s.grad.numpy() if s.grad is not None else np.zeros(s.numel())
    gc = (c.grad.numpy() if c.grad is not None else np.zeros(c.shape)) if channels_have_grad else None
    gseg = seg.grad.numpy() if seg.grad is not None else np.zeros(seg.shape)
    return gseg, gs, gc
