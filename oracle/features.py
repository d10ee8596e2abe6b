"""FP64 CPU oracle for feature channels composited across regions (NeRF-XL,
arXiv 2404.16221, App. B.2).

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute this module: only the test suite, the smoke check of the build entry
point and the CPU-baseline leg of the benchmark do.  It shares no code with the
HIP library or its Python binding (nor with oracle/render.py).

What it computes (plain, slow, float64):

App. B.2 defines breakable integrals -- those that split over ray segments into
sums of products of per-segment terms -- and shows (Property 2) that if F is
breakable then so is the integral over the ray of F(start -> t) f(t) dt.  With
F the transmittance (breakable: a product over segments) and f = sigma times a
per-sample feature vector, this gives feature compositing: any quantity
rendered with the volume-rendering weights (colour, semantic logits, normals,
the squared depth of a variance estimate) splits over regions exactly like
colour:

* ``feature_segment``: Phi_k = sum_i w_i f_i over one segment's samples, with
  the quadrature of the colour path (alpha_i = 1 - exp(-sigma_i delta_i),
  T_i = exp(-sum_{j<i} sigma_j delta_j) from 1 at the segment start,
  w_i = T_i alpha_i), and the segment's optical depth tau_k;
* ``merge_features``: Phi_ray = sum_k exp(-sum_{j<k} tau_j) Phi_k over the
  ray's segments front to back (Property 2: the product of the earlier
  segments' transmittances times the segment's own integral);
* gradients: reverse-mode autodiff (PyTorch, CPU, float64) through these
  definitions, with respect to sigma and the features.

Pins (tests marked "not gpu"): with the colour as the feature the result is
the colour of oracle/render.py; constant density and feature give
f (1 - exp(-sigma L)); any split of a ray into segments merges to the
single-segment value; the gradients match central finite differences.
"""
from __future__ import annotations

import numpy as np
import torch

F64 = np.float64


def feature_segment(sigma, feat, t0, t1):
    """(tau, Phi[F]) of one run of samples, transmittance from 1 at its start."""
    sigma = np.asarray(sigma, F64)
    feat = np.asarray(feat, F64)  # [n, F]
    delta = np.asarray(t1, F64) - np.asarray(t0, F64)
    phi = np.zeros(feat.shape[1], F64)
    depth = 0.0
    for i in range(sigma.shape[0]):
        T = np.exp(-depth)
        alpha = 1.0 - np.exp(-sigma[i] * delta[i])
        phi += T * alpha * feat[i]
        depth += sigma[i] * delta[i]
    return depth, phi


def render_feature_segments(sigma, feat, t0, t1, seg_offsets):
    """tau [n_seg], Phi [n_seg, F] of every segment."""
    n_seg = len(seg_offsets) - 1
    F = np.asarray(feat).shape[1]
    tau = np.zeros(n_seg, F64)
    phi = np.zeros((n_seg, F), F64)
    for k in range(n_seg):
        a, b = int(seg_offsets[k]), int(seg_offsets[k + 1])
        tau[k], phi[k] = feature_segment(sigma[a:b], np.asarray(feat)[a:b], t0[a:b], t1[a:b])
    return tau, phi


def merge_features(tau, phi, ray_offsets, seg_ids):
    """Phi_ray [R, F]: segments front to back, each weighted by the
    transmittance of the segments before it."""
    R = len(ray_offsets) - 1
    out = np.zeros((R, phi.shape[1]), F64)
    for r in range(R):
        before = 0.0
        for s in seg_ids[int(ray_offsets[r]):int(ray_offsets[r + 1])]:
            out[r] += np.exp(-before) * phi[s]
            before += tau[s]
    return out


def render_features(sigma, feat, t0, t1, seg_offsets, ray_offsets, seg_ids):
    """Per-segment (tau, Phi) and per-ray Phi of a packed batch."""
    tau, phi = render_feature_segments(sigma, feat, t0, t1, seg_offsets)
    return tau, phi, merge_features(tau, phi, ray_offsets, seg_ids)


def grad_features(sigma, feat, t0, t1, seg_offsets, ray_offsets, seg_ids, g_ray):
    """(dl/dsigma [n], dl/dfeat [n, F]) of l = sum(g_ray * Phi_ray) by float64
    autodiff through the definitions above (written again in torch ops)."""
    s = torch.tensor(np.asarray(sigma, F64), requires_grad=True)
    f = torch.tensor(np.asarray(feat, F64), requires_grad=True)
    d = torch.tensor(np.asarray(t1, F64) - np.asarray(t0, F64))
    n_seg = len(seg_offsets) - 1
    taus, phis = [], []
    for k in range(n_seg):
        a, b = int(seg_offsets[k]), int(seg_offsets[k + 1])
        od = s[a:b] * d[a:b]
        excl = torch.cumsum(od, 0) - od
        w = torch.exp(-excl) * (1.0 - torch.exp(-od))
        phis.append((w[:, None] * f[a:b]).sum(0) if b > a else torch.zeros(f.shape[1], dtype=torch.float64))
        taus.append(od.sum() if b > a else torch.zeros((), dtype=torch.float64))
    g = torch.tensor(np.asarray(g_ray, F64))
    loss = torch.zeros((), dtype=torch.float64)
    for r in range(len(ray_offsets) - 1):
        before = torch.zeros((), dtype=torch.float64)
        for sid in seg_ids[int(ray_offsets[r]):int(ray_offsets[r + 1])]:
            loss = loss + torch.exp(-before) * (phis[sid] * g[r]).sum()
            before = before + taus[sid]
    if loss.requires_grad:
        loss.backward()
    gs = s.grad.numpy() if s.grad is not None else np.zeros(len(sigma))
    gf = f.grad.numpy() if f.grad is not None else np.zeros(f.shape)
    return gs, gf
