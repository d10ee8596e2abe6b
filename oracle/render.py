"""FP64 CPU oracle for partitioned volume rendering (NeRF-XL, arXiv 2404.16221).

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute this module: only the test suite, the smoke check of the build entry
point and the CPU-baseline leg of the benchmark do.  It shares no code with the
HIP library or its Python binding.

What it computes (plain, slow, obviously correct; float64 throughout):

* ``composite``: the per-sample quadrature of the volume-rendering integral
  (Sec. 4.1, Eq. 1) and of the distortion loss (Sec. 4.1, Eq. 2) over one run of
  samples with transmittance starting at 1.  Readings used (the paper prints no
  discrete form): alpha_i = 1 - exp(-sigma_i delta_i); T_i = exp(-sum_{j<i}
  sigma_j delta_j); w_i = T_i alpha_i; colour C = sum w_i c_i; opacity
  A = sum w_i; unnormalised depth D = sum w_i m_i with m_i the interval
  midpoint; distortion L = sum_i sum_j w_i w_j |m_i - m_j| + 1/3 sum_i w_i^2
  delta_i (the discretisation of Mip-NeRF 360, which the paper cites for
  Eq. 2).  Applied to a segment it gives the partial tuple that a region
  reduces its samples to before any exchange (App. A.2); applied to a whole ray
  it is the single-pass render.
* ``merge``: Eq. 3-8 of Sec. 4.3 written out as sums: the exclusive product of
  segment transmittances (Eq. 4) weights each segment's colour, opacity and
  depth (Eq. 3, 5, 6), and the distortion loss is 2 sum_k T_{<k} S_k + sum_k
  T_{<k}^2 L_k with S_k = D_k A_{<k} - A_k D_{<k} (Eq. 7, 8).  Alg. 2 in
  App. A.2 prints the first term without the factor 2 and takes S from the
  local GPU's tuple; both are slips against Eq. 7/8 and their derivation in
  App. B.1, and the oracle follows Eq. 7/8.
* Gradients: reverse-mode autodiff (PyTorch, CPU, float64) through the plain
  definitions above, i.e. the exact derivative of the definition.  The
  hand-derived closed forms (``grad_*_formula``) are a second, independent
  statement of the same derivative, used only to cross-check.

Tuple conventions: a segment tuple is (tau, r, g, b, A, D, L) where tau is the
segment's optical depth (its transmittance is exp(-tau)); a ray tuple is
(T, r, g, b, A, D, L).  Gradients of a ray tuple are taken with respect to T,
those of a segment tuple with respect to tau.

Pins (tests marked "not gpu"): hand-computed worked examples in
tests/golden/, closed forms for constant density, brute-force double integrals
of step-function weights, the equivalence of any K-split merge with the single
pass, algebraic identities, the paper's sequential Alg. 1/2 loops, and central
finite differences for the gradients.
"""
from __future__ import annotations

import math
from typing import Sequence, Tuple

import numpy as np
import torch

F64 = np.float64
TUPLE = 7  # (T or tau, r, g, b, A, D, L)


# --------------------------------------------------------------------------
# Forward: one run of samples (Sec. 4.1, Eq. 1-2)
# --------------------------------------------------------------------------
def quadrature(sigma, t0, t1):
    """Per-sample quantities of the quadrature: delta, m, tau, alpha, T, w."""
    sigma = np.asarray(sigma, F64)
    t0 = np.asarray(t0, F64)
    t1 = np.asarray(t1, F64)
    delta = t1 - t0
    m = 0.5 * (t0 + t1)
    tau = sigma * delta
    alpha = -np.expm1(-tau)
    excl = np.concatenate([[0.0], np.cumsum(tau)[:-1]]) if tau.size else tau
    T = np.exp(-excl)
    w = T * alpha
    return delta, m, tau, alpha, T, w


def distortion_pairwise(w, m, delta) -> float:
    """O(N^2) distortion: sum_ij w_i w_j |m_i - m_j| + 1/3 sum_i w_i^2 delta_i."""
    w = np.asarray(w, F64)
    m = np.asarray(m, F64)
    delta = np.asarray(delta, F64)
    if w.size == 0:
        return 0.0
    pair = np.abs(m[:, None] - m[None, :])
    return float(w @ pair @ w + (w * w * delta).sum() / 3.0)


def distortion_prefix(w, m, delta) -> float:
    """O(N) form: 2 sum_i w_i (m_i W_{<i} - WM_{<i}) + 1/3 sum_i w_i^2 delta_i."""
    w = np.asarray(w, F64)
    m = np.asarray(m, F64)
    delta = np.asarray(delta, F64)
    if w.size == 0:
        return 0.0
    W = np.concatenate([[0.0], np.cumsum(w)[:-1]])
    WM = np.concatenate([[0.0], np.cumsum(w * m)[:-1]])
    return float(2.0 * (w * (m * W - WM)).sum() + (w * w * delta).sum() / 3.0)


def composite(sigma, rgb, t0, t1) -> np.ndarray:
    """Segment tuple (tau, r, g, b, A, D, L) of one run, transmittance from 1."""
    delta, m, tau, alpha, T, w = quadrature(sigma, t0, t1)
    rgb = np.asarray(rgb, F64).reshape(-1, 3)
    out = np.zeros(TUPLE, F64)
    out[0] = tau.sum()
    out[1:4] = w @ rgb if w.size else 0.0
    out[4] = w.sum()
    out[5] = (w * m).sum()
    out[6] = distortion_pairwise(w, m, delta)
    return out


def to_ray_tuple(seg_tuple: np.ndarray) -> np.ndarray:
    """(tau, ...) -> (T, ...) with T = exp(-tau)."""
    out = np.array(seg_tuple, F64, copy=True)
    out[0] = math.exp(-out[0])
    return out


# --------------------------------------------------------------------------
# Merge of segment tuples in ray order (Sec. 4.3, Eq. 3-8)
# --------------------------------------------------------------------------
def merge(seg_tuples: Sequence[np.ndarray]) -> np.ndarray:
    """Ray tuple (T, r, g, b, A, D, L) from the ray's segment tuples, front to back."""
    K = len(seg_tuples)
    if K == 0:
        out = np.zeros(TUPLE, F64)
        out[0] = 1.0
        return out
    x = np.asarray(seg_tuples, F64).reshape(K, TUPLE)
    Tk = np.exp(-x[:, 0])
    Tpre = np.concatenate([[1.0], np.cumprod(Tk)[:-1]])          # Eq. 4
    C = (Tpre[:, None] * x[:, 1:4]).sum(axis=0)                  # Eq. 3
    A_terms = Tpre * x[:, 4]
    D_terms = Tpre * x[:, 5]
    A = A_terms.sum()                                            # Eq. 5
    D = D_terms.sum()                                            # Eq. 6
    A_pre = np.concatenate([[0.0], np.cumsum(A_terms)[:-1]])     # A(t_1 -> t_k)
    D_pre = np.concatenate([[0.0], np.cumsum(D_terms)[:-1]])     # D(t_1 -> t_k)
    S = x[:, 5] * A_pre - x[:, 4] * D_pre                        # Eq. 8
    L = 2.0 * (Tpre * S).sum() + (Tpre ** 2 * x[:, 6]).sum()     # Eq. 7
    out = np.empty(TUPLE, F64)
    out[0] = float(np.prod(Tk))
    out[1:4] = C
    out[4] = A
    out[5] = D
    out[6] = L
    return out


# --------------------------------------------------------------------------
# Packed batches (region-major samples, CSR segments, per-ray order)
# --------------------------------------------------------------------------
def _f64(a):
    if isinstance(a, torch.Tensor):
        return a.detach().to("cpu", torch.float64).numpy()
    return np.asarray(a, F64)


def render_segments(sigma, rgb, t0, t1, seg_offsets, segs=None) -> np.ndarray:
    """seg_out[7, n_seg] (or for the listed segments): each segment composited alone."""
    sigma, rgb, t0, t1 = _f64(sigma), _f64(rgb).reshape(-1, 3), _f64(t0), _f64(t1)
    seg_offsets = np.asarray(seg_offsets, np.int64)
    segs = np.arange(seg_offsets.shape[0] - 1) if segs is None else np.asarray(segs)
    out = np.zeros((TUPLE, segs.shape[0]), F64)
    for j, s in enumerate(segs):
        a, b = int(seg_offsets[s]), int(seg_offsets[s + 1])
        out[:, j] = composite(sigma[a:b], rgb[a:b], t0[a:b], t1[a:b])
    return out


def ray_index(seg_offsets, ray_offsets, seg_ids, r) -> np.ndarray:
    """Sample indices of ray r, front to back (its segments in the order I)."""
    ids = seg_ids[ray_offsets[r]:ray_offsets[r + 1]]
    parts = [np.arange(seg_offsets[s], seg_offsets[s + 1]) for s in ids]
    return np.concatenate(parts) if parts else np.zeros(0, np.int64)


def render_rays_single(sigma, rgb, t0, t1, seg_offsets, ray_offsets, seg_ids,
                       rays=None) -> np.ndarray:
    """ray_out[7, R] by one pass over each ray's samples (no partitioning)."""
    sigma, rgb, t0, t1 = _f64(sigma), _f64(rgb).reshape(-1, 3), _f64(t0), _f64(t1)
    seg_offsets = np.asarray(seg_offsets, np.int64)
    ray_offsets = np.asarray(ray_offsets, np.int64)
    seg_ids = np.asarray(seg_ids, np.int64)
    rays = np.arange(ray_offsets.shape[0] - 1) if rays is None else np.asarray(rays)
    out = np.zeros((TUPLE, rays.shape[0]), F64)
    for j, r in enumerate(rays):
        idx = ray_index(seg_offsets, ray_offsets, seg_ids, r)
        out[:, j] = to_ray_tuple(composite(sigma[idx], rgb[idx], t0[idx], t1[idx]))
    return out


def render_rays_partitioned(sigma, rgb, t0, t1, seg_offsets, ray_offsets, seg_ids,
                            rays=None) -> Tuple[np.ndarray, np.ndarray]:
    """(seg tuples of the rays' segments, ray_out) for the listed rays, by the
    partitioned path: each segment composited alone, then merged (Eq. 3-8)."""
    seg_offsets = np.asarray(seg_offsets, np.int64)
    ray_offsets = np.asarray(ray_offsets, np.int64)
    seg_ids = np.asarray(seg_ids, np.int64)
    rays = np.arange(ray_offsets.shape[0] - 1) if rays is None else np.asarray(rays)
    segs = np.concatenate([seg_ids[ray_offsets[r]:ray_offsets[r + 1]] for r in rays]) \
        if rays.size else np.zeros(0, np.int64)
    seg_part = render_segments(sigma, rgb, t0, t1, seg_offsets, segs)
    col = {int(s): j for j, s in enumerate(segs)}
    out = np.zeros((TUPLE, rays.shape[0]), F64)
    for j, r in enumerate(rays):
        ids = seg_ids[ray_offsets[r]:ray_offsets[r + 1]]
        out[:, j] = merge([seg_part[:, col[int(s)]] for s in ids])
    return seg_part, out


# --------------------------------------------------------------------------
# Gradients: autodiff of the plain definitions (float64, CPU)
# --------------------------------------------------------------------------
def _composite_t(sigma, rgb, t0, t1):
    """Torch twin of ``composite`` (same definition) for autodiff."""
    delta = t1 - t0
    m = 0.5 * (t0 + t1)
    tau = sigma * delta
    alpha = -torch.expm1(-tau)
    excl = torch.cumsum(tau, 0) - tau
    T = torch.exp(-excl)
    w = T * alpha
    pair = (m[:, None] - m[None, :]).abs()
    L = w @ pair @ w + (w * w * delta).sum() / 3.0
    C = w @ rgb
    return torch.cat([tau.sum().reshape(1), C, w.sum().reshape(1),
                      (w * m).sum().reshape(1), L.reshape(1)])


def _merge_t(x):
    """Torch twin of ``merge`` (Eq. 3-8) for autodiff; x is [K, 7] segment tuples."""
    Tk = torch.exp(-x[:, 0])
    Tpre = torch.cat([x.new_ones(1), torch.cumprod(Tk, 0)[:-1]])
    C = (Tpre[:, None] * x[:, 1:4]).sum(0)
    A_terms = Tpre * x[:, 4]
    D_terms = Tpre * x[:, 5]
    A_pre = torch.cumsum(A_terms, 0) - A_terms
    D_pre = torch.cumsum(D_terms, 0) - D_terms
    S = x[:, 5] * A_pre - x[:, 4] * D_pre
    L = 2.0 * (Tpre * S).sum() + (Tpre ** 2 * x[:, 6]).sum()
    return torch.cat([torch.prod(Tk).reshape(1), C, A_terms.sum().reshape(1),
                      D_terms.sum().reshape(1), L.reshape(1)])


def _t64(a):
    return torch.as_tensor(np.asarray(a, F64), dtype=torch.float64)


def grad_composite(sigma, rgb, t0, t1, g_seg) -> Tuple[np.ndarray, np.ndarray]:
    """d<g_seg, segment tuple>/d(sigma, rgb) for one run (tuple holds tau)."""
    s = _t64(sigma).requires_grad_(True)
    c = _t64(rgb).reshape(-1, 3).requires_grad_(True)
    if s.numel() == 0:
        return np.zeros(0), np.zeros((0, 3))
    y = _composite_t(s, c, _t64(t0), _t64(t1))
    (y * _t64(g_seg)).sum().backward()
    return s.grad.numpy(), c.grad.numpy()


def grad_single(sigma, rgb, t0, t1, g_ray) -> Tuple[np.ndarray, np.ndarray]:
    """d<g_ray, ray tuple>/d(sigma, rgb) for a whole ray in one pass (tuple holds T)."""
    s = _t64(sigma).requires_grad_(True)
    c = _t64(rgb).reshape(-1, 3).requires_grad_(True)
    if s.numel() == 0:
        return np.zeros(0), np.zeros((0, 3))
    y = _composite_t(s, c, _t64(t0), _t64(t1))
    y = torch.cat([torch.exp(-y[:1]), y[1:]])
    (y * _t64(g_ray)).sum().backward()
    return s.grad.numpy(), c.grad.numpy()


def merge_bwd(seg_tuples, g_ray) -> np.ndarray:
    """[K, 7] gradients of <g_ray, merge(seg_tuples)> w.r.t. each segment tuple."""
    K = len(seg_tuples)
    if K == 0:
        return np.zeros((0, TUPLE))
    x = _t64(np.asarray(seg_tuples, F64).reshape(K, TUPLE)).requires_grad_(True)
    (_merge_t(x) * _t64(g_ray)).sum().backward()
    return x.grad.numpy()


def backward_partitioned(sigma, rgb, t0, t1, seg_offsets, ray_offsets, seg_ids,
                         grad_ray, rays=None, autodiff: bool = True):
    """Per-ray gradients by the partitioned path: merge bwd, then each segment's bwd.

    Returns (grad_seg [7, n_listed_segs], segs, {sample index: (dsigma, drgb)} as
    arrays over the listed rays' samples: (idx, dsigma, drgb)).

    autodiff=True differentiates the definitions (``merge_bwd``,
    ``grad_composite``); autodiff=False evaluates the hand-derived closed forms
    (``merge_bwd_formula``, ``grad_composite_formula``) with numpy alone, which
    the tests pin against the autodiff and against finite differences.  Worker
    processes that must not start PyTorch's autograd engine use the latter.
    """
    sigma, rgb, t0, t1 = _f64(sigma), _f64(rgb).reshape(-1, 3), _f64(t0), _f64(t1)
    seg_offsets = np.asarray(seg_offsets, np.int64)
    ray_offsets = np.asarray(ray_offsets, np.int64)
    seg_ids = np.asarray(seg_ids, np.int64)
    grad_ray = np.asarray(grad_ray, F64)
    rays = np.arange(ray_offsets.shape[0] - 1) if rays is None else np.asarray(rays)
    m_bwd = merge_bwd if autodiff else merge_bwd_formula
    s_bwd = grad_composite if autodiff else grad_composite_formula
    g_segs, segs, idx_all, ds_all, dc_all = [], [], [], [], []
    for j, r in enumerate(rays):
        ids = seg_ids[ray_offsets[r]:ray_offsets[r + 1]]
        parts = []
        for s in ids:
            a, b = int(seg_offsets[s]), int(seg_offsets[s + 1])
            parts.append(composite(sigma[a:b], rgb[a:b], t0[a:b], t1[a:b]))
        gk = m_bwd(parts, grad_ray[:, j])
        for q, s in enumerate(ids):
            a, b = int(seg_offsets[s]), int(seg_offsets[s + 1])
            ds, dc = s_bwd(sigma[a:b], rgb[a:b], t0[a:b], t1[a:b], gk[q])
            g_segs.append(gk[q])
            segs.append(int(s))
            idx_all.append(np.arange(a, b))
            ds_all.append(ds)
            dc_all.append(dc)
    cat = (lambda xs, shape: np.concatenate(xs) if xs else np.zeros(shape))
    return (np.asarray(g_segs, F64).reshape(-1, TUPLE).T, np.asarray(segs, np.int64),
            cat(idx_all, (0,)).astype(np.int64), cat(ds_all, (0,)), cat(dc_all, (0, 3)))


# --------------------------------------------------------------------------
# Hand-derived gradient formulas (independent cross-check of the autodiff)
# --------------------------------------------------------------------------
def grad_composite_formula(sigma, rgb, t0, t1, g_seg):
    """Closed form of ``grad_composite``.

    With v_j = g_C.c_j + g_A + g_D m_j + g_L u_j and
    u_j = dL/dw_j = 2 sum_i w_i |m_j - m_i| + 2/3 w_j delta_j:
      dsigma_i = delta_i [g_tau + T_{i+1} v_i - sum_{j>i} w_j v_j],
      drgb_i   = w_i g_C.
    """
    delta, m, tau, alpha, T, w = quadrature(sigma, t0, t1)
    rgb = np.asarray(rgb, F64).reshape(-1, 3)
    g = np.asarray(g_seg, F64)
    g_tau, g_C, g_A, g_D, g_L = g[0], g[1:4], g[4], g[5], g[6]
    u = 2.0 * (np.abs(m[:, None] - m[None, :]) @ w) + (2.0 / 3.0) * w * delta
    v = rgb @ g_C + g_A + g_D * m + g_L * u
    wv = w * v
    suffix = np.concatenate([np.cumsum(wv[::-1])[::-1][1:], [0.0]]) if w.size else wv
    T_next = T * np.exp(-tau)
    dsigma = delta * (g_tau + T_next * v - suffix)
    drgb = w[:, None] * g_C[None, :]
    return dsigma, drgb


def merge_bwd_formula(seg_tuples, g_ray) -> np.ndarray:
    """Closed form of ``merge_bwd`` from the exclusive prefix P and suffix S folds.

    For segment k with tuple x and P = x_1 (+) ... (+) x_{k-1}, S = x_{k+1} (+) ...:
      g_C^k = P_T g_C, g_L^k = P_T^2 g_L,
      g_A^k = P_T [g_A + 2 g_L (P_T T_k S_D - P_D)],
      g_D^k = P_T [g_D + 2 g_L (P_A - P_T T_k S_A)],
      g_T^k = P_T g_T S_T + P_T g_C.S_C + (P_T g_A - 2 g_L P_T P_D) S_A
              + (P_T g_D + 2 g_L P_T P_A) S_D
              + g_L P_T^2 (2 T_k S_L + 2 (S_D A_k - S_A D_k)),
      g_tau^k = -T_k g_T^k.
    """
    K = len(seg_tuples)
    x = np.asarray(seg_tuples, F64).reshape(K, TUPLE)
    g = np.asarray(g_ray, F64)
    gT, gC, gA, gD, gL = g[0], g[1:4], g[4], g[5], g[6]
    out = np.zeros((K, TUPLE))
    for k in range(K):
        P = merge(list(x[:k]))
        S = merge(list(x[k + 1:]))
        Tk, Ak, Dk = math.exp(-x[k, 0]), x[k, 4], x[k, 5]
        PT, PA, PD = P[0], P[4], P[5]
        ST, SC, SA, SD, SL = S[0], S[1:4], S[4], S[5], S[6]
        out[k, 1:4] = PT * gC
        out[k, 6] = gL * PT * PT
        out[k, 4] = PT * (gA + 2.0 * gL * (PT * Tk * SD - PD))
        out[k, 5] = PT * (gD + 2.0 * gL * (PA - PT * Tk * SA))
        gTk = (PT * gT * ST + PT * float(gC @ SC) + (PT * gA - 2.0 * gL * PT * PD) * SA
               + (PT * gD + 2.0 * gL * PT * PA) * SD
               + gL * PT * PT * (2.0 * Tk * SL + 2.0 * (SD * Ak - SA * Dk)))
        out[k, 0] = -Tk * gTk
    return out
