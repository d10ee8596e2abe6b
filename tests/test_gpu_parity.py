"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle."""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import render as O
from paper_2404_16221_amd import _lib as xl
from paper_2404_16221_amd import synth
from paper_2404_16221_amd.autograd import render
from tests.parity import (BF16_F16, Dev, assert_grads, assert_tuples, grad_ulps, quantize,
                          sample_rays, storage_name, to_dev, tuple_report)

pytestmark = pytest.mark.gpu

_CACHE = {}


def gen(cfg, n_rays=None, plain=False):
    key = (cfg, n_rays, plain)
    if key not in _CACHE:
        w = synth.WORKLOADS[cfg]
        if plain:
            w = w.plain()
        rays = None if n_rays is None else np.arange(n_rays)
        _CACHE[key] = synth.generate(w, rays=rays)
    return _CACHE[key]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_fwd(d: Dev, fp64=False):
    seg_out, ws = xl.xl_render_segments_fwd(d.sigma, d.rgb, d.t0, d.t1, d.seg_offsets)
    ray_out = xl.xl_merge_fwd(seg_out, d.ray_offsets, d.seg_ids, fp64=fp64)
    torch.cuda.synchronize()
    return seg_out, ws, ray_out


def run_bwd(d: Dev, seg_out, ws, grad_ray, fp64=False):
    g = torch.from_numpy(np.ascontiguousarray(grad_ray, dtype=np.float32)).cuda()
    gseg = xl.xl_merge_bwd(seg_out, d.ray_offsets, d.seg_ids, g, fp64=fp64)
    gs, gc = xl.xl_render_segments_bwd(d.sigma, d.rgb, d.t0, d.t1, d.seg_offsets, ws, gseg)
    torch.cuda.synchronize()
    return gseg, gs, gc


def oracle_rays(b, rays, sigma=None, rgb=None):
    s = b.sigma if sigma is None else sigma
    c = b.rgb if rgb is None else rgb
    return O.render_rays_single(s, c, b.t_start, b.t_end, b.seg_offsets, b.ray_offsets, b.seg_ids, rays)


def ray_segs(b, rays):
    return np.concatenate([b.seg_ids[b.ray_offsets[r]:b.ray_offsets[r + 1]] for r in rays])


# ------------------------------------------------------------------ forward
def test_k1_forward_all_rays():
    b = gen(0)
    say("k1 4096 rays: n", b.n)
    d = to_dev(b)
    seg_out, ws, ray_out = run_fwd(d)
    ref_seg = O.render_segments(b.sigma, b.rgb, b.t_start, b.t_end, b.seg_offsets)
    assert_tuples(seg_out.cpu().numpy(), ref_seg, "seg", "k1 segments")
    ref = oracle_rays(b, np.arange(b.n_rays))
    rep = assert_tuples(ray_out.cpu().numpy(), ref, "ray", "k1 rays")
    say("k1 max rel:", rep["rel"])


def test_k8_merge_equals_single_pass_and_oracle():
    b = gen(1)
    p = gen(1, plain=True)
    say("k8 65536 rays: n", b.n, "segments", b.n_seg)
    d = to_dev(b)
    seg_out, ws, ray_out = run_fwd(d)
    dp = to_dev(p)
    _, _, ray_plain = run_fwd(dp)
    # K=8 partitioned render equals the K=1 single pass on the device (all rays)
    assert_tuples(ray_out.cpu().numpy(), ray_plain.cpu().numpy().astype(np.float64), "ray",
                  "k8 vs k1 on device")
    rays = sample_rays(b.n_rays, 3000, 11)
    ref = oracle_rays(b, rays)
    assert_tuples(ray_out.cpu().numpy()[:, rays], ref, "ray", "k8 rays vs oracle")
    segs = ray_segs(b, rays)
    ref_seg = O.render_segments(b.sigma, b.rgb, b.t_start, b.t_end, b.seg_offsets, segs)
    assert_tuples(seg_out.cpu().numpy()[:, segs], ref_seg, "seg", "k8 segments vs oracle")


def test_merge_fp64_flag_k8():
    b = gen(1, n_rays=20000)
    d = to_dev(b)
    seg_out, ws, ray64 = run_fwd(d, fp64=True)
    rays = sample_rays(b.n_rays, 2000, 12)
    assert_tuples(ray64.cpu().numpy()[:, rays], oracle_rays(b, rays), "ray", "k8 fp64 merge")


# ------------------------------------------------------------------ backward
def _check_backward(b, d, rays, gseg, gs, gc, grad_ray, what, dq=None):
    s_in = b.sigma if dq is None else dq[0]
    c_in = b.rgb if dq is None else dq[1]
    g_seg_ref, segs, idx, ds_ref, dc_ref = O.backward_partitioned(
        s_in, c_in, b.t_start, b.t_end, b.seg_offsets, b.ray_offsets, b.seg_ids,
        grad_ray[:, rays], rays)
    assert_grads(gseg.cpu().numpy()[:, segs], g_seg_ref, what + " grad_seg")
    assert_grads(gs.float().cpu().numpy()[idx], ds_ref, what + " dsigma")
    assert_grads(gc.float().cpu().numpy()[idx], dc_ref, what + " drgb")


def test_k8_backward():
    b = gen(1, n_rays=8192)
    d = to_dev(b)
    seg_out, ws, ray_out = run_fwd(d)
    grad_ray = np.random.default_rng(13).normal(size=(7, b.n_rays))
    gseg, gs, gc = run_bwd(d, seg_out, ws, grad_ray)
    rays = sample_rays(b.n_rays, 1500, 14)
    _check_backward(b, d, rays, gseg, gs, gc, grad_ray, "k8")


def test_k16_forward_backward_medium():
    b = gen(2, n_rays=16384)
    say("k16 16384 rays: n", b.n)
    d = to_dev(b)
    seg_out, ws, ray_out = run_fwd(d)
    rays = sample_rays(b.n_rays, 600, 15)
    assert_tuples(ray_out.cpu().numpy()[:, rays], oracle_rays(b, rays), "ray", "k16 rays")
    grad_ray = np.random.default_rng(16).normal(size=(7, b.n_rays))
    gseg, gs, gc = run_bwd(d, seg_out, ws, grad_ray)
    _check_backward(b, d, rays[:300], gseg, gs, gc, grad_ray, "k16")


# ------------------------------------------------------------------ 16-bit storage
@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float16, BF16_F16], ids=storage_name)
def test_16bit_storage(dtype):
    b = gen(2, n_rays=16384)
    d = to_dev(b, dtype)
    seg_out, ws, ray_out = run_fwd(d)
    rays = sample_rays(b.n_rays, 600, 17)
    got = ray_out.cpu().numpy()[:, rays]
    # arithmetic on the stored values: oracle on the de-quantised inputs, FP32 bar
    dq = quantize(b, dtype)
    assert_tuples(got, oracle_rays(b, rays, *dq), "ray", f"{dtype} vs oracle(dequantised)")
    # quantisation included: oracle on the original FP32 inputs, colour within 2e-3
    ref = oracle_rays(b, rays)
    cerr = np.abs(got[1:4] - ref[1:4]).max()
    say(f"{dtype}: colour abs error vs original inputs {cerr:.3g}")
    assert cerr <= 2e-3
    grad_ray = np.random.default_rng(18).normal(size=(7, b.n_rays))
    gseg, gs, gc = run_bwd(d, seg_out, ws, grad_ray)
    g_seg_ref, segs, idx, ds_ref, dc_ref = O.backward_partitioned(
        dq[0], dq[1], b.t_start, b.t_end, b.seg_offsets, b.ray_offsets, b.seg_ids,
        grad_ray[:, rays[:200]], rays[:200])
    assert_grads(gseg.cpu().numpy()[:, segs], g_seg_ref, "16-bit grad_seg")
    # gradients are stored in the 16-bit types: judge them against their rounding
    us, uc = grad_ulps(dtype)
    assert_grads(gs.float().cpu().numpy()[idx], ds_ref, "16-bit dsigma", rtol=us, floor=1e-5,
                 norm_tol=us)
    assert_grads(gc.float().cpu().numpy()[idx], dc_ref, "16-bit drgb", rtol=uc, floor=1e-5,
                 norm_tol=uc)


# ------------------------------------------------------------------ edge cases
def _hand_batch(rays, shuffle_seed=None):
    """rays: list of rays, each a list of segments, each (sigma, rgb, t0, t1) arrays."""
    segs, seg_ray = [], []
    for r, ray in enumerate(rays):
        for sgm in ray:
            segs.append(sgm)
            seg_ray.append(r)
    order = np.arange(len(segs))
    if shuffle_seed is not None:
        np.random.default_rng(shuffle_seed).shuffle(order)
    lens = np.array([len(segs[i][0]) for i in order], np.int64)
    seg_offsets = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    cat = lambda k, shape: (np.concatenate([np.asarray(segs[i][k], np.float32).reshape(shape)
                                            for i in order]) if len(order) else np.zeros((0,) + shape[1:], np.float32))
    sigma = cat(0, (-1,)); rgb = cat(1, (-1, 3)); t0 = cat(2, (-1,)); t1 = cat(3, (-1,))
    pos = np.empty(len(segs), np.int64); pos[order] = np.arange(len(segs))
    counts = np.bincount(np.array(seg_ray, np.int64), minlength=len(rays)) if segs else np.zeros(len(rays), np.int64)
    ray_offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    seg_ids = pos  # segments were listed ray by ray, front to back
    return synth.Batch(sigma, rgb, t0, t1, seg_offsets, ray_offsets, seg_ids,
                       np.zeros(len(segs), np.int32), np.array(seg_ray, np.int64), np.arange(len(rays)))


def _seg(rng, n, t_start, sigma=None, width=None):
    w = np.full(n, 0.02) if width is None else np.asarray(width, float)
    t0 = t_start + np.concatenate([[0.0], np.cumsum(w)[:-1]])
    s = np.exp(rng.normal(0, 1.5, n)) if sigma is None else np.broadcast_to(sigma, (n,)).astype(float)
    return (s, rng.uniform(size=(n, 3)), t0, t0 + w)


def _edge_rays():
    rng = np.random.default_rng(21)
    empty = (np.zeros(0), np.zeros((0, 3)), np.zeros(0), np.zeros(0))
    rays = [
        [_seg(rng, 5, 0.1), empty, _seg(rng, 3, 0.3)],            # empty segment inside a ray
        [empty],                                                   # only an empty segment
        [],                                                        # no segments at all
        [_seg(rng, 40, 0.0, sigma=0.0)],                           # empty space
        [_seg(rng, 1, 0.5, sigma=1e4), _seg(rng, 10, 0.7)],        # one opaque sample
        [_seg(rng, 1, 0.1), _seg(rng, 1, 0.2), _seg(rng, 1, 0.3)],  # 1-sample segments
        [_seg(rng, 60, 0.0, sigma=100.0), _seg(rng, 5, 1.3)],      # tau > 104 (T underflows FP32)
        [_seg(rng, 12, 0.2, width=[0.02, 0, 0.03, 0, 0, 0.01, 0.02, 0, 0.02, 0.02, 0, 0.01])],
        [_seg(rng, 1024, 0.0, sigma=0.5, width=np.full(1024, 0.0029))],
        [_seg(rng, 2000, 0.0, width=np.full(2000, 0.001)), _seg(rng, 3000, 2.0, sigma=0.2,
                                                                width=np.full(3000, 0.0003))],
    ]
    for k in range(30):
        n = int(rng.integers(1, 90))
        cut = int(rng.integers(0, n))
        ray = [_seg(rng, cut, 0.2), _seg(rng, n - cut, 0.2 + 0.02 * cut)] if cut else [_seg(rng, n, 0.2)]
        rays.append(ray)
    return rays


@pytest.mark.parametrize("shuffle", [None, 5])
def test_edge_cases_forward_backward(shuffle):
    b = _hand_batch(_edge_rays(), shuffle)
    say("edge batch: n", b.n, "segments", b.n_seg, "rays", b.n_rays)
    d = to_dev(b)
    seg_out, ws, ray_out = run_fwd(d)
    ref_seg = O.render_segments(b.sigma, b.rgb, b.t_start, b.t_end, b.seg_offsets)
    assert_tuples(seg_out.cpu().numpy(), ref_seg, "seg", "edge segments")
    rays = np.arange(b.n_rays)
    assert_tuples(ray_out.cpu().numpy(), oracle_rays(b, rays), "ray", "edge rays")
    grad_ray = np.random.default_rng(22).normal(size=(7, b.n_rays))
    gseg, gs, gc = run_bwd(d, seg_out, ws, grad_ray)
    _check_backward(b, d, rays, gseg, gs, gc, grad_ray, "edge")


@pytest.mark.parametrize("n_samples", [1, 7, 509, 511, 512, 513, 1021, 1023, 1024, 1025, 1100, 2100])
def test_tiny_and_ragged_sizes(n_samples):
    """n_samples on the first ray plus 3 on the second: 509 and 1021 give whole
    tiles only (512, 1024 samples), the others a ragged last tile."""
    rng = np.random.default_rng(n_samples)
    # one long ray cut into segments of random length
    cuts = np.sort(rng.choice(np.arange(1, n_samples), size=min(5, n_samples - 1), replace=False)) \
        if n_samples > 1 else np.zeros(0, int)
    edges = np.concatenate([[0], cuts, [n_samples]]).astype(int)
    w = 2.9 / n_samples
    ray = [_seg(rng, int(bb - a), a * w, width=np.full(int(bb - a), w)) for a, bb in zip(edges[:-1], edges[1:])]
    b = _hand_batch([ray, [_seg(rng, 3, 0.5)]], shuffle_seed=1)
    d = to_dev(b)
    seg_out, ws, ray_out = run_fwd(d)
    assert_tuples(seg_out.cpu().numpy(), O.render_segments(b.sigma, b.rgb, b.t_start, b.t_end,
                                                           b.seg_offsets), "seg", f"n={n_samples}")
    assert_tuples(ray_out.cpu().numpy(), oracle_rays(b, np.arange(2)), "ray", f"n={n_samples}")
    grad_ray = np.random.default_rng(23).normal(size=(7, 2))
    gseg, gs, gc = run_bwd(d, seg_out, ws, grad_ray)
    _check_backward(b, d, np.arange(2), gseg, gs, gc, grad_ray, f"n={n_samples}")


def test_segments_spanning_many_tiles():
    """Segments of 9,000 and 7,000 samples (18 and 14 tiles of 512), placed
    so that neither starts on a tile boundary, with short segments around:
    the fixup's carries along long chains of tiles."""
    rng = np.random.default_rng(77)
    w = 2.9 / 16000
    a = _seg(rng, 9000, 0.0, sigma=np.exp(rng.normal(0, 1.0, 9000)) * 4.0, width=np.full(9000, w))
    b_ = _seg(rng, 7000, 9000 * w, sigma=np.exp(rng.normal(0, 1.0, 7000)) * 4.0, width=np.full(7000, w))
    batch = _hand_batch([[_seg(rng, 37, 0.2)], [a, b_], [_seg(rng, 300, 0.1), _seg(rng, 5, 2.0)]],
                        shuffle_seed=4)
    d = to_dev(batch)
    seg_out, ws, ray_out = run_fwd(d)
    assert_tuples(seg_out.cpu().numpy(), O.render_segments(batch.sigma, batch.rgb, batch.t_start,
                                                           batch.t_end, batch.seg_offsets), "seg",
                  "long segments")
    assert_tuples(ray_out.cpu().numpy(), oracle_rays(batch, np.arange(3)), "ray", "long segments")
    grad_ray = np.random.default_rng(78).normal(size=(7, 3))
    gseg, gs, gc = run_bwd(d, seg_out, ws, grad_ray)
    _check_backward(batch, d, np.arange(3), gseg, gs, gc, grad_ray, "long segments")


def test_no_samples():
    b = _hand_batch([[], [(np.zeros(0), np.zeros((0, 3)), np.zeros(0), np.zeros(0))]])
    d = to_dev(b)
    seg_out, ws, ray_out = run_fwd(d)
    assert np.all(seg_out.cpu().numpy() == 0)
    np.testing.assert_array_equal(ray_out.cpu().numpy(), [[1, 1]] + [[0, 0]] * 6)


# ------------------------------------------------------------------ autograd
def test_autograd_function_matches_oracle():
    b = gen(1, n_rays=2048)
    d = to_dev(b)
    sig = d.sigma.clone().requires_grad_(True)
    rgb = d.rgb.clone().requires_grad_(True)
    out = render(sig, rgb, d.t0, d.t1, d.seg_offsets, d.ray_offsets, d.seg_ids)
    grad_ray = np.random.default_rng(24).normal(size=(7, b.n_rays))
    (out * torch.from_numpy(grad_ray).float().cuda()).sum().backward()
    rays = np.arange(0, b.n_rays, 7)
    _, segs, idx, ds_ref, dc_ref = O.backward_partitioned(
        b.sigma, b.rgb, b.t_start, b.t_end, b.seg_offsets, b.ray_offsets, b.seg_ids,
        grad_ray[:, rays], rays)
    assert_grads(sig.grad.cpu().numpy()[idx], ds_ref, "autograd dsigma")
    assert_grads(rgb.grad.cpu().numpy()[idx], dc_ref, "autograd drgb")


def test_autograd_finite_differences_through_library():
    b = gen(0, n_rays=64)
    d = to_dev(b)
    sig = d.sigma.double()
    grad_ray = torch.from_numpy(np.random.default_rng(25).normal(size=(7, b.n_rays))).float().cuda()

    def f(s64):
        return float((render(s64.float().contiguous(), d.rgb, d.t0, d.t1, d.seg_offsets,
                             d.ray_offsets, d.seg_ids).double() * grad_ray.double()).sum())
    s = sig.clone().float().requires_grad_(True)
    out = render(s, d.rgb, d.t0, d.t1, d.seg_offsets, d.ray_offsets, d.seg_ids)
    (out * grad_ray).sum().backward()
    idx = np.random.default_rng(26).choice(b.n, 20, replace=False)
    for i in idx:
        h = 1e-2 * max(1.0, float(sig[i]))
        sp = sig.clone(); sp[i] += h
        sm = sig.clone(); sm[i] -= h
        fd = (f(sp) - f(sm)) / (2 * h)
        g = float(s.grad[i])
        assert abs(fd - g) <= 2e-3 * max(1.0, abs(g)) + 1e-3, (i, fd, g)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_crowded_tiles(dtype):
    """Tiles whose windows hold far more than 64 segments (1-4 sample segments
    and empty ones), so segment tuples and gradients take the paths that do
    not stage them in LDS."""
    rng = np.random.default_rng(41)
    empty = (np.zeros(0), np.zeros((0, 3)), np.zeros(0), np.zeros(0))
    rays = []
    for r in range(400):
        ray, t = [], 0.1
        for k in range(int(rng.integers(1, 5))):
            if rng.random() < 0.2:
                ray.append(empty)
            n = int(rng.integers(1, 5))
            ray.append(_seg(rng, n, t))
            t += 0.02 * n + 0.05
        rays.append(ray)
    b = _hand_batch(rays, shuffle_seed=7)
    per_tile = np.bincount(np.minimum(b.seg_offsets[:-1] // 512, max(b.n - 1, 0) // 512))
    say("crowded batch: n", b.n, "segments", b.n_seg, "max segments starting in a tile", per_tile.max())
    assert per_tile.max() > 64
    d = to_dev(b, dtype)
    dq = None if dtype == torch.float32 else quantize(b, dtype)
    seg_out, ws, ray_out = run_fwd(d)
    s_in, c_in = (b.sigma, b.rgb) if dq is None else dq
    assert_tuples(seg_out.cpu().numpy(), O.render_segments(s_in, c_in, b.t_start, b.t_end, b.seg_offsets),
                  "seg", f"crowded {dtype} segments")
    rays_all = np.arange(b.n_rays)
    assert_tuples(ray_out.cpu().numpy(), oracle_rays(b, rays_all, s_in, c_in), "ray", f"crowded {dtype} rays")
    grad_ray = np.random.default_rng(42).normal(size=(7, b.n_rays))
    gseg, gs, gc = run_bwd(d, seg_out, ws, grad_ray)
    if dq is None:
        _check_backward(b, d, rays_all, gseg, gs, gc, grad_ray, f"crowded {dtype}")
    else:
        g_seg_ref, segs, idx, ds_ref, dc_ref = O.backward_partitioned(
            s_in, c_in, b.t_start, b.t_end, b.seg_offsets, b.ray_offsets, b.seg_ids, grad_ray, rays_all)
        assert_grads(gseg.cpu().numpy()[:, segs], g_seg_ref, "crowded grad_seg")
        ulp = 2.0 ** -8
        assert_grads(gs.float().cpu().numpy()[idx], ds_ref, "crowded dsigma", rtol=ulp, floor=1e-5,
                     norm_tol=ulp)
        assert_grads(gc.float().cpu().numpy()[idx], dc_ref, "crowded drgb", rtol=ulp, floor=1e-5,
                     norm_tol=ulp)


# ------------------------------------------------------------------ long rays in the merge
@pytest.mark.parametrize("fp64", [False, True])
def test_merge_long_rays_empty_segments_and_invalid_ids(fp64):
    """Rays of 1-40 segments in the same waves: the merge keeps up to eight of
    a ray's tuples in registers and walks longer rays segment by segment.
    Some segments are empty, and some listed ids lie outside [0, n_seg): the
    merge skips those (their segments are listed by no ray)."""
    rng = np.random.default_rng(51)
    empty = (np.zeros(0), np.zeros((0, 3)), np.zeros(0), np.zeros(0))
    rays = []
    for r in range(400):
        nseg = int(rng.integers(9, 41)) if r % 3 else int(rng.integers(1, 9))
        ray, t = [], 0.05
        for k in range(nseg):
            if rng.random() < 0.15:
                ray.append(empty)
                continue
            n = int(rng.integers(1, 6))
            ray.append(_seg(rng, n, t))
            t += 0.02 * n + 0.01
        rays.append(ray)
    b = _hand_batch(rays, shuffle_seed=3)
    ids = b.seg_ids.copy()
    bad = rng.random(ids.size) < 0.03
    nb = int(bad.sum())
    ids[bad] = np.where(rng.random(nb) < 0.5, -1 - rng.integers(0, 5, nb), b.n_seg + rng.integers(0, 5, nb))
    # the oracle's batch: the same samples with the invalid entries dropped
    counts = np.add.reduceat((~bad).astype(np.int64), b.ray_offsets[:-1]) if b.n_rays else np.zeros(0)
    counts = np.where(np.diff(b.ray_offsets) > 0, counts, 0)
    ro = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    ob = synth.Batch(b.sigma, b.rgb, b.t_start, b.t_end, b.seg_offsets, ro, b.seg_ids[~bad],
                     b.seg_box, b.seg_ray, b.rays)
    say("long rays: segments per ray up to", np.diff(b.ray_offsets).max(), "invalid ids", nb)
    d = to_dev(b)
    d.seg_ids = torch.from_numpy(ids).cuda()
    seg_out, ws, ray_out = run_fwd(d, fp64=fp64)
    rays_all = np.arange(b.n_rays)
    assert_tuples(ray_out.cpu().numpy(), oracle_rays(ob, rays_all), "ray",
                  f"long rays fp64={fp64} ray tuples")
    grad_ray = np.random.default_rng(52).normal(size=(7, b.n_rays))
    gseg, gs, gc = run_bwd(d, seg_out, ws, grad_ray, fp64=fp64)
    g_seg_ref, segs, idx, ds_ref, dc_ref = O.backward_partitioned(
        b.sigma, b.rgb, b.t_start, b.t_end, b.seg_offsets, ro, ob.seg_ids, grad_ray, rays_all)
    g = gseg.cpu().numpy()
    assert_grads(g[:, segs], g_seg_ref, f"long rays fp64={fp64} grad_seg")
    unlisted = np.setdiff1d(np.arange(b.n_seg), segs)
    assert unlisted.size > 0 and np.all(g[:, unlisted] == 0)
    assert_grads(gs.cpu().numpy()[idx], ds_ref, f"long rays fp64={fp64} dsigma")
    assert_grads(gc.cpu().numpy()[idx], dc_ref, f"long rays fp64={fp64} drgb")
