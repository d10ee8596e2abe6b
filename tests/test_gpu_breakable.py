"""GPU parity of the breakable-integral operator (App. B.2) against its FP64
oracle (oracle/breakable.py), through the C ABI."""
import numpy as np
import pytest
import torch

from oracle import breakable as B
from paper_2404_16221_amd import _lib as xl
from paper_2404_16221_amd import synth
from tests.parity import assert_grads, quantize, record, sample_rays

pytestmark = pytest.mark.gpu

RTOL = 1e-5


def say(*a):
    print(*a, flush=True)


def run(sigma, t0, t1, so, ro, ids, pairs, grad_ray, ch=None, n_ch=None):
    """Forward and backward through the four entry points."""
    d = xl.breakable(sigma, t0, t1, pairs, ch=ch, n_ch=n_ch)
    seg = xl.xl_render_breakable_fwd(d, so)
    ray = xl.xl_merge_breakable_fwd(d, seg, ro, ids)
    gseg = xl.xl_merge_breakable_bwd(d, seg, ro, ids, grad_ray)
    gs = torch.empty_like(sigma)
    gc = torch.empty_like(ch) if ch is not None else None
    xl.xl_render_breakable_bwd(d, so, seg, gseg, gs, gc)
    torch.cuda.synchronize()
    return seg, ray, gseg, gs, gc


def check_tuples(got, ref, what, scale=None):
    """Per-row: |x - x64| <= 1e-5 |x64| + 1e-7 * max(1, max|row|) (transmittance
    row 0 of a ray tuple through tau = -log T)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    worst = 0.0
    errs = {}
    for k in range(ref.shape[0]):
        r, g = ref[k], got[k]
        s = max(1.0, np.abs(r).max()) if scale is None else scale
        lim = RTOL * np.abs(r) + 1e-7 * s
        e = np.abs(g - r)
        worst = max(worst, float((e / lim).max()) if e.size else 0.0)
        errs[f"row{k}"] = {"max_abs": float(e.max()) if e.size else 0.0}
    record(what, errs, n=int(ref.shape[1]), worst_normalised=worst)
    assert worst <= 1.0, f"{what}: worst normalised {worst:.3g}"


def _batch(rng, n_rays, nmax, F):
    rays = []
    for r in range(n_rays):
        n = int(rng.integers(0, nmax))
        w = rng.exponential(0.02, size=n)
        t0 = 0.1 + np.concatenate([[0.0], np.cumsum(w)[:-1]]) if n else np.zeros(0)
        t1 = t0 + w
        sig = np.exp(rng.normal(0.0, 1.5, size=n))
        sig[rng.uniform(size=n) < 0.2] = 0.0
        ch = rng.normal(size=(n, F))
        cuts = np.sort(rng.choice(np.arange(0, n + 1), size=int(rng.integers(0, 5)), replace=True))
        edges = np.concatenate([[0], cuts, [n]]).astype(int)
        rays.append([(sig[a:b], ch[a:b], t0[a:b], t1[a:b]) for a, b in zip(edges[:-1], edges[1:])])
    segs = [(r, s) for r, ray in enumerate(rays) for s in ray]
    order = rng.permutation(len(segs))
    lens = np.array([len(segs[i][1][0]) for i in order], np.int64)
    so = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    cat = lambda k, shape: (np.concatenate([segs[i][1][k] for i in order]).reshape(shape)
                            if len(order) else np.zeros(shape))
    sigma, ch, t0, t1 = cat(0, (-1,)), cat(1, (-1, F)), cat(2, (-1,)), cat(3, (-1,))
    pos = np.empty(len(segs), np.int64)
    pos[order] = np.arange(len(segs))
    counts = np.bincount(np.array([r for r, _ in segs], np.int64), minlength=n_rays)
    ro = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return (sigma.astype(np.float32), ch.astype(np.float32), t0.astype(np.float32),
            t1.astype(np.float32), so, ro, pos)


@pytest.mark.parametrize("pairs", [[], [(0, 1)], [(0, 1), (2, 2), (1, 0), (2, 0)]])
def test_loaded_channels_fp32(pairs):
    rng = np.random.default_rng(61 + len(pairs))
    F = 3
    sigma, ch, t0, t1, so, ro, ids = _batch(rng, 300, 120, F)
    say("loaded F=3: samples", sigma.size, "segments", so.size - 1, "pairs", pairs)
    C = lambda a, dt=None: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    g = rng.normal(size=(1 + F + len(pairs), ro.size - 1))
    seg, ray, gseg, gs, gc = run(C(sigma), C(t0), C(t1), C(so), C(ro), C(ids), pairs,
                                 C(g.astype(np.float32)), ch=C(ch))
    seg_ref, ray_ref = B.render_rays(sigma, ch, t0, t1, so, ro, ids, pairs)
    check_tuples(seg.cpu().numpy(), seg_ref, f"breakable loaded P={len(pairs)} segment tuples")
    got = ray.cpu().numpy()
    with np.errstate(divide="ignore"):
        check_tuples(-np.log(got[:1]), -np.log(ray_ref[:1]), f"breakable loaded P={len(pairs)} tau of T")
    check_tuples(got[1:], ray_ref[1:], f"breakable loaded P={len(pairs)} ray tuples")
    gseg_ref, gs_ref, gc_ref = B.backward(sigma, ch, t0, t1, so, ro, ids, pairs, g)
    listed = np.sort(ids)
    assert_grads(gseg.cpu().numpy()[:, listed], gseg_ref[:, listed], f"breakable P={len(pairs)} grad_seg")
    assert_grads(gs.cpu().numpy(), gs_ref, f"breakable P={len(pairs)} dsigma")
    assert_grads(gc.cpu().numpy(), gc_ref, f"breakable P={len(pairs)} dch")


def test_midpoint_powers_on_generated_rays_and_colour_path():
    """Channels 1, m, m^2 formed in the kernel (depth moments) with the
    distortion's pairs (m, 1) and (1, m), on rays of the K=8 workload; the
    first two moments equal the colour path's opacity and depth."""
    w = synth.WORKLOADS[1]
    b = synth.generate(w, rays=np.arange(1500))
    pairs = [(1, 0), (0, 1)]
    C = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    g = np.random.default_rng(63).normal(size=(6, b.n_rays))
    sig = C(b.sigma)
    seg, ray, gseg, gs, _ = run(sig, C(b.t_start), C(b.t_end), C(b.seg_offsets), C(b.ray_offsets),
                                C(b.seg_ids), pairs, C(g.astype(np.float32)), n_ch=3)
    ch = B.midpoint_powers(b.t_start, b.t_end, 3)
    seg_ref, ray_ref = B.render_rays(b.sigma, ch, b.t_start, b.t_end, b.seg_offsets,
                                     b.ray_offsets, b.seg_ids, pairs)
    check_tuples(seg.cpu().numpy(), seg_ref, "breakable midpoint powers segment tuples")
    got = ray.cpu().numpy()
    check_tuples(got[1:], ray_ref[1:], "breakable midpoint powers ray tuples")
    gseg_ref, gs_ref, _ = B.backward(b.sigma, ch, b.t_start, b.t_end, b.seg_offsets, b.ray_offsets,
                                     b.seg_ids, pairs, g, channels_have_grad=False)
    assert_grads(gseg.cpu().numpy(), gseg_ref, "breakable midpoint powers grad_seg")
    assert_grads(gs.cpu().numpy(), gs_ref, "breakable midpoint powers dsigma")
    # opacity and depth against the colour path on the device
    s_out, _ = xl.xl_render_segments_fwd(sig, C(b.rgb), C(b.t_start), C(b.t_end), C(b.seg_offsets))
    colour = xl.xl_merge_fwd(s_out, C(b.ray_offsets), C(b.seg_ids)).cpu().numpy()
    np.testing.assert_allclose(got[1], colour[4], rtol=2e-5, atol=1e-7)
    np.testing.assert_allclose(got[2], colour[5], rtol=2e-5, atol=3e-7)


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float16])
def test_loaded_channels_16bit(dtype):
    rng = np.random.default_rng(64)
    F, pairs = 4, [(0, 3), (1, 1)]
    sigma, ch, t0, t1, so, ro, ids = _batch(rng, 200, 100, F)
    C = lambda a, dt=None: torch.from_numpy(np.ascontiguousarray(a)).cuda().to(dt) if dt else \
        torch.from_numpy(np.ascontiguousarray(a)).cuda()
    g = rng.normal(size=(1 + F + len(pairs), ro.size - 1))
    seg, ray, gseg, gs, gc = run(C(sigma, dtype), C(t0), C(t1), C(so), C(ro), C(ids), pairs,
                                 C(g.astype(np.float32)), ch=C(ch, dtype))
    sq = torch.from_numpy(sigma).to(dtype).double().numpy()
    cq = torch.from_numpy(ch).to(dtype).double().numpy()
    seg_ref, ray_ref = B.render_rays(sq, cq, t0, t1, so, ro, ids, pairs)
    check_tuples(seg.cpu().numpy(), seg_ref, f"breakable {dtype} segment tuples")
    check_tuples(ray.cpu().numpy()[1:], ray_ref[1:], f"breakable {dtype} ray tuples")
    gseg_ref, gs_ref, gc_ref = B.backward(sq, cq, t0, t1, so, ro, ids, pairs, g)
    listed = np.sort(ids)
    assert_grads(gseg.cpu().numpy()[:, listed], gseg_ref[:, listed], f"breakable {dtype} grad_seg")
    ulp = 2.0 ** -8 if dtype == torch.bfloat16 else 2.0 ** -11
    assert_grads(gs.float().cpu().numpy(), gs_ref, f"breakable {dtype} dsigma", ulp, 1e-5, ulp)
    assert_grads(gc.float().cpu().numpy(), gc_ref, f"breakable {dtype} dch", ulp, 1e-5, ulp)


def test_k16_full_size_midpoint_powers_sampled():
    """All 262,144 rays of the training batch in one launch of each kernel
    (BF16 density, channels 1, m, m^2, distortion pairs); 256 seeded rays
    against the oracle."""
    w = synth.WORKLOADS[2]
    gd = xl.xl_gen(w, torch.bfloat16)
    pairs = [(1, 0), (0, 1)]
    g = np.random.default_rng(65).normal(size=(6, w.n_rays)).astype(np.float32)
    seg, ray, gseg, gs, _ = run(gd["sigma"], gd["t_start"], gd["t_end"], gd["seg_offsets"],
                                gd["ray_offsets"], gd["seg_ids"], pairs,
                                torch.from_numpy(g).cuda(), n_ch=3)
    rays = sample_rays(w.n_rays, 256, 66)
    h = synth.generate(w, rays=rays)
    sq, _ = quantize(h, torch.bfloat16)
    ch = B.midpoint_powers(h.t_start, h.t_end, 3)
    seg_ref, ray_ref = B.render_rays(sq, ch, h.t_start, h.t_end, h.seg_offsets, h.ray_offsets,
                                     h.seg_ids, pairs)
    check_tuples(ray.cpu().numpy()[1:, rays], ray_ref[1:], "breakable k16 full size ray tuples")
    gseg_ref, gs_ref, _ = B.backward(sq, ch, h.t_start, h.t_end, h.seg_offsets, h.ray_offsets,
                                     h.seg_ids, pairs, g[:, rays].astype(np.float64),
                                     channels_have_grad=False)
    # the same samples on the device: ray-major positions from the integer layout
    from oracle.pool import ray_major_index
    lay = [gd[k].cpu().numpy() for k in ("seg_offsets", "ray_offsets", "seg_ids")]
    segs_d, _, _, samp_d = ray_major_index(*lay, rays)
    segs_h, _, _, samp_h = ray_major_index(h.seg_offsets, h.ray_offsets, h.seg_ids, np.arange(len(rays)))
    assert_grads(gseg.cpu().numpy()[:, segs_d], gseg_ref[:, segs_h], "breakable k16 full size grad_seg")
    ulp = 2.0 ** -8
    assert_grads(gs[torch.from_numpy(samp_d).cuda()].float().cpu().numpy(), gs_ref[samp_h],
                 "breakable k16 full size dsigma", ulp, 1e-5, ulp)
