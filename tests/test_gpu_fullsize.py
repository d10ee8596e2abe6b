"""Parity with the FP64 oracle at the workloads' full sizes, in the launch
configuration the benchmark times.

Inputs are generated on the device; the device generator is bit-identical to
the host one (layout, interval ends and densities: tests/test_gpu_gen.py).
The oracle regenerates the compared rays on the host and never sees device
data; it runs in worker processes over the host cores.  Device results are
located through the device's integer layout (segment offsets and per-ray
segment lists), which the comparison first checks against the host's.

Coverage: every ray of the K=8 workload; 16,384 seeded rays of the K=16
training batch in FP32 and BF16 storage; 16,384 seeded rays plus every sampled
ray with more than eight segments of the K=64 large partition (BF16 storage,
float64 merge), all of it launched at once as the benchmark does; chunked K=64
launches on 4,096 rays each; 16,384 rays of a 1280x720 FP16 view served by the
render server.
"""
import numpy as np
import pytest
import torch

from oracle import pool as OP
from paper_2404_16221_amd import _lib as xl
from paper_2404_16221_amd import synth
from paper_2404_16221_amd.serve import Server, request
from tests.parity import (BF16_F16, assert_grads, assert_tuples, grad_ulps, quantize, sample_rays,
                          storage_name)

pytestmark = [pytest.mark.gpu, pytest.mark.oracle_pool]


def say(*a):
    print(*a, flush=True)


def run(g, grad_ray, fp64=False):
    seg_out, ws = xl.xl_render_segments_fwd(g["sigma"], g["rgb"], g["t_start"], g["t_end"],
                                            g["seg_offsets"])
    # the region-aware merge, as the bench times it
    roff = g.get("region_offsets")
    ray_out = xl.xl_merge_fwd(seg_out, g["ray_offsets"], g["seg_ids"], fp64=fp64, region_offsets=roff)
    gseg = xl.xl_merge_bwd(seg_out, g["ray_offsets"], g["seg_ids"], grad_ray, fp64=fp64,
                           region_offsets=roff)
    gs, gc = xl.xl_render_segments_bwd(g["sigma"], g["rgb"], g["t_start"], g["t_end"],
                                       g["seg_offsets"], ws, gseg)
    torch.cuda.synchronize()
    return dict(seg_out=seg_out, ray_out=ray_out, grad_seg=gseg, gs=gs, gc=gc)


def device_layout(g):
    return (g["seg_offsets"].cpu().numpy(), g["ray_offsets"].cpu().numpy(),
            g["seg_ids"].cpu().numpy())


def gather(res, layout, rays):
    """The listed rays' device results, ray-major (segments front to back)."""
    segs, seg_len, spr, samples = OP.ray_major_index(*layout, rays)
    dev = res["ray_out"].device
    at_s = torch.from_numpy(segs).to(dev)
    out = {"ray": res["ray_out"][:, torch.from_numpy(np.asarray(rays)).to(dev)].cpu().numpy(),
           "seg": res["seg_out"][:, at_s].cpu().numpy(), "seg_len": seg_len, "spr": spr}
    if "grad_seg" in res:
        at = torch.from_numpy(samples).to(dev)
        out.update(grad_seg=res["grad_seg"][:, at_s].cpu().numpy(),
                   dsigma=res["gs"][at].float().cpu().numpy(),
                   drgb=res["gc"][at].float().cpu().numpy())
    return out


def compare(pool, w, got, rays, dtype, grad, what, host=None):
    """Oracle on the host regeneration of `rays` (ray ids of w) against the
    gathered device results `got`; grad: [7, len(rays)] or None."""
    h = synth.generate(w, rays=rays) if host is None else host
    local = np.arange(len(rays)) if host is None else np.asarray(rays)
    _, seg_len, spr, _ = OP.ray_major_index(h.seg_offsets, h.ray_offsets, h.seg_ids, local)
    # the device located the same segments (integer layout, bit-exact)
    np.testing.assert_array_equal(spr, got["spr"])
    np.testing.assert_array_equal(seg_len, got["seg_len"])
    s_in, c_in = (h.sigma, h.rgb) if dtype == torch.float32 else quantize(h, dtype)
    ref = OP.run(pool, s_in, c_in, h.t_start, h.t_end, h.seg_offsets, h.ray_offsets, h.seg_ids,
                 local, grad)
    label = f"{what} ({len(rays)} rays)"
    assert_tuples(got["ray"], ref["ray"], "ray", label + " ray tuples")
    assert_tuples(got["seg"], ref["seg"], "seg", label + " segment tuples")
    if dtype != torch.float32:
        # quantisation included: the oracle on the original FP32 inputs
        orig = OP.run(pool, h.sigma, h.rgb, h.t_start, h.t_end, h.seg_offsets, h.ray_offsets,
                      h.seg_ids, local)
        cerr = np.abs(got["ray"][1:4] - orig["ray"][1:4]).max()
        from tests.parity import record
        record(label + " colour vs original FP32 inputs", {"rgb": {"max_abs": float(cerr)}},
               n=len(rays))
        say(f"{label}: colour abs error vs the original FP32 inputs {cerr:.3g}")
        assert cerr <= 2e-3
    if grad is None:
        return
    assert_grads(got["grad_seg"], ref["grad_seg"], label + " grad_seg")
    if dtype == torch.float32:
        assert_grads(got["dsigma"], ref["dsigma"], label + " dsigma", 1e-5, 1e-6, 1e-5)
        assert_grads(got["drgb"], ref["drgb"], label + " drgb", 1e-5, 1e-6, 1e-5)
    else:
        # stored in the 16-bit types: judged against their rounding
        us, uc = grad_ulps(dtype)
        assert_grads(got["dsigma"], ref["dsigma"], label + " dsigma", us, 1e-5, us)
        assert_grads(got["drgb"], ref["drgb"], label + " drgb", uc, 1e-5, uc)


def test_k8_all_rays(oracle_pool):
    """All 65,536 rays of the K=8 workload, forward and backward, FP32."""
    w = synth.WORKLOADS[1]
    g = xl.xl_gen(w, torch.float32)
    say(f"k8 all rays: {g['sigma'].shape[0]} samples, {g['seg_ids'].shape[0]} segments")
    grad = np.random.default_rng(30).normal(size=(7, w.n_rays)).astype(np.float32)
    res = run(g, torch.from_numpy(grad).cuda())
    rays = np.arange(w.n_rays)
    got = gather(res, device_layout(g), rays)
    compare(oracle_pool, w, got, rays, torch.float32, grad.astype(np.float64), "k8 FP32")


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16, BF16_F16], ids=storage_name)
def test_k16_training_batch_full_size(oracle_pool, dtype):
    """All 262,144 rays launched at once; 16,384 seeded rays against the oracle."""
    w = synth.WORKLOADS[2]
    g = xl.xl_gen(w, dtype)
    say(f"k16 full size {dtype}: {g['sigma'].shape[0]} samples, {g['seg_ids'].shape[0]} segments")
    grad = np.random.default_rng(31).normal(size=(7, w.n_rays)).astype(np.float32)
    res = run(g, torch.from_numpy(grad).cuda())
    rays = sample_rays(w.n_rays, 16384, 32)
    got = gather(res, device_layout(g), rays)
    del res, g
    compare(oracle_pool, w, got, rays, dtype, grad[:, rays].astype(np.float64),
            f"k16 {storage_name(dtype)}")


def test_k16_partitioned_equals_plain_full_size():
    """All 262,144 rays: the K=16 partitioned render equals the K=1 single pass."""
    w = synth.WORKLOADS[2]
    g = xl.xl_gen(w, torch.float32)
    p = xl.xl_gen(w.plain(), torch.float32)
    assert torch.equal(p["seg_offsets"][-1:], g["seg_offsets"][-1:])
    z = torch.zeros((7, w.n_rays), device="cuda")
    ray_k = run(g, z)["ray_out"]
    ray_1 = run(p, z)["ray_out"]
    rep = assert_tuples(ray_k.cpu().numpy(), ray_1.cpu().numpy().astype(np.float64), "ray",
                        "k16 vs k1 on device, all rays")
    say("k16 vs plain max rel:", rep["rel"])


@pytest.mark.parametrize("chunk", [0, 11])
def test_k64_chunk_bf16_fp64_merge(oracle_pool, chunk):
    """The large partition streamed in chunks of 262,144 rays."""
    w = synth.WORKLOADS[4]
    ray0 = chunk * synth.CHUNK_RAYS_K64
    g = xl.xl_gen(w, torch.bfloat16, ray0, synth.CHUNK_RAYS_K64)
    say(f"k64 chunk {chunk}: {g['sigma'].shape[0]} samples, {g['seg_ids'].shape[0]} segments")
    grad = np.random.default_rng(40 + chunk).normal(size=(7, synth.CHUNK_RAYS_K64)).astype(np.float32)
    res = run(g, torch.from_numpy(grad).cuda(), fp64=True)
    rays = sample_rays(synth.CHUNK_RAYS_K64, 4096, 41 + chunk)
    got = gather(res, device_layout(g), rays)
    compare(oracle_pool, w, got, ray0 + rays, torch.bfloat16, grad[:, rays].astype(np.float64),
            f"k64 chunk {chunk} bf16 fp64-merge")


@pytest.mark.parametrize("dtype", [torch.bfloat16, BF16_F16], ids=storage_name)
def test_k64_all_rays_one_launch_fp64_merge(oracle_pool, dtype):
    """The large partition as the benchmark runs it: all 4,194,304 rays in one
    launch of each kernel (about 1.1G samples).  Compared: 16,384 seeded rays
    and up to 2,048 rays with more than eight segments."""
    w = synth.WORKLOADS[4]
    g = xl.xl_gen(w, dtype)
    say(f"k64 all rays: {g['sigma'].shape[0]} samples, {g['seg_ids'].shape[0]} segments")
    grad = np.random.default_rng(44).normal(size=(7, w.n_rays)).astype(np.float32)
    res = run(g, torch.from_numpy(grad).cuda(), fp64=True)
    layout = device_layout(g)
    spr = np.diff(layout[1])
    long_rays = np.flatnonzero(spr > 8)
    say(f"k64: {long_rays.size} rays with more than 8 segments (max {spr.max()})")
    long_rays = long_rays[np.sort(np.random.default_rng(46).choice(long_rays.size,
                                                                   min(2048, long_rays.size),
                                                                   replace=False))]
    rays = np.union1d(sample_rays(w.n_rays, 16384, 45), long_rays)
    got = gather(res, layout, rays)
    del res, g
    compare(oracle_pool, w, got, rays, dtype, grad[:, rays].astype(np.float64),
            f"k64 all rays {storage_name(dtype)} fp64-merge")


def test_k32_served_view_1280x720(oracle_pool):
    """A 1280x720 view (921,600 rays, K=32, FP16 storage) through the render
    server; 16,384 seeded rays against the oracle."""
    wd, ht, seed = 1280, 720, 77
    w3 = synth.WORKLOADS[3]
    scene = dict(grid=w3.grid, n_min=w3.n_min, n_max=w3.n_max, sigma_mu=w3.sigma_mu,
                 sigma_s=w3.sigma_s, zero_frac=w3.zero_frac)
    with Server(max_slots=2, dtype=torch.float16) as srv:
        t = srv.submit(request(wd, ht, seed=seed, **scene))
        r = srv.poll(t, timeout_us=60_000_000)
        assert r["rc"] == 0, r
        assert r["n_rays"] == wd * ht
        out = srv.result(t, r["n_rays"])
        torch.cuda.synchronize()
        srv.release(t)
    say(f"served {wd}x{ht}: {r['n_samples']} samples")
    w = synth.serve_workload(wd, ht, seed)
    rays = sample_rays(w.n_rays, 16384, 78)
    h = synth.generate(w, rays=rays)
    dq = quantize(h, torch.float16)
    local = np.arange(len(rays))
    ref = OP.run(oracle_pool, dq[0], dq[1], h.t_start, h.t_end, h.seg_offsets, h.ray_offsets,
                 h.seg_ids, local)
    got = out[:, torch.from_numpy(rays).cuda()].cpu().numpy()
    label = f"k32 served {wd}x{ht} fp16 ({len(rays)} rays)"
    assert_tuples(got, ref["ray"], "ray", label + " ray tuples")
    orig = OP.run(oracle_pool, h.sigma, h.rgb, h.t_start, h.t_end, h.seg_offsets, h.ray_offsets,
                  h.seg_ids, local)
    cerr = np.abs(got[1:4] - orig["ray"][1:4]).max()
    from tests.parity import record
    record(label + " colour vs original FP32 inputs", {"rgb": {"max_abs": float(cerr)}}, n=len(rays))
    say(f"{label}: colour abs error vs the original FP32 inputs {cerr:.3g}")
    assert cerr <= 2e-3
