"""Feature channels on the GPU against the FP64 oracle: per-segment and per-ray
features, the merge backward and the per-sample gradients."""
import numpy as np
import pytest
import torch

from oracle import features as Fo
from paper_2404_16221_amd import _lib as xl
from paper_2404_16221_amd import synth
from tests.parity import assert_grads, to_dev

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def batch(rays=300, w=1, F=8, seed=0, dtype=torch.float32):
    b = synth.generate(synth.WORKLOADS[w], rays=np.arange(rays))
    feat = np.random.default_rng(seed).normal(size=(b.n, F)).astype(np.float32)
    if dtype != torch.float32:  # the oracle sees the stored (rounded) values
        b.sigma = torch.from_numpy(b.sigma).to(dtype).float().numpy()
        feat = torch.from_numpy(feat).to(dtype).float().numpy()
    return b, feat


def check_close(got, ref, scale, rtol, what):
    err = np.abs(np.asarray(got, np.float64) - ref)
    lim = rtol * scale + 1e-7
    worst = float((err / lim).max()) if err.size else 0.0
    assert worst <= 1.0, f"{what}: worst normalised error {worst:.3g}"


def run(b, feat, dtype, g_ray):
    d = to_dev(b, dtype)
    f = torch.from_numpy(feat).cuda().to(dtype)
    phi, tau = xl.xl_render_features_fwd(d.sigma, f, d.t0, d.t1, d.seg_offsets)
    out = xl.xl_merge_features_fwd(tau, phi, d.ray_offsets, d.seg_ids)
    gphi, gtau = xl.xl_merge_features_bwd(tau, phi, d.ray_offsets, d.seg_ids,
                                          torch.from_numpy(g_ray).cuda())
    gs, gf = xl.xl_render_features_bwd(d.sigma, f, d.t0, d.t1, d.seg_offsets, phi, gphi, gtau)
    torch.cuda.synchronize()
    return [x.float().cpu().numpy() for x in (phi, tau, out, gphi, gtau, gs, gf)]


@pytest.mark.parametrize("F", [4, 8, 16, 32])
def test_features_fp32_against_oracle(F):
    say(f"features fp32 F={F}")
    b, feat = batch(F=F, seed=F)
    g = np.random.default_rng(100 + F).normal(size=(F, b.n_rays)).astype(np.float32)
    phi, tau, out, gphi, gtau, gs, gf = run(b, feat, torch.float32, g)
    tau_r, phi_r, out_r = Fo.render_features(b.sigma, feat, b.t_start, b.t_end, b.seg_offsets,
                                              b.ray_offsets, b.seg_ids)
    _, scale_seg, scale_ray = Fo.render_features(b.sigma, np.abs(feat), b.t_start, b.t_end,
                                                 b.seg_offsets, b.ray_offsets, b.seg_ids)
    check_close(phi.T, phi_r, scale_seg, 1e-5, "phi_seg")
    check_close(tau, tau_r, tau_r, 1e-5, "tau_seg")
    check_close(out.T, out_r, scale_ray, 1e-5, "phi_ray")
    gs_r, gf_r = Fo.grad_features(b.sigma, feat, b.t_start, b.t_end, b.seg_offsets, b.ray_offsets,
                                  b.seg_ids, g.T)
    assert_grads(gs, gs_r, f"F={F} dsigma", rtol=1e-5, floor=1e-6, norm_tol=1e-5)
    assert_grads(gf, gf_r, f"F={F} dfeat", rtol=1e-5, floor=1e-6, norm_tol=1e-5)


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float16])
def test_features_16bit_storage(dtype):
    say(f"features {dtype}")
    F = 16
    b, feat = batch(rays=200, F=F, seed=3, dtype=dtype)
    g = np.random.default_rng(5).normal(size=(F, b.n_rays)).astype(np.float32)
    phi, tau, out, gphi, gtau, gs, gf = run(b, feat, dtype, g)
    _, phi_r, out_r = Fo.render_features(b.sigma, feat, b.t_start, b.t_end, b.seg_offsets,
                                         b.ray_offsets, b.seg_ids)
    _, scale_seg, scale_ray = Fo.render_features(b.sigma, np.abs(feat), b.t_start, b.t_end,
                                                 b.seg_offsets, b.ray_offsets, b.seg_ids)
    check_close(out.T, out_r, scale_ray, 1e-5, "phi_ray on rounded inputs")
    gs_r, gf_r = Fo.grad_features(b.sigma, feat, b.t_start, b.t_end, b.seg_offsets, b.ray_offsets,
                                  b.seg_ids, g.T)
    ulp = 2.0 ** -8 if dtype == torch.bfloat16 else 2.0 ** -11
    assert_grads(gs, gs_r, "16-bit dsigma", rtol=ulp, floor=1e-5, norm_tol=ulp)
    assert_grads(gf, gf_r, "16-bit dfeat", rtol=ulp, floor=1e-5, norm_tol=ulp)


def test_colour_channels_equal_the_colour_path():
    """Features (r, g, b, 0) through the feature kernels give the colour of the
    composite kernels, segment by segment and per ray."""
    b, _ = batch(rays=256)
    feat = np.concatenate([b.rgb, np.zeros((b.n, 1), np.float32)], axis=1)
    d = to_dev(b)
    f = torch.from_numpy(feat).cuda()
    phi, tau = xl.xl_render_features_fwd(d.sigma, f, d.t0, d.t1, d.seg_offsets)
    seg_out, _ = xl.xl_render_segments_fwd(d.sigma, d.rgb, d.t0, d.t1, d.seg_offsets)
    ray = xl.xl_merge_fwd(seg_out, d.ray_offsets, d.seg_ids)
    out = xl.xl_merge_features_fwd(tau, phi, d.ray_offsets, d.seg_ids)
    torch.cuda.synchronize()
    np.testing.assert_allclose(phi[:3].cpu().numpy(), seg_out[1:4].cpu().numpy(), rtol=2e-5, atol=1e-6)
    np.testing.assert_allclose(out[:3].cpu().numpy(), ray[1:4].cpu().numpy(), rtol=2e-5, atol=1e-6)
    assert float(out[3].abs().max()) == 0.0


def test_accumulate_into_colour_gradient_and_edge_cases():
    # empty segments, rays without segments, and a single-sample segment
    sigma = np.array([0.5, 2.0, 0.0, 3.0], np.float32)
    t0 = np.array([0.0, 0.1, 0.3, 0.35], np.float32)
    t1 = np.array([0.1, 0.3, 0.35, 0.5], np.float32)
    seg_offsets = np.array([0, 2, 2, 4])
    ray_offsets = np.array([0, 0, 2, 3])
    seg_ids = np.array([0, 1, 2])
    feat = np.random.default_rng(1).normal(size=(4, 4)).astype(np.float32)
    g = np.random.default_rng(2).normal(size=(4, 3)).astype(np.float32)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    phi, tau = xl.xl_render_features_fwd(T(sigma), T(feat), T(t0), T(t1), T(seg_offsets))
    out = xl.xl_merge_features_fwd(tau, phi, T(ray_offsets), T(seg_ids))
    gphi, gtau = xl.xl_merge_features_bwd(tau, phi, T(ray_offsets), T(seg_ids), T(g))
    base = T(np.array([1.0, -2.0, 0.5, 4.0], np.float32))
    gs, gf = xl.xl_render_features_bwd(T(sigma), T(feat), T(t0), T(t1), T(seg_offsets), phi, gphi,
                                       gtau, grad_sigma=base.clone(), accumulate_sigma=True)
    torch.cuda.synchronize()
    _, phi_r, out_r = Fo.render_features(sigma, feat, t0, t1, seg_offsets, ray_offsets, seg_ids)
    np.testing.assert_allclose(out.cpu().numpy().T, out_r, rtol=1e-5, atol=1e-6)
    assert np.all(out.cpu().numpy()[:, 0] == 0.0) and np.all(phi.cpu().numpy()[:, 1] == 0.0)
    gs_r, gf_r = Fo.grad_features(sigma, feat, t0, t1, seg_offsets, ray_offsets, seg_ids, g.T)
    np.testing.assert_allclose(gs.cpu().numpy(), gs_r + base.cpu().numpy(), rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(gf.cpu().numpy(), gf_r, rtol=1e-5, atol=1e-6)


def test_k16_full_size_sampled():
    """All 262,144 k16 rays (135M samples) with 16 BF16 channels in one launch
    of each kernel, as the benchmark times it; sampled rays against the oracle
    (per-ray features and per-sample gradients of those rays)."""
    w = synth.WORKLOADS[2]
    F = 16
    gdev = xl.xl_gen(w, torch.bfloat16)
    n = gdev["sigma"].shape[0]
    say(f"features k16 full size: {n} samples")
    feat = features_of(torch.arange(n, device="cuda"), F).to(torch.bfloat16)
    g = torch.from_numpy(np.random.default_rng(9).normal(size=(F, w.n_rays)).astype(np.float32)).cuda()
    phi, tau = xl.xl_render_features_fwd(gdev["sigma"], feat, gdev["t_start"], gdev["t_end"],
                                         gdev["seg_offsets"])
    out = xl.xl_merge_features_fwd(tau, phi, gdev["ray_offsets"], gdev["seg_ids"])
    gphi, gtau = xl.xl_merge_features_bwd(tau, phi, gdev["ray_offsets"], gdev["seg_ids"], g)
    gs, gf = xl.xl_render_features_bwd(gdev["sigma"], feat, gdev["t_start"], gdev["t_end"],
                                       gdev["seg_offsets"], phi, gphi, gtau)
    torch.cuda.synchronize()
    from tests.parity import sample_rays
    rays = sample_rays(w.n_rays, 24, 12)
    ro = gdev["ray_offsets"].cpu().numpy()
    so = gdev["seg_offsets"]
    for r in rays:
        segs = gdev["seg_ids"][ro[r]:ro[r + 1]]
        idx = torch.cat([torch.arange(int(so[s]), int(so[s + 1]), device="cuda") for s in segs]) \
            if segs.numel() else torch.zeros(0, dtype=torch.int64, device="cuda")
        lens = [int(so[s + 1] - so[s]) for s in segs]
        sig = gdev["sigma"][idx].float().cpu().numpy()
        t0 = gdev["t_start"][idx].cpu().numpy()
        t1 = gdev["t_end"][idx].cpu().numpy()
        fr = feat[idx].float().cpu().numpy()
        seg_off = np.concatenate([[0], np.cumsum(lens)])
        ids = np.arange(len(lens))
        _, _, o_r = Fo.render_features(sig, fr, t0, t1, seg_off, np.array([0, len(lens)]), ids)
        _, _, sc = Fo.render_features(sig, np.abs(fr), t0, t1, seg_off, np.array([0, len(lens)]), ids)
        check_close(out[:, r].cpu().numpy(), o_r[0], sc[0], 1e-5, f"ray {r} phi")
        gs_r, gf_r = Fo.grad_features(sig, fr, t0, t1, seg_off, np.array([0, len(lens)]), ids,
                                      g[:, r].cpu().numpy()[None, :])
        assert_grads(gs[idx].float().cpu().numpy(), gs_r, f"ray {r} dsigma", rtol=2.0 ** -8,
                     floor=1e-5, norm_tol=2.0 ** -8)
        assert_grads(gf[idx].float().cpu().numpy(), gf_r, f"ray {r} dfeat", rtol=2.0 ** -8,
                     floor=1e-5, norm_tol=2.0 ** -8)


def features_of(i, F):
    """Deterministic features in [-1, 1) from the sample index (a hash), F per sample."""
    x = i[:, None] * F + torch.arange(F, device=i.device)[None, :]
    x = (x * 2654435761) % 4294967296
    x = (x ^ (x >> 13)) * 1274126177 % 4294967296
    return (x.float() / 2147483648.0) - 1.0


def test_autograd_colour_and_features_share_sigma():
    """render() and render_features() on the same sigma: autograd adds the two
    density gradients; checked against the two oracles' gradients summed."""
    from oracle import render as O
    from paper_2404_16221_amd.autograd import render, render_features
    b, feat = batch(rays=128, F=8, seed=21)
    d = to_dev(b)
    sig = d.sigma.clone().requires_grad_(True)
    rgb = d.rgb.clone().requires_grad_(True)
    f = torch.from_numpy(feat).cuda().requires_grad_(True)
    rng = np.random.default_rng(22)
    g_col = rng.normal(size=(7, b.n_rays))
    g_ft = rng.normal(size=(8, b.n_rays))
    ray = render(sig, rgb, d.t0, d.t1, d.seg_offsets, d.ray_offsets, d.seg_ids)
    out = render_features(sig, f, d.t0, d.t1, d.seg_offsets, d.ray_offsets, d.seg_ids)
    loss = (ray * torch.from_numpy(g_col).cuda().float()).sum() + \
        (out * torch.from_numpy(g_ft).cuda().float()).sum()
    loss.backward()
    torch.cuda.synchronize()
    _, _, idx, ds_col, _ = O.backward_partitioned(b.sigma, b.rgb, b.t_start, b.t_end, b.seg_offsets,
                                                  b.ray_offsets, b.seg_ids, g_col)
    ds_ft, df = Fo.grad_features(b.sigma, feat, b.t_start, b.t_end, b.seg_offsets, b.ray_offsets,
                                 b.seg_ids, g_ft.T)
    ds_ref = ds_ft.copy()
    ds_ref[idx] += ds_col
    assert_grads(sig.grad.cpu().numpy(), ds_ref, "dsigma, colour + features", rtol=1e-5, floor=1e-6,
                 norm_tol=1e-5)
    assert_grads(f.grad.cpu().numpy(), df, "dfeat", rtol=1e-5, floor=1e-6, norm_tol=1e-5)
