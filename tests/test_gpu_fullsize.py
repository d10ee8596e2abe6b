"""Parity at full workload sizes, in the launch configuration the benchmark times.

Inputs are generated on the device (bit-identical layout and interval ends to
the host generator, densities within ~1e-6); the oracle regenerates only the
sampled rays on the host and never sees device data.
"""
import numpy as np
import pytest
import torch

from oracle import render as O
from paper_2404_16221_amd import _lib as xl
from paper_2404_16221_amd import synth
from tests.parity import assert_grads, assert_tuples, quantize, sample_rays

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def run(g, grad_ray, fp64=False):
    seg_out, ws = xl.xl_render_segments_fwd(g["sigma"], g["rgb"], g["t_start"], g["t_end"],
                                            g["seg_offsets"])
    ray_out = xl.xl_merge_fwd(seg_out, g["ray_offsets"], g["seg_ids"], fp64=fp64)
    gseg = xl.xl_merge_bwd(seg_out, g["ray_offsets"], g["seg_ids"], grad_ray, fp64=fp64)
    gs, gc = xl.xl_render_segments_bwd(g["sigma"], g["rgb"], g["t_start"], g["t_end"],
                                       g["seg_offsets"], ws, gseg)
    torch.cuda.synchronize()
    return ray_out, gs, gc


def ray_sample_positions(g, rays):
    """Device sample indices of each listed ray, front to back (integer layout only)."""
    ro = g["ray_offsets"].cpu().numpy()
    out = []
    for r in rays:
        ids = g["seg_ids"][ro[r]:ro[r + 1]]
        so = torch.stack([g["seg_offsets"][ids], g["seg_offsets"][ids + 1]]).cpu().numpy()
        out.append(np.concatenate([np.arange(a, b) for a, b in so.T]) if so.shape[1]
                   else np.zeros(0, np.int64))
    return out


def check_sampled(w, g, ray0, rays_local, ray_out, gs, gc, grad_ray_np, dtype, what):
    h = synth.generate(w, rays=ray0 + rays_local)  # host regeneration of the sampled rays
    if dtype == torch.float32:
        s_in, c_in = h.sigma, h.rgb
    else:
        s_in, c_in = quantize(h, dtype)
    ref = O.render_rays_single(s_in, c_in, h.t_start, h.t_end, h.seg_offsets, h.ray_offsets,
                               h.seg_ids)
    assert_tuples(ray_out.cpu().numpy()[:, rays_local], ref, "ray", what + " rays")
    _, _, idx, ds_ref, dc_ref = O.backward_partitioned(
        s_in, c_in, h.t_start, h.t_end, h.seg_offsets, h.ray_offsets, h.seg_ids,
        grad_ray_np[:, rays_local])
    # the same samples on the device, in the same (t) order as the host batch
    dev_pos = ray_sample_positions(g, rays_local)
    host_pos = [h.ray_sample_index(k) for k in range(len(rays_local))]
    order = np.empty(h.n, np.int64)
    order[np.concatenate(host_pos)] = np.concatenate(dev_pos)
    ref_at = np.empty(h.n, np.int64)
    ref_at[idx] = np.arange(idx.size)
    hp = np.concatenate(host_pos)
    # gather the sampled rays' gradients on the device (the full arrays can be
    # tens of GB)
    at = torch.from_numpy(order[hp]).to(gs.device)
    gs_dev = gs[at].float().cpu().numpy()
    gc_dev = gc[at].float().cpu().numpy()
    if dtype == torch.float32:
        rtol, floor, nt = 1e-5, 1e-6, 1e-5
    else:
        rtol = 2.0 ** -8 if dtype == torch.bfloat16 else 2.0 ** -11
        floor, nt = 1e-5, rtol
    assert_grads(gs_dev, ds_ref[ref_at[hp]], what + " dsigma", rtol, floor, nt)
    assert_grads(gc_dev, dc_ref[ref_at[hp]], what + " drgb", rtol, floor, nt)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_k16_training_batch_full_size(dtype):
    w = synth.WORKLOADS[2]
    g = xl.xl_gen(w, dtype)
    say(f"k16 full size {dtype}: {g['sigma'].shape[0]} samples, {g['seg_ids'].shape[0]} segments")
    grad_np = np.random.default_rng(31).normal(size=(7, w.n_rays)).astype(np.float32)
    ray_out, gs, gc = run(g, torch.from_numpy(grad_np).cuda())
    rays = sample_rays(w.n_rays, 48, 32)
    check_sampled(w, g, 0, rays, ray_out, gs, gc, grad_np.astype(np.float64), dtype, f"k16 {dtype}")


def test_k16_partitioned_equals_plain_full_size():
    """All 262,144 rays: the K=16 partitioned render equals the K=1 single pass."""
    w = synth.WORKLOADS[2]
    g = xl.xl_gen(w, torch.float32)
    p = xl.xl_gen(w.plain(), torch.float32)
    assert torch.equal(p["seg_offsets"][-1:], g["seg_offsets"][-1:])
    z = torch.zeros((7, w.n_rays), device="cuda")
    ray_k, _, _ = run(g, z)
    ray_1, _, _ = run(p, z)
    from tests.parity import tuple_report
    rep = assert_tuples(ray_k.cpu().numpy(), ray_1.cpu().numpy().astype(np.float64), "ray",
                        "k16 vs k1 on device, all rays")
    say("k16 vs plain max rel:", rep["rel"])


@pytest.mark.parametrize("chunk", [0, 11])
def test_k64_chunk_bf16_fp64_merge(chunk):
    w = synth.WORKLOADS[4]
    ray0 = chunk * synth.CHUNK_RAYS_K64
    g = xl.xl_gen(w, torch.bfloat16, ray0, synth.CHUNK_RAYS_K64)
    say(f"k64 chunk {chunk}: {g['sigma'].shape[0]} samples, {g['seg_ids'].shape[0]} segments")
    grad_np = np.random.default_rng(40 + chunk).normal(size=(7, synth.CHUNK_RAYS_K64)).astype(np.float32)
    ray_out, gs, gc = run(g, torch.from_numpy(grad_np).cuda(), fp64=True)
    rays = sample_rays(synth.CHUNK_RAYS_K64, 40, 41 + chunk)
    check_sampled(w, g, ray0, rays, ray_out, gs, gc, grad_np.astype(np.float64), torch.bfloat16,
                  f"k64 chunk {chunk}")


def test_k64_all_rays_one_launch_bf16_fp64_merge():
    """The large partition as the benchmark runs it: all 4,194,304 rays in one
    launch of each kernel (about 1.1G samples), sampled rays against the oracle."""
    w = synth.WORKLOADS[4]
    g = xl.xl_gen(w, torch.bfloat16)
    say(f"k64 all rays: {g['sigma'].shape[0]} samples, {g['seg_ids'].shape[0]} segments")
    grad_np = np.random.default_rng(44).normal(size=(7, w.n_rays)).astype(np.float32)
    ray_out, gs, gc = run(g, torch.from_numpy(grad_np).cuda(), fp64=True)
    rays = sample_rays(w.n_rays, 40, 45)
    check_sampled(w, g, 0, rays, ray_out, gs, gc, grad_np.astype(np.float64), torch.bfloat16,
                  "k64 all rays")
