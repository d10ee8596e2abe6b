"""Render server on the GPU: correctness, alone-vs-mix equality, admission, failures."""
import time

import numpy as np
import pytest
import torch

from oracle import render as O
from paper_2404_16221_amd import synth
from paper_2404_16221_amd.serve import Server, request
from tests.parity import assert_tuples, quantize, sample_rays

pytestmark = pytest.mark.gpu

SCENE = dict(grid=(4, 4, 2), n_min=16, n_max=512, sigma_mu=0.0, sigma_s=1.5)


def workload_of(width, height, seed):
    return synth.Workload(f"req-{width}x{height}", width * height, SCENE["n_min"], SCENE["n_max"],
                          SCENE["sigma_mu"], SCENE["sigma_s"], 0.0, SCENE["grid"], seed)


def wait_all(srv, tickets):
    return {t: srv.poll(t, timeout_us=60_000_000) for t in tickets}


def test_served_view_matches_oracle():
    with Server(max_slots=2, dtype=torch.float16) as srv:
        t = srv.submit(request(64, 48, seed=11, **SCENE))
        r = srv.poll(t, timeout_us=60_000_000)
        assert r["rc"] == 0, r
        out = srv.result(t, r["n_rays"]).cpu().numpy()
        srv.release(t)
    w = workload_of(64, 48, 11)
    rays = sample_rays(w.n_rays, 300, 1)
    b = synth.generate(w, rays=rays)
    assert r["n_rays"] == 64 * 48
    dq = quantize(b, torch.float16)
    ref = O.render_rays_single(dq[0], dq[1], b.t_start, b.t_end, b.seg_offsets, b.ray_offsets,
                               b.seg_ids)
    assert_tuples(out[:, rays], ref, "ray", "served view vs oracle (FP16 inputs)")


def test_result_is_the_same_alone_and_in_a_mix():
    target = request(200, 150, seed=5, **SCENE)
    with Server(max_slots=1, dtype=torch.float16) as srv:
        t = srv.submit(target)
        assert srv.poll(t, timeout_us=60_000_000)["rc"] == 0
        alone = srv.result(t, 200 * 150)
        srv.release(t)
    others = [request(w, h, seed=100 + k, **SCENE)
              for k, (w, h) in enumerate([(256, 256), (300, 200), (128, 128), (512, 256), (64, 64)])]
    with Server(max_slots=4, dtype=torch.float16) as srv:
        ts = [srv.submit(q) for q in others[:3]]
        tt = srv.submit(target)
        ts += [srv.submit(q) for q in others[3:]]
        res = wait_all(srv, ts + [tt])
        assert all(v["rc"] == 0 for v in res.values()), res
        mixed = srv.result(tt, 200 * 150)
        torch.cuda.synchronize()
        assert torch.equal(alone, mixed)
        st = srv.stats()
        assert st["completed"] == 6 and st["p99_latency_us"] >= st["p50_latency_us"] > 0
        for t in ts + [tt]:
            srv.release(t)


def test_slot_workspace_grows_and_results_stay_the_same():
    """One slot takes a small view, a larger one (its generator workspace,
    held outside the budget, grows), then the small one again: each result
    equals the same request served alone by a fresh server, bit for bit."""
    sizes = {"small": (64, 48), "large": (320, 240)}
    reqs = {k: request(w, h, seed=21 + i, **SCENE) for i, (k, (w, h)) in enumerate(sizes.items())}

    def alone(k):
        with Server(max_slots=1, dtype=torch.float16) as srv:
            t = srv.submit(reqs[k])
            assert srv.poll(t, timeout_us=60_000_000)["rc"] == 0
            out = srv.result(t, sizes[k][0] * sizes[k][1])
            torch.cuda.synchronize()
            srv.release(t)
        return out

    ref = {k: alone(k) for k in sizes}
    order = ["small", "large", "small"]
    with Server(max_slots=1, dtype=torch.float16) as srv:
        ts = [srv.submit(reqs[k]) for k in order]
        res = wait_all(srv, ts)
        assert all(v["rc"] == 0 for v in res.values()), res
        for k, t in zip(order, ts):
            out = srv.result(t, sizes[k][0] * sizes[k][1])
            torch.cuda.synchronize()
            assert torch.equal(out, ref[k]), k
            srv.release(t)
        assert srv.stats()["budget_used_bytes"] == 0


def test_queue_full_returns_eagain_and_accepted_requests_finish():
    with Server(max_slots=1, max_queue=2, dtype=torch.float16) as srv:
        tickets, rejected = [], 0
        for k in range(12):
            t = srv.submit(request(256, 256, seed=200 + k, **SCENE))
            if t is None:
                rejected += 1
            else:
                tickets.append(t)
        assert rejected > 0
        res = wait_all(srv, tickets)
        assert all(v["rc"] == 0 for v in res.values())
        for t in tickets:
            srv.release(t)


def test_budget_admission_and_injected_fault():
    # 24 MB: a 256x256 view (~17M samples) cannot fit, a 32x32 view can
    with Server(hbm_budget_bytes=24 << 20, max_slots=2, dtype=torch.float16) as srv:
        big = srv.submit(request(256, 256, seed=1, **SCENE))
        bad = srv.submit(request(32, 32, seed=2, inject_fault=True, **SCENE))
        small = [srv.submit(request(32, 32, seed=3 + k, **SCENE)) for k in range(4)]
        rb = srv.poll(big, timeout_us=60_000_000)
        rf = srv.poll(bad, timeout_us=60_000_000)
        assert rb["rc"] == -2 and "budget" in rb["error"]
        assert rf["rc"] == -5
        for t in small:
            r = srv.poll(t, timeout_us=60_000_000)
            assert r["rc"] == 0 and r["footprint_bytes"] <= 24 << 20
            srv.release(t)
        st = srv.stats()
        assert st["completed"] == 4 and st["failed"] == 2 and st["budget_used_bytes"] == 0


def test_continuous_batching_overlaps_requests():
    """Requests submitted while others run are admitted into free slots at once,
    and their device work overlaps (device intervals from one origin)."""
    with Server(max_slots=4, dtype=torch.float16) as srv:
        ts = [srv.submit(request(512, 512, seed=300 + k, **SCENE)) for k in range(4)]
        res = wait_all(srv, ts)
        assert all(v["rc"] == 0 for v in res.values())
        # all four were admitted without waiting for each other to finish
        assert max(v["queue_us"] for v in res.values()) < min(v["latency_us"] for v in res.values())
        iv = sorted((v["device_start_us"], v["device_end_us"]) for v in res.values())
        assert all(0 <= a < b for a, b in iv), iv
        overlap = sum(max(0, min(b1, b2) - max(a1, a2))
                      for i, (a1, b1) in enumerate(iv) for (a2, b2) in iv[i + 1:])
        print("device intervals (us):", iv, "pairwise overlap", overlap, flush=True)
        assert overlap > 0
        for t in ts:
            srv.release(t)


def test_held_result_and_over_budget_request():
    """A result the client still holds and a request larger than the whole
    budget: the latter fails with XL_ENOMEM at once instead of waiting for
    memory that could never suffice."""
    with Server(hbm_budget_bytes=64 << 20, max_slots=2, dtype=torch.float16) as srv:
        held = srv.submit(request(64, 64, seed=9, **SCENE))
        assert srv.poll(held, timeout_us=60_000_000)["rc"] == 0
        big = srv.submit(request(1280, 720, seed=10, **SCENE))
        t0 = time.perf_counter()
        r = srv.poll(big, timeout_us=60_000_000)
        assert r["rc"] == -2 and "budget" in r["error"], r
        assert time.perf_counter() - t0 < 30
        # a request that fits next to the held result still runs
        small = srv.submit(request(64, 64, seed=11, **SCENE))
        assert srv.poll(small, timeout_us=60_000_000)["rc"] == 0
        srv.release(small)
        srv.release(held)
        assert srv.stats()["budget_used_bytes"] == 0
