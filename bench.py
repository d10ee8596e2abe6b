#!/usr/bin/env python3
"""Benchmark of the partitioned renderer on one MI355X.

Metric: composited samples/s for one training step (per-segment composite,
merge, merge backward, per-segment backward) over the K=16 training batch
(262,144 rays, 8..1024 samples per ray, about 135M samples, density
lognormal(0, 2) with 30% empty samples), BF16 sample storage.  The same step
is also timed with FP32 storage and in the plain form (FP32, the same samples
as one K=1 segment per ray).  Inputs are resident in HBM before timing starts.

Prints one JSON line.  Options: --steps K --warmup W --gpus 1 [--no-cpu-baseline].
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "composited samples/s (fwd+bwd) at K regions vs FP32 plain; p50/p99 render ms"
HBM_PEAK_GBS = 8000.0
# Sources that define the segment kernels; HBM traffic measured with rocprofv3
# counters is reported only while these are unchanged.
KERNEL_SOURCES = ("paper_2404_16221_amd/csrc/segments.hip", "paper_2404_16221_amd/csrc/xl_device.hpp")
TRAFFIC_PROFILE = "profiles/seg_bwd_kernel_k16-262144r_bf16_traffic.md"


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def profile_fields():
    """Fields of the committed counter summary of the dominant kernel (HBM
    bytes from FETCH_SIZE and WRITE_SIZE, each scaled by the same counter on a
    1 GiB device copy; VALU busy), or {} if the kernel sources changed since
    the counters were taken."""
    path = os.path.join(HERE, TRAFFIC_PROFILE)
    if not os.path.exists(path):
        return {}
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line and line.strip().startswith("- "):
                k, v = line.strip()[2:].split(":", 1)
                fields[k.strip()] = v.strip().strip("`")
    if fields.get("kernel_source_sha256") != kernel_source_hash():
        return {}
    return fields


def profile_number(key):
    try:
        return float(profile_fields()[key])
    except (KeyError, ValueError):
        return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def plain_arrays(b):
    """The same samples as one segment per ray (ray-major), from a packed batch."""
    seg_len = np.diff(b.seg_offsets)
    order = b.seg_ids  # ray-major list of segments, front to back
    lens = seg_len[order]
    starts = b.seg_offsets[:-1][order]
    dst = np.zeros(lens.size + 1, np.int64)
    np.cumsum(lens, out=dst[1:])
    gather = np.repeat(starts - dst[:-1], lens) + np.arange(b.n, dtype=np.int64)
    counts = np.diff(b.ray_offsets)
    per_ray = np.add.reduceat(lens, b.ray_offsets[:-1]) if b.n_rays else np.zeros(0, np.int64)
    per_ray = np.where(counts > 0, per_ray, 0)
    seg_offsets = np.zeros(b.n_rays + 1, np.int64)
    np.cumsum(per_ray, out=seg_offsets[1:])
    return gather, seg_offsets


class Form:
    """Device buffers of one form of the step, preallocated."""

    def __init__(self, name, sigma, rgb, t0, t1, seg_offsets, ray_offsets, seg_ids, grad_ray,
                 regions, fp64=False):
        from paper_2404_16221_amd import _lib as xl
        self.xl = xl
        self.name, self.regions, self.fp64 = name, regions, fp64
        self.sigma, self.rgb, self.t0, self.t1 = sigma, rgb, t0, t1
        self.seg_offsets, self.ray_offsets, self.seg_ids = seg_offsets, ray_offsets, seg_ids
        self.n, self.n_seg, self.n_rays = sigma.shape[0], seg_offsets.shape[0] - 1, ray_offsets.shape[0] - 1
        dev = sigma.device
        self.seg_out = torch.empty((7, self.n_seg), dtype=torch.float32, device=dev)
        self.ws = torch.empty(xl.xl_segments_workspace_bytes(self.n), dtype=torch.uint8, device=dev)
        self.ray_out = torch.empty((7, self.n_rays), dtype=torch.float32, device=dev)
        self.grad_ray = grad_ray
        self.grad_seg = torch.zeros((7, self.n_seg), dtype=torch.float32, device=dev)
        self.gs = torch.empty_like(sigma)
        self.gc = torch.empty_like(rgb)

    def release(self):
        for k in list(vars(self)):
            if isinstance(getattr(self, k), torch.Tensor):
                setattr(self, k, None)

    def step(self, ev=None):
        xl = self.xl
        xl.xl_render_segments_fwd(self.sigma, self.rgb, self.t0, self.t1, self.seg_offsets,
                                  self.seg_out, self.ws)
        xl.xl_merge_fwd(self.seg_out, self.ray_offsets, self.seg_ids, self.ray_out, fp64=self.fp64)
        xl.xl_merge_bwd(self.seg_out, self.ray_offsets, self.seg_ids, self.grad_ray, self.grad_seg,
                        fp64=self.fp64)
        if ev is not None:
            ev[0].record()
        xl.xl_render_segments_bwd(self.sigma, self.rgb, self.t0, self.t1, self.seg_offsets, self.ws,
                                  self.grad_seg, self.gs, self.gc)
        if ev is not None:
            ev[1].record()

    def bytes_step(self):
        """Algorithmic HBM bytes of one step (fwd+bwd): per sample, segment and ray."""
        es = self.sigma.element_size()
        per_sample = 2 * (4 * es + 8) + 4 * es        # read sigma,rgb,t0,t1 twice; write dsigma,drgb
        per_seg = 8 + 28 + (28 + 8) + (28 + 8 + 28) + (8 + 28)  # offsets, tuple, merge, merge bwd, seg bwd
        per_ray = 16 + 28 + 16 + 28                   # offsets + out, offsets + grad
        return self.n * per_sample + self.n_seg * per_seg + self.n_rays * per_ray

    def bytes_seg_bwd(self):
        es = self.sigma.element_size()
        return self.n * (4 * es + 8 + 4 * es) + self.n_seg * (8 + 28)


def time_form(f: Form, steps: int, warmup: int):
    for _ in range(warmup):
        f.step()
    torch.cuda.synchronize()
    kern = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            for _ in range(steps)]
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall = time.perf_counter()
    t0.record()
    for k in range(steps):
        f.step(kern[k])
    t1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall
    ms = t0.elapsed_time(t1) / steps
    kms = float(np.mean([a.elapsed_time(b) for a, b in kern]))
    return ms, kms, wall


def cpu_baseline(w, budget_s=15.0):
    """The FP64 oracle, single thread, fwd+bwd on a bounded sample of rays."""
    from oracle import render as O
    from paper_2404_16221_amd import synth
    torch.set_num_threads(1)
    rng = np.random.default_rng(7)

    def run(k):
        rays = np.sort(rng.choice(w.n_rays, size=k, replace=False))
        b = synth.generate(w, rays=rays)
        g = rng.normal(size=(7, b.n_rays))
        t = time.perf_counter()
        O.render_rays_partitioned(b.sigma, b.rgb, b.t_start, b.t_end, b.seg_offsets, b.ray_offsets,
                                  b.seg_ids)
        O.backward_partitioned(b.sigma, b.rgb, b.t_start, b.t_end, b.seg_offsets, b.ray_offsets,
                               b.seg_ids, g)
        return time.perf_counter() - t, b.n

    dt, n = run(4)
    k = int(max(4, min(16384, 4 * budget_s / max(dt, 1e-3))))
    dt, n = run(k)
    return {"value": n / dt, "unit": "samples/s", "cores": 1, "kind": "oracle",
            "sample": f"{k} random rays of the {w.name} workload ({n} samples), FP64 oracle, "
                      f"segment composite + merge + merge backward + segment backward, {dt:.1f} s"}


def serve_stream(n_req, warmup, rate, dtype, slots, seed=2404_16221 + 103):
    """Poisson arrivals of view requests (sizes uniform over the four image sizes,
    K=32 scene) against the render server; latency per request."""
    import threading
    from paper_2404_16221_amd import synth
    from paper_2404_16221_amd.serve import Server, request
    w3 = synth.WORKLOADS[3]
    scene = dict(grid=w3.grid, n_min=w3.n_min, n_max=w3.n_max, sigma_mu=w3.sigma_mu,
                 sigma_s=w3.sigma_s, zero_frac=w3.zero_frac)
    rng = np.random.default_rng(seed)
    total = n_req + warmup
    gaps = rng.exponential(1.0 / rate, size=total)
    sizes = rng.integers(0, len(synth.SERVE_SIZES), size=total)
    tickets = [None] * total
    submitted = [0.0] * total
    srv = Server(hbm_budget_bytes=64 << 30, max_slots=slots, max_queue=4096, dtype=dtype)
    t_start = time.perf_counter()

    def producer():
        t = t_start
        for i in range(total):
            t += gaps[i]
            d = t - time.perf_counter()
            if d > 0:
                time.sleep(d)
            wdt, hgt = synth.SERVE_SIZES[sizes[i]]
            submitted[i] = time.perf_counter()
            tickets[i] = srv.submit(request(wdt, hgt, seed=seed + 1000 + i, **scene))

    th = threading.Thread(target=producer)
    th.start()
    res = []
    for i in range(total):
        while tickets[i] is None:
            time.sleep(0.0005)
        r = srv.poll(tickets[i], timeout_us=-1)
        if r["rc"] != 0:
            raise RuntimeError(f"request {i} failed: {r}")
        srv.release(tickets[i])
        res.append(r)
    th.join()
    srv.close()
    m = res[warmup:]
    lat = np.array([r["latency_us"] for r in m]) / 1e3
    sub = np.array(submitted[warmup:])
    span = float((sub + lat / 1e3).max() - sub.min())
    samples = sum(r["n_samples"] for r in m)
    return {"requests": n_req, "warmup": warmup, "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
            "device_ms_mean": float(np.mean([r["device_us"] for r in m]) / 1e3),
            "requests_per_s": n_req / span, "samples_per_s": samples / span}


def serving(n_req, warmup, rate):
    """Continuous batching (FP16, 4 slots) and the FIFO single-request FP32 baseline
    at the offered rate; then continuous batching again at 70 % of the rate it
    sustained, where latency is service time rather than queueing."""
    cb = serve_stream(n_req, warmup, rate, torch.float16, slots=4)
    log("serving fp16 x4 slots:", json.dumps(cb))
    fifo = serve_stream(max(n_req // 3, 20), max(warmup // 3, 5), rate, torch.float32, slots=1)
    log("serving fifo fp32:", json.dumps(fifo))
    out = {"workload": "k32 scene, Poisson %.0f/s, sizes 256^2/512^2/1280x720/1920x1080" % rate,
           "continuous_batching_fp16": cb, "fifo_fp32_baseline": fifo}
    sustained = min(rate, cb["requests_per_s"])
    if sustained < rate:
        light = 0.7 * sustained
        lt = serve_stream(max(n_req // 2, 20), max(warmup // 2, 5), light, torch.float16, slots=4)
        lt["rate_per_s"] = light
        log("serving fp16 x4 slots below capacity:", json.dumps(lt))
        out["continuous_batching_fp16_at_70pct_capacity"] = lt
    return out


def distribution(steps, warmup):
    """Sample distribution (tag / split / pack) of all rays of a workload
    (ray-major) into its boxes, for the uniform grid and for the CDF partition
    built from the samples of a subset of its rays; time per pack (plan, whose
    size read-back synchronises, plus fill) and samples per box.  The k16
    batch (16 boxes) and the k64 large partition (64 boxes)."""
    from paper_2404_16221_amd import _lib as xl
    from paper_2404_16221_amd import synth
    res = {}
    for w, every, dtype in ((synth.WORKLOADS[2], 64, torch.float32),
                            (synth.WORKLOADS[4], 1024, torch.bfloat16)):
        g = xl.xl_gen(w.plain(), dtype)
        del g["sigma"], g["rgb"], g["seg_ids"]
        o, d = synth.ray_geometry(w, np.arange(w.n_rays))
        o = torch.from_numpy(o.astype(np.float32)).cuda()
        d = torch.from_numpy(d.astype(np.float32)).cuda()
        grid_axis, grid_plane, levels = synth.grid_tree(w.grid)
        K = 1 << levels
        t = time.perf_counter()
        pts = synth.sample_points(w, np.arange(0, w.n_rays, every))
        t_pts = time.perf_counter() - t
        t = time.perf_counter()
        cdf = xl.xl_partition_build(pts, levels)
        t_build = time.perf_counter() - t
        n_in = g["t_start"].shape[0]
        r = {"workload": f"{w.name} rays, ray-major, {n_in} samples, {K} boxes",
             "cdf_points": int(pts.shape[0]), "cdf_build_s": t_build, "cdf_points_s": t_pts}
        gname = "grid_" + "x".join(str(v) for v in w.grid)
        for name, (axis, plane) in ((gname, (grid_axis, grid_plane)), ("cdf", cdf)):
            def call(src=True):
                return xl.xl_pack(o, d, g["t_start"], g["t_end"], g["seg_offsets"], axis, plane,
                                  levels, with_src=src)
            for _ in range(warmup):
                out = call()
            del out
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(steps):
                out = call()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            n, n_seg = out["t_start"].shape[0], out["seg_ids"].shape[0]
            seg_len = (out["seg_offsets"][1:] - out["seg_offsets"][:-1]).double()
            per_box = torch.zeros(K, dtype=torch.float64, device="cuda").index_add_(
                0, out["seg_box"].long(), seg_len).cpu().numpy()
            del out, seg_len
            alg = n_in * 8 + w.n_rays * (24 + 8 + 8) + n * 16 + n_seg * 20
            r[name] = {"ms": ms, "samples_per_s": n_in / (ms * 1e-3), "pieces": int(n),
                       "segments": int(n_seg), "algorithmic_gbs": alg / (ms * 1e-3) / 1e9,
                       "samples_per_box_max_over_mean": float(per_box.max() / per_box.mean()),
                       "samples_per_box_min_over_mean": float(per_box.min() / per_box.mean()),
                       "samples_per_box_cv": float(per_box.std() / per_box.mean())}
            # the same pack without the optional source index of every piece
            e0.record()
            for _ in range(steps):
                out = call(False)
            e1.record()
            torch.cuda.synchronize()
            r[name]["ms_without_src"] = e0.elapsed_time(e1) / steps
            del out
            log("distribution", w.name, name, json.dumps(r[name]))
        res[w.name] = r
        del g, o, d
        torch.cuda.empty_cache()
    return res


def feature_channels(f, steps, warmup, F=16):
    """F feature channels (App. B.2) over the samples of form f: segment
    features, merge, merge backward and per-sample backward per step; the
    features are a hash of the sample index in f's storage type."""
    from paper_2404_16221_amd import _lib as xl
    dev = f.sigma.device
    idx = torch.arange(f.n, device=dev)
    x = idx[:, None] * F + torch.arange(F, device=dev)[None, :]
    x = (x * 2654435761) % 4294967296
    feat = ((x.float() / 2147483648.0) - 1.0).to(f.sigma.dtype)
    del idx, x
    g = torch.from_numpy(np.random.default_rng(6).normal(size=(F, f.n_rays)).astype(np.float32)).to(dev)
    phi = torch.empty((F, f.n_seg), dtype=torch.float32, device=dev)
    tau = torch.empty(f.n_seg, dtype=torch.float32, device=dev)
    out = torch.empty((F, f.n_rays), dtype=torch.float32, device=dev)
    gs = torch.empty_like(f.sigma)
    gf = torch.empty_like(feat)

    def step(ev=None):
        xl.xl_render_features_fwd(f.sigma, feat, f.t0, f.t1, f.seg_offsets, phi, tau)
        xl.xl_merge_features_fwd(tau, phi, f.ray_offsets, f.seg_ids, out)
        gphi, gtau = xl.xl_merge_features_bwd(tau, phi, f.ray_offsets, f.seg_ids, g)
        if ev is not None:
            ev[0].record()
        xl.xl_render_features_bwd(f.sigma, feat, f.t0, f.t1, f.seg_offsets, phi, gphi, gtau, gs, gf)
        if ev is not None:
            ev[1].record()

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    kern = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            for _ in range(steps)]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(steps):
        step(kern[k])
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    kms = float(np.mean([a.elapsed_time(b) for a, b in kern]))
    es = f.sigma.element_size()
    # algorithmic bytes: per sample sigma, t0, t1, features read twice, dsigma and
    # dfeat written; per segment the features, depth and their gradients
    per_sample = 2 * (es + 8 + F * es) + es + F * es
    per_seg = (8 + 4 * F + 4) + (8 + 4 * F + 4) + (8 + 4 * F + 4 + 4 * F + 4) + (8 + 8 * F + 4)
    per_ray = 16 + 4 * F + 16 + 4 * F
    step_bytes = f.n * per_sample + f.n_seg * per_seg + f.n_rays * per_ray
    bwd_bytes = f.n * (es + 8 + F * es + es + F * es) + f.n_seg * (8 + 8 * F + 4)
    res = {"workload": f"{f.name} samples, {F} feature channels ({str(f.sigma.dtype)[6:]})",
           "ms_per_step": ms, "samples_per_s": f.n / (ms * 1e-3),
           "step_gbs": step_bytes / (ms * 1e-3) / 1e9, "bwd_ms": kms,
           "bwd_gbs": bwd_bytes / (kms * 1e-3) / 1e9,
           "bwd_frac_of_hbm_peak": bwd_bytes / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    log("features", json.dumps(res))
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="bf16,fp32,plain,k64")
    ap.add_argument("--no-features", action="store_true", help="skip the feature-channel timing")
    ap.add_argument("--no-distribution", action="store_true",
                    help="skip the tag/split/pack timing")
    ap.add_argument("--serve-requests", type=int, default=300,
                    help="measured serving requests (0 skips the serving run)")
    ap.add_argument("--serve-warmup", type=int, default=30)
    ap.add_argument("--serve-rate", type=float, default=200.0, help="Poisson arrivals per second")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy 1 GiB device to device (scales HBM byte counters)")
    args = ap.parse_args()
    if args.calibrate_copy:
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "device copy", "bytes_read": x.numel() * 4,
                          "bytes_written": y.numel() * 4}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): the exchange of segment "
              "tuples between GPUs is not implemented.", file=sys.stderr)
        sys.exit(2)
    import paper_2404_16221_amd  # noqa: F401  (fails loudly without libxl.so)
    from paper_2404_16221_amd import _lib as xl
    from paper_2404_16221_amd import synth
    from paper_2404_16221_amd.exchange import allgather_bytes
    dev = torch.device("cuda:0")
    w = synth.WORKLOADS[2]
    want = args.forms.split(",")
    forms, results = {}, {}
    grad_ray = torch.from_numpy(
        np.random.default_rng(3).normal(size=(7, w.n_rays)).astype(np.float32)).to(dev)

    def make(name, workload, dtype, regions, fp64=False, grad=None):
        t = time.perf_counter()
        g = xl.xl_gen(workload, dtype)
        torch.cuda.synchronize()
        log(f"generated {name} on the device: {g['sigma'].shape[0]} samples, "
            f"{g['seg_ids'].shape[0]} segments in {time.perf_counter() - t:.2f} s")
        return Form(name, g["sigma"], g["rgb"], g["t_start"], g["t_end"], g["seg_offsets"],
                    g["ray_offsets"], g["seg_ids"], grad_ray if grad is None else grad, regions,
                    fp64=fp64)

    if "bf16" in want:
        forms["bf16"] = make("k16-bf16", w, torch.bfloat16, 16)
    if "fp32" in want:
        forms["fp32"] = make("k16-fp32", w, torch.float32, 16)
    if "plain" in want:
        forms["plain"] = make("k1-plain-fp32", w.plain(), torch.float32, 1)
    if "k64" in want:
        # the large partition, all 4,194,304 rays resident at once (18 GB of
        # BF16/FP32 samples fit in HBM), with the FP64 cross-segment merge
        w64 = synth.WORKLOADS[4]
        g64 = torch.from_numpy(
            np.random.default_rng(4).normal(size=(7, w64.n_rays)).astype(np.float32)).to(dev)
        forms["k64"] = make("k64-bf16-fp64merge", w64, torch.bfloat16, 64, fp64=True, grad=g64)
    for key, f in forms.items():
        ms, kms, wall = time_form(f, args.steps, args.warmup)
        results[key] = dict(name=f.name, ms_per_step=ms, samples_per_s=f.n / (ms * 1e-3),
                            step_gbs=f.bytes_step() / (ms * 1e-3) / 1e9,
                            seg_bwd_ms=kms, seg_bwd_gbs=f.bytes_seg_bwd() / (kms * 1e-3) / 1e9,
                            wall_s=wall)
        # bytes the K regions would all-gather per training step (one GPU
        # moves none): per-sample (sigma, rgb) in the storage type vs FP32
        # segment tuples
        xb = allgather_bytes(f.n, f.n_seg, f.regions, 4 * f.sigma.element_size())
        results[key]["exchange_sample_mb"] = xb["sample_based"] / 1e6
        results[key]["exchange_tuple_mb"] = xb["segment_based"] / 1e6
        log(key, json.dumps(results[key]))
    head = "bf16" if "bf16" in results else next(iter(results))
    hf, hr = forms[head], results[head]
    out = {
        "metric": METRIC, "value": hr["samples_per_s"], "unit": "samples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": hr["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "rays": hf.n_rays, "samples": hf.n, "segments": hf.n_seg,
                   "regions": hf.regions, "storage": str(hf.sigma.dtype).replace("torch.", ""),
                   "passes": "segment fwd + merge fwd + merge bwd + segment bwd"},
        "forms": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                  for k, v in results.items()},
        "roofline": {"bound": "hbm", "achieved": hr["seg_bwd_gbs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": hr["seg_bwd_gbs"] / HBM_PEAK_GBS,
                     "traffic": profile_number("hbm_bytes_per_launch") if head == "bf16" else None,
                     "valu_busy": profile_number("valu_busy") if head == "bf16" else None,
                     "algorithmic_bytes": hf.bytes_seg_bwd(),
                     "kernel": "seg_bwd_kernel", "step_achieved": hr["step_gbs"],
                     "step_frac": hr["step_gbs"] / HBM_PEAK_GBS},
    }
    if not args.no_features and "bf16" in forms:
        out["features"] = feature_channels(forms["bf16"], args.steps, args.warmup)
    if not args.no_distribution:
        out["distribution"] = distribution(max(args.steps // 2, 3), 2)
    if args.serve_requests > 0:
        for f in forms.values():
            f.release()
        forms.clear()
        torch.cuda.empty_cache()
        out["serving"] = serving(args.serve_requests, args.serve_warmup, args.serve_rate)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
