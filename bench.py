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
    k = int(max(4, min(2048, 4 * budget_s / max(dt, 1e-3))))
    dt, n = run(k)
    return {"value": n / dt, "unit": "samples/s", "cores": 1, "kind": "oracle",
            "sample": f"{k} random rays of the {w.name} workload ({n} samples), FP64 oracle, "
                      f"segment composite + merge + merge backward + segment backward, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="bf16,fp32,plain")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU exchange "
              "of segment tuples is a design in DESIGN.md, not part of this build.", file=sys.stderr)
        sys.exit(2)
    import paper_2404_16221_amd  # noqa: F401  (fails loudly without libxl.so)
    from paper_2404_16221_amd import synth
    dev = torch.device("cuda:0")
    w = synth.WORKLOADS[2]
    t = time.perf_counter()
    b = synth.generate(w, processes=min(16, os.cpu_count() or 1))
    log(f"generated {w.name}: {b.n} samples, {b.n_seg} segments in {time.perf_counter() - t:.1f} s")
    grad_ray = torch.from_numpy(np.random.default_rng(3).normal(size=(7, b.n_rays)).astype(np.float32)).to(dev)
    T = lambda a, dt=None: torch.from_numpy(np.ascontiguousarray(a)).to(dev, dtype=dt)
    t0, t1 = T(b.t_start), T(b.t_end)
    so, ro, ids = T(b.seg_offsets), T(b.ray_offsets), T(b.seg_ids)
    forms = {}
    want = args.forms.split(",")
    results = {}
    if "bf16" in want:
        forms["bf16"] = Form("k16-bf16", T(b.sigma, torch.bfloat16), T(b.rgb, torch.bfloat16), t0, t1,
                             so, ro, ids, grad_ray, 16)
    if "fp32" in want:
        forms["fp32"] = Form("k16-fp32", T(b.sigma), T(b.rgb), t0, t1, so, ro, ids, grad_ray, 16)
    if "plain" in want:
        gather, pso = plain_arrays(b)
        forms["plain"] = Form("k1-plain-fp32", T(b.sigma[gather]), T(b.rgb[gather]),
                              T(b.t_start[gather]), T(b.t_end[gather]), T(pso),
                              T(np.arange(b.n_rays + 1, dtype=np.int64)),
                              T(np.arange(b.n_rays, dtype=np.int64)), grad_ray, 1)
    del b
    for key, f in forms.items():
        ms, kms, wall = time_form(f, args.steps, args.warmup)
        results[key] = dict(name=f.name, ms_per_step=ms, samples_per_s=f.n / (ms * 1e-3),
                            step_gbs=f.bytes_step() / (ms * 1e-3) / 1e9,
                            seg_bwd_ms=kms, seg_bwd_gbs=f.bytes_seg_bwd() / (kms * 1e-3) / 1e9,
                            wall_s=wall)
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
                     "unit": "GB/s", "frac": hr["seg_bwd_gbs"] / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "seg_bwd_kernel", "step_achieved": hr["step_gbs"],
                     "step_frac": hr["step_gbs"] / HBM_PEAK_GBS},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
