"""The FP64 oracle run over many rays in worker processes.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute this module: only the test suite, the smoke check of the build entry
point and the CPU-baseline leg of the benchmark do.  It shares no code with the
HIP library or its Python binding.

This module adds no arithmetic of its own.  It cuts a list of rays into chunks,
lays each chunk out ray by ray (a ray's segments front to back, each
segment's samples in t order), and has ``oracle.render`` compute, per chunk:

* every listed ray in one pass over its samples (the single-pass render);
* every segment of those rays alone (the per-region partial tuples);
* with upstream ray gradients, the partitioned backward (merge backward, then
  each segment's backward) from the hand-derived closed forms, which the tests
  pin against float64 autodiff of the definitions and against finite
  differences.  Workers use numpy alone: PyTorch's autograd engine counts the
  GPUs on its first use, which would open the GPU in every worker.

Results come back in that ray-major order, so a caller compares them with any
other layout of the same samples through ``ray_major_index``.

Processes are forked.  Create the pool before the calling process touches a
GPU (a forked child of a process with an initialised GPU runtime is not safe),
and keep it for the whole session: ``Pool(n)``, then pass it to ``run``.
"""
from __future__ import annotations

import multiprocessing as mp
import os
from typing import Optional

import numpy as np

from . import render as R


def ranges(starts, lens) -> np.ndarray:
    """Concatenation of arange(s, s + l) over the pairs (int64)."""
    starts = np.asarray(starts, np.int64)
    lens = np.asarray(lens, np.int64)
    tot = int(lens.sum())
    if tot == 0:
        return np.zeros(0, np.int64)
    first = np.zeros(lens.shape[0], np.int64)
    np.cumsum(lens[:-1], out=first[1:])
    return np.repeat(starts - first, lens) + np.arange(tot, dtype=np.int64)


def ray_major_index(seg_offsets, ray_offsets, seg_ids, rays):
    """Layout of the listed rays, ray by ray.

    Returns (segs, seg_len, segs_per_ray, samples): the ids of the rays'
    segments front to back, their lengths, the segment count of each ray, and
    the indices of their samples in that order.
    """
    seg_offsets = np.asarray(seg_offsets, np.int64)
    ray_offsets = np.asarray(ray_offsets, np.int64)
    seg_ids = np.asarray(seg_ids, np.int64)
    rays = np.asarray(rays, np.int64)
    k0 = ray_offsets[rays]
    spr = ray_offsets[rays + 1] - k0
    segs = seg_ids[ranges(k0, spr)]
    seg_len = seg_offsets[segs + 1] - seg_offsets[segs]
    samples = ranges(seg_offsets[segs], seg_len)
    return segs, seg_len, spr, samples


def _one_chunk(args):
    sigma, rgb, t0, t1, seg_len, spr, grad = args
    seg_offsets = np.zeros(seg_len.shape[0] + 1, np.int64)
    np.cumsum(seg_len, out=seg_offsets[1:])
    ray_offsets = np.zeros(spr.shape[0] + 1, np.int64)
    np.cumsum(spr, out=ray_offsets[1:])
    seg_ids = np.arange(seg_len.shape[0], dtype=np.int64)
    out = {"ray": R.render_rays_single(sigma, rgb, t0, t1, seg_offsets, ray_offsets, seg_ids),
           "seg": R.render_segments(sigma, rgb, t0, t1, seg_offsets)}
    if grad is not None:
        g_seg, segs, idx, ds, dc = R.backward_partitioned(sigma, rgb, t0, t1, seg_offsets,
                                                          ray_offsets, seg_ids, grad,
                                                          autodiff=False)
        # ray-major chunk: segments and samples come back in storage order
        assert np.array_equal(segs, seg_ids) and np.array_equal(idx, np.arange(sigma.shape[0]))
        out.update(grad_seg=g_seg, dsigma=ds, drgb=dc)
    return out


def _init_worker():
    # one thread per worker: the workers already use every core
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:
        pass


def Pool(processes: Optional[int] = None):
    """A fork-based worker pool (one process per host core by default, at most 16)."""
    if processes is None:
        processes = min(16, os.cpu_count() or 1)
    return mp.get_context("fork").Pool(processes, initializer=_init_worker)


def run(pool, sigma, rgb, t0, t1, seg_offsets, ray_offsets, seg_ids, rays, grad_ray=None,
        chunk_samples: int = 1 << 17):
    """Oracle results for the listed rays, ray-major (see the module docstring).

    sigma, rgb, t0, t1, seg_offsets, ray_offsets, seg_ids: any packed batch
    (host arrays).  grad_ray: [7, len(rays)] upstream gradients of the listed
    rays' (T, r, g, b, A, D, L), or None for the forward only.

    Returns a dict: ray [7, R]; seg [7, S] (the rays' segments front to back);
    with grad_ray also grad_seg [7, S], dsigma [N], drgb [N, 3] (the rays'
    samples front to back); and the layout (segs, samples) of
    ``ray_major_index``.
    """
    rays = np.asarray(rays, np.int64)
    segs, seg_len, spr, samples = ray_major_index(seg_offsets, ray_offsets, seg_ids, rays)
    sigma = np.asarray(sigma)[samples]
    rgb = np.asarray(rgb).reshape(-1, 3)[samples]
    t0 = np.asarray(t0)[samples]
    t1 = np.asarray(t1)[samples]
    # chunks of whole rays with about chunk_samples samples each
    seg_first = np.zeros(rays.shape[0] + 1, np.int64)
    np.cumsum(spr, out=seg_first[1:])
    per_seg_first = np.zeros(seg_len.shape[0] + 1, np.int64)
    np.cumsum(seg_len, out=per_seg_first[1:])
    ray_n = per_seg_first[seg_first[1:]] - per_seg_first[seg_first[:-1]]
    ray_first = np.zeros(rays.shape[0] + 1, np.int64)
    np.cumsum(ray_n, out=ray_first[1:])
    bounds = [0]
    acc = 0
    for r in range(rays.shape[0]):
        acc += int(ray_n[r])
        if acc >= chunk_samples:
            bounds.append(r + 1)
            acc = 0
    if bounds[-1] != rays.shape[0]:
        bounds.append(rays.shape[0])
    jobs = []
    for a, b in zip(bounds[:-1], bounds[1:]):
        s0, s1 = ray_first[a], ray_first[b]
        g0, g1 = seg_first[a], seg_first[b]
        jobs.append((sigma[s0:s1], rgb[s0:s1], t0[s0:s1], t1[s0:s1], seg_len[g0:g1], spr[a:b],
                     None if grad_ray is None else np.asarray(grad_ray, np.float64)[:, a:b]))
    parts = pool.map(_one_chunk, jobs) if pool is not None else [_one_chunk(j) for j in jobs]
    out = {"segs": segs, "samples": samples}
    if not parts:
        out.update(ray=np.zeros((7, 0)), seg=np.zeros((7, 0)))
        if grad_ray is not None:
            out.update(grad_seg=np.zeros((7, 0)), dsigma=np.zeros(0), drgb=np.zeros((0, 3)))
        return out
    for k in parts[0]:
        axis = 0 if k in ("dsigma", "drgb") else 1
        out[k] = np.concatenate([p[k] for p in parts], axis=axis)
    return out
