"""Bytes the regions would exchange on K GPUs, sample-based vs segment-based.

Sample-based exchange (Sec. 4.2, the straightforward scheme): so that every GPU
can composite whole rays, each GPU broadcasts the attributes (density and
colour) of every sample it owns to the K - 1 others; the volume grows with
the samples per ray (the paper's O(S K^2) per ray).

Segment-based exchange (Sec. 4.3): each GPU first reduces its samples to one
tuple per ray segment (tau, colour, opacity, depth, distortion: 7 floats) and
broadcasts only those, independent of the sample count.

For inference both schemes gather to one GPU instead, which needs only what
the other GPUs own.  These are counts over a packed batch (no data moves on
one GPU).  The experiments (Sec. 5, multi-GPU communication) report the
measured synchronisation time falling by more than 2x between the two.
"""
from __future__ import annotations

import numpy as np

SAMPLE_BYTES = {"float32": 16, "bfloat16": 8, "float16": 8}  # density + rgb
TUPLE_BYTES = 7 * 4  # (tau, r, g, b, A, D, L) float32


def exchange_bytes(samples_per_region, segments_per_region, sample_bytes=16,
                   tuple_bytes=TUPLE_BYTES, gather_to=0) -> dict:
    """Exchange volume of both schemes for one batch.

    samples_per_region, segments_per_region: counts owned by each of the K
    regions (GPUs).  Training is an all-gather (each region's data reaches
    the K - 1 others); inference gathers to region `gather_to`."""
    s = np.asarray(samples_per_region, np.int64)
    g = np.asarray(segments_per_region, np.int64)
    if s.shape != g.shape or s.ndim != 1 or s.size == 0:
        raise ValueError("one sample count and one segment count per region")
    k = s.size
    others_s = int(s.sum() - s[gather_to])
    others_g = int(g.sum() - g[gather_to])
    train_s = int(s.sum()) * sample_bytes * (k - 1)
    train_g = int(g.sum()) * tuple_bytes * (k - 1)
    infer_s = others_s * sample_bytes
    infer_g = others_g * tuple_bytes

    def ratio(a, b):
        return a / b if b else float("inf") if a else 1.0

    return {"regions": k, "sample_bytes": sample_bytes, "tuple_bytes": tuple_bytes,
            "train_sample_based": train_s, "train_segment_based": train_g,
            "train_ratio": ratio(train_s, train_g),
            "infer_sample_based": infer_s, "infer_segment_based": infer_g,
            "infer_ratio": ratio(infer_s, infer_g)}


def allgather_bytes(n_samples, n_segments, regions, sample_bytes=16,
                    tuple_bytes=TUPLE_BYTES) -> dict:
    """Training all-gather volume of both schemes from batch totals alone:
    every sample (or segment tuple) reaches the K - 1 other regions."""
    k1 = max(int(regions) - 1, 0)
    a = int(n_samples) * sample_bytes * k1
    b = int(n_segments) * tuple_bytes * k1
    return {"regions": int(regions), "sample_based": a, "segment_based": b,
            "ratio": (a / b) if b else None}


def batch_exchange(b, sample_bytes=16, tuple_bytes=TUPLE_BYTES, regions=None) -> dict:
    """exchange_bytes of a packed host batch (synth.Batch, with seg_box)."""
    k = int(regions if regions is not None else (b.seg_box.max() + 1 if b.n_seg else 1))
    seg_len = np.diff(b.seg_offsets)
    samples = np.bincount(b.seg_box, weights=seg_len, minlength=k).astype(np.int64)
    segments = np.bincount(b.seg_box, minlength=k).astype(np.int64)
    return exchange_bytes(samples, segments, sample_bytes, tuple_bytes)
