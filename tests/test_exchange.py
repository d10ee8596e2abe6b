"""Exchange-volume counts (host logic; no GPU)."""
import numpy as np
import pytest

from paper_2404_16221_amd import synth
from paper_2404_16221_amd.exchange import allgather_bytes, batch_exchange, exchange_bytes


def test_hand_counts():
    # 3 regions: 10, 0, 5 samples in 2, 0, 1 segments
    e = exchange_bytes([10, 0, 5], [2, 0, 1], sample_bytes=16, tuple_bytes=28)
    assert e["train_sample_based"] == 15 * 16 * 2
    assert e["train_segment_based"] == 3 * 28 * 2
    assert e["infer_sample_based"] == 5 * 16          # what regions 1, 2 own
    assert e["infer_segment_based"] == 1 * 28
    assert e["train_ratio"] == pytest.approx(480 / 168)


def test_one_region_exchanges_nothing():
    e = exchange_bytes([7], [1])
    assert e["train_sample_based"] == e["train_segment_based"] == 0
    assert e["infer_sample_based"] == e["infer_segment_based"] == 0


def test_batch_counts_match_layout():
    b = synth.generate(synth.WORKLOADS[1], rays=np.arange(512))
    e = batch_exchange(b)
    assert e["regions"] == 8
    assert e["train_sample_based"] == b.n * 16 * 7
    assert e["train_segment_based"] == b.n_seg * 28 * 7
    # segments hold many samples each: the segment-based exchange is far smaller
    assert e["train_ratio"] > 2.0 and e["infer_ratio"] > 2.0


def test_rejects_mismatched_counts():
    with pytest.raises(ValueError):
        exchange_bytes([1, 2], [1])


def test_allgather_totals_agree_with_per_region_counts():
    b = synth.generate(synth.WORKLOADS[1], rays=np.arange(300))
    e = batch_exchange(b, regions=8)
    a = allgather_bytes(b.n, b.n_seg, 8)
    assert a["sample_based"] == e["train_sample_based"]
    assert a["segment_based"] == e["train_segment_based"]
    assert allgather_bytes(b.n, b.n_seg, 1)["sample_based"] == 0
