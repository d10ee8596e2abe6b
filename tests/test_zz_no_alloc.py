"""The no-allocation forward entry point (tile records in the library's static
scratch) against the workspace entry point, through the C ABI."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2404_16221_amd import _lib as xl
from paper_2404_16221_amd import synth

MAX_SAMPLES = 168_427_520  # largest n whose tile records fit XL_STATIC_SCRATCH_BYTES


def test_static_limit_and_rejection_on_the_host():
    L = xl.lib()
    assert L.xl_segments_workspace_bytes(MAX_SAMPLES) <= 64 << 20 < L.xl_segments_workspace_bytes(MAX_SAMPLES + 1)
    # beyond the limit: rejected before anything touches the device
    s = xl.XLSamples(0, 16, 16, 16, 16, MAX_SAMPLES + 1)
    assert L.xl_render_segments_fwd_static(ctypes.byref(s), 16, 1, 16, None) == xl.XL_EINVAL
    assert "static scratch" in L.xl_last_error().decode()
    assert L.xl_render_segments_fwd_static(None, 16, 1, 16, None) == xl.XL_EINVAL


def _inputs(cfg, n_rays, dtype):
    g = xl.xl_gen(synth.WORKLOADS[cfg], dtype, 0, n_rays)
    return g["sigma"], g["rgb"], g["t_start"], g["t_end"], g["seg_offsets"]


@pytest.mark.gpu
def test_static_forward_equals_workspace_forward_twice():
    # a large call, then a smaller one: the second must not see the first's records
    for cfg, n_rays, dtype in ((2, 65536, torch.bfloat16), (0, 1000, torch.float32),
                               (1, 300, torch.float16)):
        args = _inputs(cfg, n_rays, dtype)
        ref, _ = xl.xl_render_segments_fwd(*args)
        got = xl.xl_render_segments_fwd_static(*args)
        torch.cuda.synchronize()
        print(f"workload {cfg}, {n_rays} rays: {args[0].shape[0]} samples", flush=True)
        assert torch.equal(got, ref)
