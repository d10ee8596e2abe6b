"""Partitioned volume rendering (NeRF-XL, arXiv 2404.16221) on AMD MI355X.

The compute path is libxl.so (hand-written HIP for gfx950 behind a C ABI,
include/xl.h); this package holds its ctypes binding (``_lib``), a
``torch.autograd.Function``s over it (``autograd``), the build script, the
seeded input generator (``synth``) and exchange-volume counts (``exchange``).
"""
from . import _lib  # noqa: F401
from ._lib import (xl_check_inputs, xl_merge_bwd, xl_merge_fwd, xl_render_segments_bwd,  # noqa: F401
                   xl_render_segments_fwd, xl_segments_workspace_bytes, xl_version)
from .autograd import XLFeatures, XLRender, render, render_features  # noqa: F401
