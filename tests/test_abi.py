"""C ABI checks that need no GPU: exported symbols and host-side argument errors."""
import ctypes
import os
import re

import pytest

from paper_2404_16221_amd import _lib as xl
from paper_2404_16221_amd import serve, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "xl.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(xl_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_function_is_exported():
    names = declared_functions()
    assert len(names) >= 18, names
    L = ctypes.CDLL(xl.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_bindings_cover_the_header():
    bound = set(xl.SIGNATURES) | set(serve.SERVE_SIGNATURES)
    assert set(declared_functions()) <= bound | {"xl_serve_create"}


def _fwd(s, seg_offsets=None, n_seg=1, seg_out=None, ws=None, wsb=0):
    return xl.lib().xl_render_segments_fwd(ctypes.byref(s) if s is not None else None,
                                           seg_offsets, n_seg, seg_out, ws, wsb, None)


def test_host_side_argument_errors():
    L = xl.lib()
    assert _fwd(None) == xl.XL_EINVAL
    s = xl.XLSamples(7, 16, 16, 16, 16, 4)
    assert _fwd(s, 16) == xl.XL_EINVAL and "dtype" in L.xl_last_error().decode()
    s = xl.XLSamples(0, 16, 16, 16, 16, -1)
    assert _fwd(s, 16) == xl.XL_EINVAL and "negative" in L.xl_last_error().decode()
    s = xl.XLSamples(0, 0x1004, 16, 16, 16, 4)
    assert _fwd(s, 16, 1, 16, 16, 1 << 20) == xl.XL_EINVAL and "aligned" in L.xl_last_error().decode()
    s = xl.XLSamples(0, 16, 16, 16, 16, 4)
    assert _fwd(s, 16, 0) == xl.XL_EINVAL and "no segments" in L.xl_last_error().decode()
    assert _fwd(s, 16, 1, 16, 16, 1) == xl.XL_EINVAL and "too small" in L.xl_last_error().decode()
    assert L.xl_merge_fwd(16, 1, None, 0, 16, 16, 1, 16, 4, None) == xl.XL_EINVAL
    assert "flags" in L.xl_last_error().decode()
    # tuple records must be 16-byte aligned
    assert L.xl_merge_fwd(8, 1, None, 0, 16, 16, 1, 16, 0, None) == xl.XL_EINVAL
    assert "aligned" in L.xl_last_error().decode()
    assert L.xl_merge_bwd(16, 1, None, 0, 16, 16, 1, 16, 8, 0, None) == xl.XL_EINVAL
    assert "aligned" in L.xl_last_error().decode()
    assert L.xl_merge_bwd(16, -1, None, 0, 16, 16, 1, 16, 16, 0, None) == xl.XL_EINVAL
    assert L.xl_merge_fwd(16, 1, 16, 0, 16, 16, 1, 16, 0, None) == xl.XL_EINVAL
    assert "n_regions" in L.xl_last_error().decode()
    assert L.xl_merge_bwd(16, 1, 16, -2, 16, 16, 1, 16, 16, 0, None) == xl.XL_EINVAL
    assert L.xl_render_segments_bwd(ctypes.byref(s), 16, 1, None, 0, 16, 16, 16, None) == xl.XL_EINVAL


def test_workspace_sizes():
    L = xl.lib()
    rec = L.xl_segments_workspace_bytes(1)
    assert rec > 0 and rec % 16 == 0
    assert L.xl_segments_workspace_bytes(0) == rec
    # one record per tile of a power-of-two number of samples
    tile = next(n for n in (2 ** k for k in range(6, 16)) if L.xl_segments_workspace_bytes(n + 1) > rec)
    assert L.xl_segments_workspace_bytes(tile) == rec
    assert L.xl_segments_workspace_bytes(tile + 1) == 2 * rec
    assert L.xl_segments_workspace_bytes(3 * tile + 1) == 4 * rec
    p = xl.gen_params(synth.WORKLOADS[2])
    assert L.xl_gen_workspace_bytes(ctypes.byref(p)) > 262144 * 8
    bad = xl.gen_params(synth.WORKLOADS[2])
    bad.grid[0] = 0
    assert L.xl_gen_workspace_bytes(ctypes.byref(bad)) == 0
    n, ns = ctypes.c_int64(), ctypes.c_int64()
    assert L.xl_gen_plan(ctypes.byref(bad), None, 0, ctypes.byref(n), ctypes.byref(ns), None) == xl.XL_EINVAL


def test_serve_argument_errors():
    L = serve._bind()
    cfg = serve.XLServeConfig(1 << 30, 0, 4, 0, 0, 0, 0)
    h = ctypes.c_void_p()
    assert L.xl_serve_create(ctypes.byref(cfg), ctypes.byref(h)) == xl.XL_EINVAL
    cfg = serve.XLServeConfig(1 << 30, 1, 4, 0, 9, 0, 0)
    assert L.xl_serve_create(ctypes.byref(cfg), ctypes.byref(h)) == xl.XL_EINVAL
    t = ctypes.c_uint64()
    req = serve.request(4, 4)
    assert L.xl_serve_submit(None, ctypes.byref(req), ctypes.byref(t)) == xl.XL_EINVAL
    r = serve.XLResult()
    assert L.xl_serve_poll(None, 1, ctypes.byref(r), 0) == xl.XL_EINVAL
    assert L.xl_serve_release(None, 1) == xl.XL_EINVAL


def test_pack_and_feature_argument_errors():
    L = xl.lib()
    assert L.xl_pack_workspace_bytes(-1, 4) == 0 and L.xl_pack_workspace_bytes(10, 7) == 0
    assert L.xl_pack_workspace_bytes(1000, 4) > 1000 * 16 * 8
    n, ns = ctypes.c_int64(), ctypes.c_int64()
    assert L.xl_pack_plan(None, 16, 16, 4, 16, 1 << 20, ctypes.byref(n), ctypes.byref(ns), None) == xl.XL_EINVAL
    rays = xl.XLRays(16, 16, 16, 16, 16, 10)
    assert L.xl_pack_plan(ctypes.byref(rays), 16, 16, 7, 16, 1 << 30, ctypes.byref(n), ctypes.byref(ns),
                          None) == xl.XL_EINVAL
    assert "levels" in L.xl_last_error().decode()
    assert L.xl_pack_plan(ctypes.byref(rays), None, None, 2, 16, 1 << 30, ctypes.byref(n),
                          ctypes.byref(ns), None) == xl.XL_EINVAL
    assert L.xl_pack_plan(ctypes.byref(rays), 16, 16, 2, 16, 1, ctypes.byref(n), ctypes.byref(ns),
                          None) == xl.XL_EINVAL and "too small" in L.xl_last_error().decode()
    f = xl.XLFeatures(0, 5, 16, 16, 16, 16, 4)
    assert L.xl_render_features_fwd(ctypes.byref(f), 16, 1, 16, 16, None) == xl.XL_EINVAL
    assert "n_feat" in L.xl_last_error().decode()
    f = xl.XLFeatures(0, 8, 16, 0x1008, 16, 16, 4)
    assert L.xl_render_features_fwd(ctypes.byref(f), 16, 1, 16, 16, None) == xl.XL_EINVAL
    assert "aligned" in L.xl_last_error().decode()
    assert L.xl_merge_features_fwd(16, 16, 3, 1, 16, 16, 1, 16, None) == xl.XL_EINVAL
    assert L.xl_merge_features_bwd(16, 16, 8, 1, 16, 16, 1, None, 16, 16, None) == xl.XL_EINVAL


def test_breakable_argument_errors():
    L = xl.lib()
    B = xl.XLBreakable

    def desc(dtype=0, source=0, F=3, pairs=((0, 1),), n=4):
        pa = ([a for a, _ in pairs] + [0] * 4)[:4]
        pb = ([b for _, b in pairs] + [0] * 4)[:4]
        return B(dtype, source, F, len(pairs), (ctypes.c_int32 * 4)(*pa), (ctypes.c_int32 * 4)(*pb),
                 16, 16, 16, 16, n)

    def fwd(d):
        return L.xl_render_breakable_fwd(ctypes.byref(d), 16, 1, 16, None)

    assert L.xl_render_breakable_fwd(None, 16, 1, 16, None) == xl.XL_EINVAL
    assert fwd(desc(dtype=9)) == xl.XL_EINVAL and "dtype" in L.xl_last_error().decode()
    assert fwd(desc(source=5)) == xl.XL_EINVAL and "source" in L.xl_last_error().decode()
    assert fwd(desc(F=0)) == xl.XL_EINVAL and "n_ch" in L.xl_last_error().decode()
    assert fwd(desc(F=9)) == xl.XL_EINVAL
    assert fwd(desc(pairs=((0, 3),))) == xl.XL_EINVAL and "outside" in L.xl_last_error().decode()
    assert fwd(desc(pairs=((0, 0),) * 5)) == xl.XL_EINVAL
    assert fwd(desc(n=-1)) == xl.XL_EINVAL
    d = desc()
    assert L.xl_merge_breakable_fwd(ctypes.byref(d), 16, 1, None, 16, 1, 16, None) == xl.XL_EINVAL
    assert L.xl_render_breakable_bwd(ctypes.byref(d), 16, 1, 16, 16, 16, None, 0, None) == xl.XL_EINVAL
