"""The region-aware merge (tuples staged through LDS per workgroup) against the
gathering merge, which the oracle tests pin: the two fold every ray in the
same order with the same arithmetic, so their results must be bitwise equal,
also where a workgroup falls back to gathering (ids of a region that are not
contiguous, more listed ids than LDS slots, invalid ids, boundaries that do
not describe the layout)."""
import sys

import numpy as np
import pytest
import torch

from paper_2404_16221_amd import _lib as xl
from paper_2404_16221_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def both(seg_out, ro, ids, roff, grad_ray, fp64):
    """(fwd, bwd) of the gathering merge and of the staged merge (forced at
    these sizes; by default it starts at 4M segments)."""
    out = []
    for r in (None, roff):
        f = xl.xl_merge_fwd(seg_out, ro, ids, fp64=fp64, region_offsets=r, staged=True)
        # every entry first holds a mark, so that untouched entries are seen
        g = xl.tuple_buffer(seg_out.shape[1], seg_out.device).fill_(7.0)
        g = xl.xl_merge_bwd(seg_out, ro, ids, grad_ray, g, fp64=fp64, region_offsets=r, staged=True)
        out.append((f, g))
    torch.cuda.synchronize()
    return out


def assert_same(res, what):
    (f0, g0), (f1, g1) = res
    assert torch.equal(f0, f1), what + ": forward differs"
    assert torch.equal(g0, g1), what + ": backward differs"


def tuples(n_seg, seed):
    """Random but plausible segment tuples [7, n_seg] on the device."""
    rng = np.random.default_rng(seed)
    t = np.empty((7, n_seg), np.float32)
    t[0] = rng.exponential(0.7, n_seg)          # tau
    a = -np.expm1(-t[0])
    t[1:4] = a * rng.random((3, n_seg))         # colour
    t[4] = a                                    # opacity
    t[5] = a * rng.uniform(0.5, 3.0, n_seg)     # depth
    t[6] = a * a * rng.random(n_seg)            # distortion
    return xl.as_tuples(torch.from_numpy(t).cuda())


def region_layout(n_rays, K, present, order_seed):
    """Region-major ids: region k holds, in ray order, the rays r with
    present[r, k]; each ray lists its segments in a random order."""
    rng = np.random.default_rng(order_seed)
    counts = present.sum(axis=0)
    roff = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    rank = np.cumsum(present, axis=0) - 1          # rank of ray r inside region k
    ids, ro = [], [0]
    for r in range(n_rays):
        ks = np.flatnonzero(present[r])
        rng.shuffle(ks)
        ids.extend(int(roff[k] + rank[r, k]) for k in ks)
        ro.append(len(ids))
    return (np.asarray(ro, np.int64), np.asarray(ids, np.int64), roff)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("fp64", [False, True])
def test_generated_k8_layout(fp64):
    """All 65,536 rays of the K=8 workload, generated on the device."""
    w = synth.WORKLOADS[1]
    g = xl.xl_gen(w, torch.float32)
    seg_out, _ = xl.xl_render_segments_fwd(g["sigma"], g["rgb"], g["t_start"], g["t_end"],
                                           g["seg_offsets"])
    grad = torch.from_numpy(np.random.default_rng(5).normal(size=(7, w.n_rays)).astype(np.float32)).cuda()
    say(f"k8: {seg_out.shape[1]} segments, regions {g['region_offsets'].cpu().numpy().tolist()}")
    assert_same(both(seg_out, g["ray_offsets"], g["seg_ids"], g["region_offsets"], grad, fp64),
                f"k8 fp64={fp64}")


@pytest.mark.parametrize("segs", [1, 3, 5])
def test_synthetic_region_layouts(segs):
    """Rays crossing `segs` of 8 regions on average (up to all 8: 2,048 ids
    for a workgroup of 256 rays, beyond the LDS slots, falls back)."""
    n_rays, K = 5000, 8
    rng = np.random.default_rng(segs)
    present = rng.random((n_rays, K)) < segs / K
    present[rng.random(n_rays) < 0.05] = False      # rays without segments
    present[1024:1280] = True                       # one workgroup over the slots
    ro, ids, roff = region_layout(n_rays, K, present, 100 + segs)
    seg_out = tuples(ids.size, 200 + segs)
    grad = dev(rng.normal(size=(7, n_rays)).astype(np.float32))
    say(f"segs {segs}: {ids.size} segments")
    for fp64 in (False, True):
        assert_same(both(seg_out, dev(ro), dev(ids), dev(roff), grad, fp64), f"segs {segs} fp64={fp64}")


def test_long_rays():
    """Rays of 9 to 70 segments (backward: up to 64 staged, longer gather)."""
    rng = np.random.default_rng(11)
    n_rays, K = 800, 80
    present = rng.random((n_rays, K)) < 0.02
    present[100:105, :70] = True          # 70 segments: the workgroup gathers backward
    present[300:320, :40] = True          # 40 segments: staged, five groups of eight
    present[600:620, :9] = True           # 9 segments: two groups
    ro, ids, roff = region_layout(n_rays, K, present, 12)
    per_block = [int(ro[min(b + 256, n_rays)] - ro[b]) for b in range(0, n_rays, 256)]
    assert max(per_block) <= 1280, per_block  # every workgroup fits its LDS slots
    seg_out = tuples(ids.size, 13)
    grad = dev(rng.normal(size=(7, n_rays)).astype(np.float32))
    for fp64 in (False, True):
        assert_same(both(seg_out, dev(ro), dev(ids), dev(roff), grad, fp64), f"long rays fp64={fp64}")


def test_default_policy_small_layout_gathers():
    """Boundaries given, 122K segments, no flag: the gathering form (same bits)."""
    w = synth.WORKLOADS[1]
    g = xl.xl_gen(w, torch.float32)
    seg_out, _ = xl.xl_render_segments_fwd(g["sigma"], g["rgb"], g["t_start"], g["t_end"],
                                           g["seg_offsets"])
    a = xl.xl_merge_fwd(seg_out, g["ray_offsets"], g["seg_ids"])
    b = xl.xl_merge_fwd(seg_out, g["ray_offsets"], g["seg_ids"], region_offsets=g["region_offsets"])
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_fallback_cases():
    n_rays, K = 3000, 6
    rng = np.random.default_rng(7)
    present = rng.random((n_rays, K)) < 0.5
    ro, ids, roff = region_layout(n_rays, K, present, 8)
    n_seg = ids.size
    seg_out = tuples(n_seg, 9)
    grad = dev(rng.normal(size=(7, n_rays)).astype(np.float32))
    # 1. ids of region 2 permuted inside the region: runs no longer contiguous
    perm = np.arange(n_seg)
    a, b = roff[2], roff[3]
    perm[a:b] = a + rng.permutation(b - a)
    ids_p = perm[ids]
    seg_p = xl.tuple_buffer(n_seg, seg_out.device)
    seg_p[:, dev(perm)] = seg_out
    ref = both(seg_out, dev(ro), dev(ids), dev(roff), grad, False)
    got = both(seg_p, dev(ro), dev(ids_p), dev(roff), grad, False)
    assert_same(got, "permuted region")
    assert torch.equal(got[1][0], ref[1][0]), "permuted ids change the rays"
    # 2. invalid ids inside the lists (skipped as identities)
    ids_bad = ids.copy()
    ids_bad[::97] = -1
    ids_bad[5::101] = n_seg + 3
    assert_same(both(seg_out, dev(ro), dev(ids_bad), dev(roff), grad, False), "invalid ids")
    # 3. one region for everything, and boundaries that are not increasing
    assert_same(both(seg_out, dev(ro), dev(ids), dev(np.array([0, n_seg], np.int64)), grad, False),
                "one region")
    bad = roff.copy()
    bad[2], bad[3] = bad[3], bad[2]
    assert_same(both(seg_out, dev(ro), dev(ids), dev(bad), grad, False), "boundaries not increasing")
    # 4. no rays and no segments
    e = torch.zeros((7, 0), device="cuda")
    z = both(e, dev(np.zeros(1, np.int64)), dev(np.zeros(0, np.int64)), dev(np.zeros(2, np.int64)),
             torch.zeros((7, 0), device="cuda"), False)
    assert z[1][0].shape == (7, 0)


def test_tuple_arrays_must_be_records():
    """A plain [7, n] tensor is not the records layout: refused before any launch."""
    for n in (3, 1):
        ro = dev(np.array([0, n], np.int64))
        ids = dev(np.arange(n, dtype=np.int64))
        plain = torch.zeros((7, n), device="cuda")
        with pytest.raises(ValueError, match="tuple records"):
            xl.xl_merge_fwd(plain, ro, ids)
    ro = dev(np.array([0, 2, 3], np.int64))
    ids = dev(np.array([0, 1, 2], np.int64))
    rec = xl.tuple_buffer(3, "cuda", zero=True)
    out = xl.xl_merge_fwd(rec, ro, ids)
    torch.cuda.synchronize()
    assert torch.equal(out[0].cpu(), torch.ones(2))  # identity tuples: T = 1
