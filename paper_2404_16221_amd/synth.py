"""Seeded synthetic ray samples packed by spatial region.

This module is the input generator shared by the tests, the benchmark and the
oracle checks.  It holds none of the rendering arithmetic: it draws samples
and lays them out, nothing else.

Shape of the data (the paper's setting, Sec. 4.2 "Non-overlapped NeRFs"): the
scene cube [-1, 1]^3 is split into a grid of disjoint axis-aligned boxes, one
NeRF (in the paper, one GPU) per box.  Every ray carries sorted, non-overlapping
sample intervals; the samples of one ray that fall in one box form one
contiguous run, a *segment* (boxes are convex, so a straight ray meets each box
in one interval).  Samples are stored region-major: all segments of box 0 (in
ray order), then box 1, and so on, which is how each GPU in the paper holds the
samples of its own box.  The per-ray order of segments (Alg. 1/2's index list
I) is given by ``ray_offsets``/``seg_ids``.

Random numbers are counter based, so any ray can be regenerated alone: value
``s`` of ray ``r`` is ``mix64(key(r) + (s + 1) * GAMMA)``, where ``mix64`` is
the SplitMix64 output function (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) and ``key(r) = mix64(mix64(seed)
+ r * GAMMA)``.

Per ray (slots 0..255):
  * origin o ~ U[-1, 1)^3 (53-bit uniforms)                 (slots 0, 1, 2)
  * sample count N ~ U{n_min..n_max} (multiply-shift range)  (slot 3)
  * start offset u                                          (slot 4)
  * direction: uniform on the sphere by rejection from the cube (tries j, slots
    16 + 3j .. 16 + 3j + 2, at most 64 tries)
Per sample i, two draws (slots 256 + 2 i and 256 + 2 i + 1), cut into fields:
  * first draw, bits 63..40: width delta = -width_mean * log(u), u in (0, 1]
    bits 39..20 and 19..0: density sigma = exp(mu + s z) with
    z = sqrt(-2 ln u1) cos(2 pi u2), u1 in (0, 1], u2 in [0, 1)
  * second draw, 16-bit fields: bits 63..48 zero the density when below
    zero_frac; bits 47..32, 31..16, 15..0: colour r, g, b in [0, 1)
Widths are rescaled to sum to t_far when they exceed it; the intervals are
contiguous from a start drawn uniformly in [0, t_far - sum].

Bit-exact reproducibility: every value is built only from IEEE operations in a
fixed order -- float32 ``log_f32``, ``exp_f32`` and ``cos2pi_f32`` below (series
with exact range reductions, no fused multiply-add), correctly rounded square
roots and divisions, sequential float64 position sums -- so the device twin of
this generator yields bit-identical samples, box tags and layout.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Dict, Optional, Sequence, Tuple

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_S30, _S27, _S31 = np.uint64(30), np.uint64(27), np.uint64(31)
_S11, _S32 = np.uint64(11), np.uint64(32)
_INV53 = 1.0 / 9007199254740992.0  # 2^-53

SEED_BASE = 2404_16221
RAY_SLOTS = 256
SAMPLE_STRIDE = 2
DIR_TRIES = 64
_S40 = np.uint64(40)
_LO32 = np.uint64(0xFFFFFFFF)
_INV32 = 1.0 / 4294967296.0  # 2^-32
_INV24 = np.float32(1.0 / 16777216.0)  # 2^-24
# float32 constants of log_f32, given as exact bit patterns
_F32 = lambda bits: np.array([bits], dtype=np.uint32).view(np.float32)[0]
_SQRT2 = _F32(0x3FB504F3)     # 1.41421354
_THIRD = _F32(0x3EAAAAAB)     # 1/3
_FIFTH = _F32(0x3E4CCCCD)     # 1/5
_SEVENTH = _F32(0x3E124925)   # 1/7
_NINTH = _F32(0x3DE38E39)     # 1/9
_LN2 = _F32(0x3F317218)       # ln 2
_ONE = np.float32(1.0)
_TWO = np.float32(2.0)
_HALF = np.float32(0.5)


_INV_LN2 = _F32(0x3FB8AA3B)   # 1/ln 2
_LN2_HI = _F32(0x3F317200)    # ln 2, high part (few mantissa bits: k * hi is exact)
_LN2_LO = _F32(0x35BFBE8E)    # ln 2 - hi
_PI_2 = _F32(0x3FC90FDB)      # pi / 2


def exp_f32(y: np.ndarray) -> np.ndarray:
    """exp of float32 values in (-87, 88), float32 IEEE operations only.

    k = rint(y / ln 2), r = (y - k ln2_hi) - k ln2_lo (Cody & Waite), exp r by its
    Taylor series to r^7 in Horner form, times 2^k (exact)."""
    y = np.asarray(y, dtype=np.float32)
    k = np.rint(y * _INV_LN2).astype(np.float32)
    r = (y - k * _LN2_HI) - k * _LN2_LO
    p = np.float32(1.0) + r * np.float32(1.0 / 7.0)
    for d in (6, 5, 4, 3, 2, 1):
        p = np.float32(1.0) + (r * np.float32(1.0 / d)) * p
    return np.ldexp(p, k.astype(np.int32)).astype(np.float32)


def cos2pi_f32(u: np.ndarray) -> np.ndarray:
    """cos(2 pi u) for float32 u in [0, 1), float32 IEEE operations only.

    Quadrant n and fraction f of 4u are exact; the angle a in [0, pi/4] is f or
    1 - f times pi/2; sin a and cos a by their Taylor series to a^9 and a^8."""
    u = np.asarray(u, dtype=np.float32)
    t = u * np.float32(4.0)
    n = np.floor(t)
    f = t - n
    flip = f > np.float32(0.5)
    a = np.where(flip, np.float32(1.0) - f, f).astype(np.float32) * _PI_2
    a2 = a * a
    c = np.float32(1.0) - (a2 * np.float32(0.5)) * (np.float32(1.0) - (a2 * np.float32(1.0 / 12.0)) * (
        np.float32(1.0) - (a2 * np.float32(1.0 / 30.0)) * (np.float32(1.0) - a2 * np.float32(1.0 / 56.0))))
    sn = a * (np.float32(1.0) - (a2 * np.float32(1.0 / 6.0)) * (np.float32(1.0) - (a2 * np.float32(1.0 / 20.0)) * (
        np.float32(1.0) - (a2 * np.float32(1.0 / 42.0)) * (np.float32(1.0) - a2 * np.float32(1.0 / 72.0)))))
    ca = np.where(flip, sn, c)   # cos of the quadrant's angle
    sa = np.where(flip, c, sn)   # sin of the quadrant's angle
    n = n.astype(np.int32) & 3
    out = np.where(n == 0, ca, np.where(n == 1, -sa, np.where(n == 2, -ca, sa)))
    return out.astype(np.float32)


def log_f32(u: np.ndarray) -> np.ndarray:
    """Natural log of positive normal float32 values, float32 IEEE operations only.

    u = 2^e x with x in [sqrt(1/2), sqrt(2)); log x = 2 atanh(s), s = (x-1)/(x+1),
    summed as 2 (s + s^3/3 + s^5/5 + s^7/7 + s^9/9) (|s| < 0.172).  Every step is
    one correctly rounded float32 operation in a fixed order, so any IEEE twin
    gives the same bits.
    """
    u = np.asarray(u, dtype=np.float32)
    bits = u.view(np.int32)
    e = ((bits >> 23) & 0xFF).astype(np.int32) - 127
    x = ((bits & 0x7FFFFF) | 0x3F800000).view(np.float32)
    big = x > _SQRT2
    x = np.where(big, x * _HALF, x).astype(np.float32)
    e = e + big.astype(np.int32)
    s = (x - _ONE) / (x + _ONE)
    s2 = s * s
    p = _SEVENTH + s2 * _NINTH
    p = _FIFTH + s2 * p
    p = _THIRD + s2 * p
    p = s2 * p
    lx = _TWO * (s + s * p)
    return (e.astype(np.float32) * _LN2 + lx).astype(np.float32)


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function on uint64 arrays (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64).copy()
    z ^= z >> _S30
    z *= _M1
    z ^= z >> _S27
    z *= _M2
    z ^= z >> _S31
    return z


def ray_keys(seed: int, rays: np.ndarray) -> np.ndarray:
    s = mix64(np.array([seed], dtype=np.uint64))[0]
    with np.errstate(over="ignore"):
        return mix64(s + np.asarray(rays, dtype=np.uint64) * GAMMA)


def draw(keys: np.ndarray, slots) -> np.ndarray:
    with np.errstate(over="ignore"):
        return mix64(keys + (np.asarray(slots, dtype=np.uint64) + np.uint64(1)) * GAMMA)


def u01(v: np.ndarray) -> np.ndarray:
    """Uniform double in [0, 1)."""
    return (v >> _S11).astype(np.float64) * _INV53


def u01_open0(v: np.ndarray) -> np.ndarray:
    """Uniform double in (0, 1]."""
    return ((v >> _S11) + np.uint64(1)).astype(np.float64) * _INV53


def field(v: np.ndarray, shift: int, bits: int) -> np.ndarray:
    """Bits [shift, shift + bits) of v as a uniform double k / 2^bits in [0, 1)."""
    k = (v >> np.uint64(shift)) & np.uint64((1 << bits) - 1)
    return k.astype(np.float64) * (1.0 / float(1 << bits))


def u24_open0(v: np.ndarray) -> np.ndarray:
    """Upper 24 bits as a uniform float32 in (0, 1] (exact)."""
    return ((v >> _S40) + np.uint64(1)).astype(np.float32) * _INV24


@dataclass(frozen=True)
class Workload:
    """Generator parameters for one synthetic workload."""
    name: str
    n_rays: int
    n_min: int
    n_max: int
    sigma_mu: float
    sigma_s: float
    zero_frac: float
    grid: Tuple[int, int, int]
    seed: int
    width_mean: float = 0.02
    t_far: float = 3.0

    @property
    def k(self) -> int:
        return self.grid[0] * self.grid[1] * self.grid[2]

    def plain(self) -> "Workload":
        """The same samples as one K=1 region (one segment per ray)."""
        return replace(self, name=self.name + "-plain", grid=(1, 1, 1))


# The five workloads: 0 parity (K=1), 1 merge check (K=8), 2 training batch
# (K=16), 3 serving scene (K=32, rays per request set by the image size),
# 4 large partition (K=64, processed in chunks of 262,144 rays).
WORKLOADS: Dict[int, Workload] = {
    0: Workload("k1-4096r", 4096, 1, 128, 0.0, 1.5, 0.0, (1, 1, 1), SEED_BASE + 0),
    1: Workload("k8-65536r", 65536, 1, 256, 0.0, 1.5, 0.0, (2, 2, 2), SEED_BASE + 1),
    2: Workload("k16-262144r", 262144, 8, 1024, 0.0, 2.0, 0.3, (4, 2, 2), SEED_BASE + 2),
    3: Workload("k32-serve", 256 * 256, 16, 512, 0.0, 1.5, 0.0, (4, 4, 2), SEED_BASE + 3),
    4: Workload("k64-4194304r", 4194304, 32, 512, 0.0, 1.5, 0.0, (4, 4, 4), SEED_BASE + 4),
}
CHUNK_RAYS_K64 = 262144
SERVE_SIZES = ((256, 256), (512, 512), (1280, 720), (1920, 1080))


@dataclass
class Batch:
    """Packed samples of a set of rays (host arrays).

    sigma[n] f32, rgb[n,3] f32, t_start[n] f32, t_end[n] f32: samples,
    region-major.  seg_offsets[n_seg+1] i64: CSR over samples.  ray_offsets[R+1]
    i64 and seg_ids[n_seg] i64: segment ids of each ray, front to back.
    seg_box[n_seg] i32, seg_ray[n_seg] i64: bookkeeping for tests.
    """
    sigma: np.ndarray
    rgb: np.ndarray
    t_start: np.ndarray
    t_end: np.ndarray
    seg_offsets: np.ndarray
    ray_offsets: np.ndarray
    seg_ids: np.ndarray
    seg_box: np.ndarray
    seg_ray: np.ndarray
    rays: np.ndarray
    workload: Optional[Workload] = None

    @property
    def n(self) -> int:
        return int(self.sigma.shape[0])

    @property
    def n_seg(self) -> int:
        return int(self.seg_offsets.shape[0] - 1)

    @property
    def n_rays(self) -> int:
        return int(self.ray_offsets.shape[0] - 1)

    def region_offsets(self, n_regions: Optional[int] = None) -> np.ndarray:
        """First segment of each region, then n_seg: int64 [K + 1] (K defaults
        to the workload's box count, else one more than the largest box)."""
        if n_regions is None:
            if self.workload is not None:
                g = self.workload.grid
                n_regions = int(g[0] * g[1] * g[2])
            else:
                n_regions = int(self.seg_box.max()) + 1 if self.seg_box.size else 1
        return np.searchsorted(self.seg_box, np.arange(n_regions + 1), side="left").astype(np.int64)

    def ray_sample_index(self, r: int) -> np.ndarray:
        """Indices of ray r's samples in t order (its segments front to back)."""
        parts = [np.arange(self.seg_offsets[s], self.seg_offsets[s + 1])
                 for s in self.seg_ids[self.ray_offsets[r]:self.ray_offsets[r + 1]]]
        if not parts:
            return np.zeros(0, dtype=np.int64)
        return np.concatenate(parts)

    def ray_segments(self, r: int) -> np.ndarray:
        return self.seg_ids[self.ray_offsets[r]:self.ray_offsets[r + 1]]


def _directions(keys: np.ndarray) -> np.ndarray:
    n = keys.shape[0]
    d = np.zeros((n, 3), dtype=np.float64)
    d[:, 2] = 1.0
    todo = np.arange(n)
    for j in range(DIR_TRIES):
        if todo.size == 0:
            break
        k = keys[todo]
        v = np.stack([2.0 * u01(draw(k, 16 + 3 * j + c)) - 1.0 for c in range(3)], axis=1)
        r2 = (v * v).sum(axis=1)
        ok = (r2 > 1e-12) & (r2 <= 1.0)
        sel = todo[ok]
        d[sel] = v[ok] / np.sqrt(r2[ok])[:, None]
        todo = todo[~ok]
    return d


def _gen_ray_major(w: Workload, rays: np.ndarray):
    """Samples of `rays` in ray-major order plus per-sample box tags."""
    rays = np.asarray(rays, dtype=np.int64)
    keys = ray_keys(w.seed, rays)
    R = rays.shape[0]
    o = np.stack([2.0 * u01(draw(keys, c)) - 1.0 for c in range(3)], axis=1)
    span = np.uint64(w.n_max - w.n_min + 1)
    cnt = (np.int64(w.n_min) + (((draw(keys, 3) >> _S32) * span) >> _S32).astype(np.int64))
    u_start = u01(draw(keys, 4))
    d = _directions(keys)

    off = np.zeros(R + 1, dtype=np.int64)
    np.cumsum(cnt, out=off[1:])
    n = int(off[-1])
    ray_of = np.repeat(np.arange(R, dtype=np.int64), cnt)
    idx = np.arange(n, dtype=np.int64) - off[ray_of]
    sk = keys[ray_of]
    base = np.uint64(RAY_SLOTS) + idx.astype(np.uint64) * np.uint64(SAMPLE_STRIDE)

    wm = np.float32(w.width_mean)
    v1 = draw(sk, base)
    v2 = draw(sk, base + np.uint64(1))
    width = (-(wm * log_f32(u24_open0(v1)))).astype(np.float64)
    u1 = (field(v1, 20, 20) + 2.0 ** -20).astype(np.float32)   # exact: 20-bit values
    u2 = field(v1, 0, 20).astype(np.float32)
    z = np.sqrt(np.float32(-2.0) * log_f32(u1)) * cos2pi_f32(u2)
    sigma = exp_f32(np.float32(w.sigma_mu) + np.float32(w.sigma_s) * z).astype(np.float64)
    if w.zero_frac > 0.0:
        sigma[field(v2, 48, 16) < w.zero_frac] = 0.0
    rgb = np.stack([field(v2, 32, 16), field(v2, 16, 16), field(v2, 0, 16)], axis=1)
    del sk, base, v1, v2, z

    # Per-ray width sums and starts; positions by a sequential per-ray sum.
    nmax = int(cnt.max()) if R else 0
    pad = np.zeros((R, nmax), dtype=np.float64)
    pad[ray_of, idx] = width
    tot = np.cumsum(pad, axis=1)[:, -1] if nmax else np.zeros(R)
    scale = np.where(tot > w.t_far, w.t_far / np.where(tot > 0, tot, 1.0), 1.0)
    pad *= scale[:, None]
    s0 = u_start * np.maximum(w.t_far - tot * scale, 0.0)
    # Sample i ends at s0 + (delta_0 + ... + delta_i), summed left to right, and
    # starts where sample i-1 ends, so consecutive intervals share an end point.
    pad[:, 0] += s0
    edges = np.cumsum(pad, axis=1)
    del pad
    t_end64 = edges[ray_of, idx]
    t_start64 = s0[ray_of].copy()
    inner = idx > 0
    t_start64[inner] = edges[ray_of[inner], idx[inner] - 1]
    del edges
    t_start = t_start64.astype(np.float32)
    t_end = t_end64.astype(np.float32)

    # Box tag of each sample from its midpoint (computed from the stored f32 ends).
    mid = 0.5 * (t_start.astype(np.float64) + t_end.astype(np.float64))
    p = o[ray_of] + mid[:, None] * d[ray_of]
    g = np.array(w.grid, dtype=np.int64)
    cell = np.clip(np.floor((p + 1.0) * 0.5 * g).astype(np.int64), 0, g - 1)
    box = (cell[:, 0] + g[0] * (cell[:, 1] + g[1] * cell[:, 2])).astype(np.int32)
    return dict(sigma=sigma.astype(np.float32), rgb=rgb.astype(np.float32),
                t_start=t_start, t_end=t_end, box=box, off=off, ray_of=ray_of)


def _gen_chunk(args):
    w, sub = args
    return _gen_ray_major(w, sub)


def generate(w: Workload, rays: Optional[Sequence[int]] = None,
             chunk: int = 32768, processes: int = 1) -> Batch:
    """Generate the rays `rays` (default: all of w) and pack them region-major.

    `processes` > 1 generates ray chunks in worker processes (same result)."""
    if rays is None:
        rays = np.arange(w.n_rays, dtype=np.int64)
    rays = np.asarray(rays, dtype=np.int64)
    subs = [rays[c0:c0 + chunk] for c0 in range(0, rays.shape[0], chunk)]
    if processes > 1 and len(subs) > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(min(processes, len(subs))) as pool:
            parts = pool.map(_gen_chunk, [(w, sub) for sub in subs])
    else:
        parts = [_gen_ray_major(w, sub) for sub in subs]
    if not parts:
        z32 = np.zeros(0, np.float32)
        return Batch(z32, np.zeros((0, 3), np.float32), z32, z32,
                     np.zeros(1, np.int64), np.zeros(1, np.int64),
                     np.zeros(0, np.int64), np.zeros(0, np.int32),
                     np.zeros(0, np.int64), rays, w)
    sigma = np.concatenate([q["sigma"] for q in parts])
    rgb = np.concatenate([q["rgb"] for q in parts])
    t_start = np.concatenate([q["t_start"] for q in parts])
    t_end = np.concatenate([q["t_end"] for q in parts])
    box = np.concatenate([q["box"] for q in parts])
    ray_of, base = [], 0
    for q in parts:
        ray_of.append(q["ray_of"] + base)
        base += q["off"].shape[0] - 1
    ray_of = np.concatenate(ray_of)
    del parts
    return pack(sigma, rgb, t_start, t_end, box, ray_of, rays.shape[0], rays, w)


def pack(sigma, rgb, t_start, t_end, box, ray_of, n_rays, rays=None, w=None) -> Batch:
    """Cut ray-major samples into segments (runs of one box) and pack region-major."""
    n = sigma.shape[0]
    head = np.ones(n, dtype=bool)
    if n > 1:
        head[1:] = (box[1:] != box[:-1]) | (ray_of[1:] != ray_of[:-1])
    seg_start = np.flatnonzero(head)
    n_seg = seg_start.shape[0]
    seg_len = np.diff(np.append(seg_start, n))
    seg_box = box[seg_start]
    seg_ray = ray_of[seg_start]
    # Region-major: stable order by box keeps ray order (and t order) inside a box.
    order = np.argsort(seg_box.astype(np.uint8 if seg_box.size == 0 or seg_box.max() < 256
                                      else np.int32), kind="stable")
    new_len = seg_len[order]
    seg_offsets = np.zeros(n_seg + 1, dtype=np.int64)
    np.cumsum(new_len, out=seg_offsets[1:])
    gather = np.repeat(seg_start[order] - seg_offsets[:-1], new_len) + np.arange(n, dtype=np.int64)
    new_of_old = np.empty(n_seg, dtype=np.int64)
    new_of_old[order] = np.arange(n_seg, dtype=np.int64)
    segs_per_ray = np.bincount(seg_ray, minlength=n_rays).astype(np.int64)
    ray_offsets = np.zeros(n_rays + 1, dtype=np.int64)
    np.cumsum(segs_per_ray, out=ray_offsets[1:])
    return Batch(sigma=sigma[gather], rgb=rgb[gather], t_start=t_start[gather],
                 t_end=t_end[gather], seg_offsets=seg_offsets, ray_offsets=ray_offsets,
                 seg_ids=new_of_old, seg_box=seg_box[order].astype(np.int32),
                 seg_ray=seg_ray[order].astype(np.int64),
                 rays=np.arange(n_rays) if rays is None else np.asarray(rays), workload=w)


def serve_workload(width: int, height: int, seed: int) -> Workload:
    """The serving scene (K=32) at one image size: one ray per pixel."""
    return replace(WORKLOADS[3], name=f"k32-serve-{width}x{height}", n_rays=width * height,
                   seed=seed)


# ---------------------------------------------------------------- ray-major inputs
# Inputs of the sample-distribution step: rays (origin, direction) and their
# samples before any region is known.  The same seeded rays as the workloads.

def ray_geometry(w: Workload, rays: Sequence[int]) -> Tuple[np.ndarray, np.ndarray]:
    """Origins and unit directions (float64 [R, 3]) of rays `rays` of workload w."""
    rays = np.asarray(rays, dtype=np.int64)
    keys = ray_keys(w.seed, rays)
    o = np.stack([2.0 * u01(draw(keys, c)) - 1.0 for c in range(3)], axis=1)
    return o, _directions(keys)


def sample_points(w: Workload, rays: Sequence[int]) -> np.ndarray:
    """Float32 [n, 3] midpoints of the samples of `rays`: a point cloud from
    discretised rays, the stand-in for structure-from-motion points."""
    b = generate(w.plain(), rays=rays)
    o, d = ray_geometry(w, rays)
    ray_of = np.repeat(np.arange(len(rays)), np.diff(b.ray_offsets))
    seg_len = np.diff(b.seg_offsets)
    sample_ray = np.repeat(ray_of, seg_len)
    mid = 0.5 * (b.t_start.astype(np.float64) + b.t_end.astype(np.float64))
    return (o[sample_ray] + mid[:, None] * d[sample_ray]).astype(np.float32)


def random_rays(seed: int, n_rays: int, n_max: int, spread: float = 1.0,
                zero_frac: float = 0.05):
    """Small random ray batches for parity cases: origins U[-spread, spread)^3,
    unit directions, 0..n_max samples per ray with exponential widths (mean
    0.05) and a fraction of zero-length samples.  Returns float32 origins,
    dirs [R, 3], t_start, t_end [n] and int64 ray_offsets [R + 1]."""
    rng = np.random.default_rng(seed)
    o = rng.uniform(-spread, spread, size=(n_rays, 3)).astype(np.float32)
    d = rng.normal(size=(n_rays, 3))
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    cnt = rng.integers(0, n_max + 1, size=n_rays)
    ro = np.zeros(n_rays + 1, np.int64)
    np.cumsum(cnt, out=ro[1:])
    ts, te = [], []
    for c in cnt:
        wd = rng.exponential(0.05, size=c)
        wd[rng.random(c) < zero_frac] = 0.0
        e = np.cumsum(wd) + rng.uniform(0, 0.5)
        s = np.concatenate([[e[0] - wd[0]], e[:-1]]) if c else e
        ts.append(s.astype(np.float32))
        te.append(e.astype(np.float32))
    ts = np.concatenate(ts) if ts else np.zeros(0, np.float32)
    te = np.concatenate(te) if te else np.zeros(0, np.float32)
    return o, d, ts, np.maximum(te, ts), ro


def grid_tree(grid: Tuple[int, int, int], lo: float = -1.0, hi: float = 1.0):
    """A uniform gx x gy x gz grid over [lo, hi]^3 (power-of-two sides) as a
    partition tree in heap order: each level halves the axis with the most
    cells left (ties to x, then y).  Returns (axis, plane, levels)."""
    g = [int(v) for v in grid]
    for v in g:
        if v < 1 or v & (v - 1):
            raise ValueError("grid sides must be powers of two")
    levels = sum(v.bit_length() - 1 for v in g)
    axis = np.zeros((1 << levels) - 1, np.int32)
    plane = np.zeros((1 << levels) - 1, np.float32)

    def split(node, c0, c1, depth):
        if depth == levels:
            return
        sizes = [c1[a] - c0[a] for a in range(3)]
        a = int(np.argmax(sizes))
        m = (c0[a] + c1[a]) // 2
        axis[node] = a
        plane[node] = np.float32(lo + (hi - lo) * m / g[a])
        c1_low, c0_high = list(c1), list(c0)
        c1_low[a] = c0_high[a] = m
        split(2 * node + 1, c0, c1_low, depth + 1)
        split(2 * node + 2, c0_high, c1, depth + 1)

    split(0, [0, 0, 0], g, 0)
    return axis, plane, levels
