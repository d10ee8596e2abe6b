"""CPU oracle for spatial partitioning and sample distribution (NeRF-XL, arXiv 2404.16221).

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute this module: only the test suite, the smoke check of the build entry
point and the CPU-baseline leg of the benchmark do.  It shares no code with the
HIP library or its Python binding.

What it computes (plain and slow, no blocking or reordering):

* ``cdf_partition``: the recursive partition of Sec. 4.4 and App. A.3.  At
  every node, for each axis, the candidate plane is where the empirical CDF of
  the node's points along that axis reaches one half; the axis kept is the one
  whose two children are closest to cubic; the two children are split the same
  way, ``levels`` times, giving 2**levels boxes.  Readings (the paper states
  none of these details):
    - the CDF-one-half plane of m points is their order statistic of rank
      floor(m / 2) (0-based): with distinct coordinates exactly floor(m / 2)
      points lie below it; a node with no points uses the middle of its box;
    - a point goes to the low child when its coordinate is below the plane,
      else to the high child;
    - box extents for the aspect ratio are taken inside the bounding box of all
      points; the aspect ratio of a box is its longest extent over its
      shortest (a box with a zero extent has ratio infinity, or 1 when all
      three are zero); an axis scores the larger of its two children's ratios;
      the lowest score wins, ties going to the lower axis (x, y, z);
    - the outermost boxes extend to infinity, so every point of space belongs
      to exactly one box.
  The tree is stored in heap order: node i has children 2i+1 (low) and 2i+2
  (high); leaves are nodes 2**levels - 1 ... 2**(levels+1) - 2, and box b is
  leaf node b + 2**levels - 1.

* ``leaf_bounds``: the half-open box [lo, hi) of every leaf, by walking the
  splits from the root.

* ``tag_split_pack``: the distribution of ray samples to boxes (Sec. 4.2): no
  sample interval may reach across a box boundary, so every interval is cut
  at the points where its ray crosses box faces, every piece is tagged with
  its box, and the pieces are packed region-major (box 0's segments in ray
  order, then box 1's, ...), each ray's pieces in one box forming one segment
  (boxes are convex).  Written as the definition, box by box: box b's
  parameter interval along the ray is the slab intersection [t_in, t_out) in
  float64 (each face parameter is (face - origin) / direction), rounded to
  float32; the piece of sample [s, e) in box b is [max(s, t_in), min(e, t_out))
  when it has positive length, and a sample of zero length is kept whole in
  the box whose [t_in, t_out) holds s.  Pieces of one ray tile its samples.

Pins (tests marked "not gpu"): a uniform grid written as a tree tags points
like the grid's cell formula; balanced counts per box follow from the order
statistic; elongated point sets split along their long axis first; pieces
tile their samples and lie inside their boxes; brute-force point tagging of
piece midpoints; the one-box tree returns its input unchanged.
"""
from __future__ import annotations

import numpy as np


def aspect_ratio(ext) -> float:
    """Longest over shortest extent of a box (inf for a flat box, 1 for a point)."""
    mx = max(ext)
    mn = min(ext)
    if mn == 0.0:
        return 1.0 if mx == 0.0 else float("inf")
    return mx / mn


def cdf_partition(points, levels: int):
    """Recursive CDF-median partition of `points` [n, 3] (float32) into
    2**levels boxes.  Returns (axis int32 [2**levels - 1], plane float32 [...])."""
    p = np.asarray(points, dtype=np.float32).reshape(-1, 3)
    K = 1 << levels
    axis = np.zeros(K - 1, dtype=np.int32)
    plane = np.zeros(K - 1, dtype=np.float32)
    if p.shape[0]:
        lo0 = [float(p[:, a].min()) for a in range(3)]
        hi0 = [float(p[:, a].max()) for a in range(3)]
    else:
        lo0, hi0 = [0.0] * 3, [0.0] * 3

    def split(node, idx, lo, hi, depth):
        if depth == levels:
            return
        m = idx.shape[0]
        best = None
        for a in range(3):
            if m > 0:
                v = np.sort(p[idx, a])
                cut = np.float32(v[m // 2])
            else:
                cut = np.float32((lo[a] + hi[a]) / 2.0)
            left_ext = [hi[c] - lo[c] for c in range(3)]
            right_ext = list(left_ext)
            left_ext[a] = float(cut) - lo[a]
            right_ext[a] = hi[a] - float(cut)
            score = max(aspect_ratio(left_ext), aspect_ratio(right_ext))
            if best is None or score < best[0]:
                best = (score, a, cut)
        _, a, cut = best
        axis[node] = a
        plane[node] = cut
        low = idx[p[idx, a] < cut]
        high = idx[p[idx, a] >= cut]
        lo_h = list(lo)
        hi_l = list(hi)
        hi_l[a] = float(cut)
        lo_h[a] = float(cut)
        split(2 * node + 1, low, lo, hi_l, depth + 1)
        split(2 * node + 2, high, lo_h, hi, depth + 1)

    split(0, np.arange(p.shape[0]), lo0, hi0, 0)
    return axis, plane


def leaf_bounds(axis, plane, levels: int):
    """lo, hi float64 [K, 3]: the half-open box of every leaf (infinite outside)."""
    K = 1 << levels
    lo = np.full((K, 3), -np.inf)
    hi = np.full((K, 3), np.inf)
    for b in range(K):
        node = b + K - 1
        while node > 0:
            parent = (node - 1) // 2
            a = int(axis[parent])
            if node == 2 * parent + 2:
                lo[b, a] = max(lo[b, a], float(plane[parent]))
            else:
                hi[b, a] = min(hi[b, a], float(plane[parent]))
            node = parent
    return lo, hi


def box_of_point(axis, plane, levels: int, x) -> int:
    """Box holding point x: walk the tree, high side when x[axis] >= plane."""
    node = 0
    for _ in range(levels):
        node = 2 * node + (2 if x[int(axis[node])] >= float(plane[node]) else 1)
    return node - ((1 << levels) - 1)


def ray_box_interval(o, d, lo, hi):
    """[t_in, t_out) of the ray o + t d inside the box [lo, hi) (float64 slab
    test; an axis the ray runs parallel to keeps the ray iff lo <= o < hi).
    Empty boxes give t_in >= t_out."""
    t_in, t_out = -np.inf, np.inf
    for a in range(3):
        oa, da = float(o[a]), float(d[a])
        if da == 0.0:
            if not (lo[a] <= oa < hi[a]):
                return np.inf, -np.inf
            continue
        t1 = (lo[a] - oa) / da
        t2 = (hi[a] - oa) / da
        near = t1 if t1 < t2 else t2
        far = t2 if t1 < t2 else t1
        t_in = near if near > t_in else t_in
        t_out = far if far < t_out else t_out
    return t_in, t_out


def tag_split_pack(origins, dirs, t_start, t_end, ray_offsets, axis, plane, levels: int):
    """Cut, tag and pack ray-major samples into the region-major layout.

    origins, dirs: float32 [R, 3]; t_start, t_end: float32 [N], ray r's samples
    at [ray_offsets[r], ray_offsets[r+1]), sorted and non-overlapping.
    Returns dict of t_start, t_end (float32 [n]), src (int64 [n]: the input
    sample each piece comes from), seg_offsets [n_seg+1], ray_offsets [R+1],
    seg_ids [n_seg] (each ray's segments front to back), seg_box int32 [n_seg]."""
    origins = np.asarray(origins, np.float32).reshape(-1, 3)
    dirs = np.asarray(dirs, np.float32).reshape(-1, 3)
    ts = np.asarray(t_start, np.float32)
    te = np.asarray(t_end, np.float32)
    ro = np.asarray(ray_offsets, np.int64)
    R = origins.shape[0]
    K = 1 << levels
    lo, hi = leaf_bounds(axis, plane, levels)
    # pieces[b][r] = list of (t0, t1, src); ray_boxes[r] = [(t_in, b), ...]
    pieces = [[[] for _ in range(R)] for _ in range(K)]
    ray_boxes = [[] for _ in range(R)]
    for r in range(R):
        for b in range(K):
            t_in64, t_out64 = ray_box_interval(origins[r], dirs[r], lo[b], hi[b])
            t_in = np.float32(t_in64)
            t_out = np.float32(t_out64)
            got = []
            for i in range(ro[r], ro[r + 1]):
                s, e = ts[i], te[i]
                if s < e:
                    a0 = s if s > t_in else t_in
                    a1 = e if e < t_out else t_out
                    if a0 < a1:
                        got.append((a0, a1, i))
                elif s == e and t_in <= s < t_out:
                    got.append((s, e, i))
            if got:
                pieces[b][r] = got
                ray_boxes[r].append((t_in, b))
    t0, t1, src, seg_len, seg_box, seg_ray = [], [], [], [], [], []
    seg_id = {}
    for b in range(K):
        for r in range(R):
            if pieces[b][r]:
                seg_id[(b, r)] = len(seg_len)
                seg_len.append(len(pieces[b][r]))
                seg_box.append(b)
                seg_ray.append(r)
                for a0, a1, i in pieces[b][r]:
                    t0.append(a0)
                    t1.append(a1)
                    src.append(i)
    seg_offsets = np.zeros(len(seg_len) + 1, dtype=np.int64)
    np.cumsum(np.asarray(seg_len, dtype=np.int64), out=seg_offsets[1:])
    out_ray_offsets = np.zeros(R + 1, dtype=np.int64)
    seg_ids = []
    for r in range(R):
        front_to_back = sorted(ray_boxes[r])
        seg_ids.extend(seg_id[(b, r)] for _, b in front_to_back)
        out_ray_offsets[r + 1] = len(seg_ids)
    return dict(t_start=np.asarray(t0, np.float32), t_end=np.asarray(t1, np.float32),
                src=np.asarray(src, np.int64), seg_offsets=seg_offsets,
                ray_offsets=out_ray_offsets, seg_ids=np.asarray(seg_ids, np.int64),
                seg_box=np.asarray(seg_box, np.int32), seg_ray=np.asarray(seg_ray, np.int64))
