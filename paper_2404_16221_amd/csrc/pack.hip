// Sample distribution to regions (Sec. 4.2): every ray's samples are cut at
// the points where the ray crosses a box face, so that no interval reaches
// across a box boundary, each piece is tagged with its box, and the pieces are
// packed region-major -- the input layout of the per-region composite.
//
// Boxes are the leaves of the partition tree (partition.cpp): heap-ordered
// nodes with an axis and a plane each, box b = leaf node b + K - 1, K =
// 2^levels <= 64, outermost boxes unbounded.  Box b's parameter interval on a
// ray is the slab intersection [t_in, t_out), each face parameter (face -
// origin) / direction computed in float64 and the ends rounded to float32; the
// piece of sample [s, e) in box b is [max(s, t_in), min(e, t_out)) when it has
// positive length, and a zero-length sample stays whole in the box whose
// interval holds s.  Boxes sharing a face get the same rounded parameter, so
// the pieces of a sample tile it exactly.
//
// Passes:
//   pack_count  a wave examines 256 (ray, box) pairs: the box's interval on
//               the ray; pairs that can meet the ray's samples are compacted
//               and searched 64 at a time (two binary searches over the ray's
//               sorted samples give the run of samples that meet the box) ->
//               run length and first sample, ray-major at [r][b], and the
//               ray's segment count;
//   block sums  pieces and segments of every box in every block of 16 rays,
//               box-major at [b][block], so that an exclusive scan gives each
//               (box, block) its first slot and first segment id in
//               region-major order, and (up to 16 boxes), ray-major, each (ray,
//               box)'s pieces and segments in the earlier rays of its block; a
//               scan of the segments per ray gives the per-ray lists;
//   pack_fill   up to 16 boxes one wave per ray: lanes take their box's
//               slot and segment id from those two prefixes; above 16 boxes
//               one wave per block of 16 rays taken in order, lanes carrying
//               their box's running slot and segment id.  Lanes rank the
//               ray's boxes front to back through LDS and write the segment
//               lists; then the wave strides over the ray's samples and writes
//               every piece to its slot (consecutive samples of one box go to
//               consecutive slots).
// The workspace is 16 bytes per ray and box (8 above 16 boxes) plus 32 per
// box and block of rays.
// A ray's run in one box is capped at 2^31 / 16 samples (int32 prefixes).
// Every store index is bounded by the counts of the plan, so inputs that break
// the sortedness contract give unspecified pieces but never out-of-range
// stores.
#include <hip/hip_runtime.h>

#include <cmath>

#include "../../include/xl.h"
#include "internal.h"
#include "xl_device.hpp"

namespace xl {
namespace {

constexpr int kPackWaves = 4;
constexpr int kPackBlock = kPackWaves * kWave;
constexpr int kRayBlock = 16;  // rays per block of the region-major slot prefix
constexpr int kPairs = 256;     // (ray, box) pairs a count wave examines
constexpr int64_t kMaxRun = INT32_MAX / kRayBlock;  // samples of one ray in one box
// Up to this many boxes the fill takes one wave per ray (the block sums then
// also write in-block prefixes); above it one wave per block of rays, whose
// per-ray set-up is shared by fewer lanes' worth of samples.
constexpr int kRayFillMaxK = 16;

struct PackDev {
  const float* o;        // [R][3]
  const float* d;        // [R][3]
  const float* t0;       // samples, ray-major
  const float* t1;
  const int64_t* ray_off;  // [R + 1] samples of each ray
  const int32_t* axis;   // [K - 1]
  const float* plane;    // [K - 1]
  int64_t R, nblk;
  int32_t levels, K;
};

struct PackWs {
  int32_t* cnt;      // [R][K] pieces of ray r in box b
  int32_t* first;    // [R][K] first sample of that run (index inside the ray)
  int32_t* pre;      // [R][K] pieces of box b in the earlier rays of r's block
  int32_t* presg;    // [R][K] segments of box b in the earlier rays of r's block
  int64_t* bsum;     // [K][nblk] pieces of box b in block blk
  int64_t* bseg;     // [K][nblk] rays of block blk with pieces in box b
  int64_t* bpre;     // [K * nblk + 1] first slot of (b, blk)
  int64_t* bsegpre;  // [K * nblk + 1] first segment id of (b, blk)
  int64_t* nseg;     // [R] segments of each ray
  int64_t* ray_off;  // [R + 1] first entry of each ray in seg_ids
  int64_t* scan_tmp;
};

struct Box {
  float lo[3], hi[3];
};

// Leaf b of the tree as the intersection of the half-spaces on its path.
__device__ Box leaf_box(const PackDev& p, int b) {
  Box bx;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    bx.lo[c] = -INFINITY;
    bx.hi[c] = INFINITY;
  }
  int node = b + p.K - 1;
  for (int l = 0; l < p.levels; ++l) {
    const int parent = (node - 1) >> 1;
    const int a = p.axis[parent];
    const float pl = p.plane[parent];
    const bool high = node == 2 * parent + 2;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (a != c) continue;
      if (high) bx.lo[c] = pl > bx.lo[c] ? pl : bx.lo[c];
      else bx.hi[c] = pl < bx.hi[c] ? pl : bx.hi[c];
    }
    node = parent;
  }
  return bx;
}

// The box's parameter interval [t_in, t_out) on ray r: float64 slab test,
// ends rounded to float32; an empty box gives (inf, -inf).
__device__ float2 ray_span(const PackDev& p, int64_t r, const Box& bx) {
  double tin = -INFINITY, tout = INFINITY;
  bool empty = false;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double oc = static_cast<double>(p.o[3 * r + c]);
    const double dc = static_cast<double>(p.d[3 * r + c]);
    const double l = static_cast<double>(bx.lo[c]), h = static_cast<double>(bx.hi[c]);
    if (dc == 0.0) {
      empty |= !(l <= oc && oc < h);
    } else {
      const double ta = (l - oc) / dc, tb = (h - oc) / dc;
      const double near = ta < tb ? ta : tb, far = ta < tb ? tb : ta;
      tin = near > tin ? near : tin;
      tout = far < tout ? far : tout;
    }
  }
  return empty ? make_float2(INFINITY, -INFINITY)
               : make_float2(static_cast<float>(tin), static_cast<float>(tout));
}

// Samples [first, first + count) of the ray (s0, n) that meet [tin, tout).
// Probe of a search over [a, c) (c > a) for a key at `key`, with v_lo and
// v_hi bounds of the keys at a and at c - 1: the interpolated position for
// the first kInterp probes (positions along a ray are close to evenly
// spread), the midpoint after that.  Always inside [a, c - 1], so every
// probe shrinks the range and the search ends within kInterp + log2(n) + 1.
constexpr int kInterp = 6;
__device__ __forceinline__ int64_t probe(int64_t a, int64_t c, float v_lo, float v_hi, float key, int it) {
  if (it < kInterp) {
    float g = (key - v_lo) / (v_hi - v_lo) * static_cast<float>(c - a);
    if (!(g >= 0.f)) g = 0.f;  // also NaN (equal bounds)
    const float top = static_cast<float>(c - a - 1);
    if (g > top) g = top;
    return a + static_cast<int64_t>(g);
  }
  return (a + c) >> 1;
}

__device__ void run_of(const PackDev& p, float tin, float tout, int64_t s0, int64_t n,
                       int64_t& first, int64_t& count) {
  first = 0;
  count = 0;
  if (!(tin < tout) || n <= 0) return;
  // first sample reaching into the box: it ends after t_in, or has zero
  // length at t_in
  int64_t a = 0, c = n;
  float v_lo = p.t0[s0], v_hi = p.t1[s0 + n - 1];
  for (int it = 0; a < c; ++it) {
    const int64_t m = probe(a, c, v_lo, v_hi, tin, it);
    const float e = p.t1[s0 + m];
    const bool in = e > tin || (e == tin && p.t0[s0 + m] == tin);
    if (in) {
      c = m;
      v_hi = e;
    } else {
      a = m + 1;
      v_lo = e;
    }
  }
  first = a;
  // first sample starting at or after t_out
  c = n;
  v_lo = tin;
  v_hi = p.t1[s0 + n - 1];
  for (int it = 0; a < c; ++it) {
    const int64_t m = probe(a, c, v_lo, v_hi, tout, it);
    const float s = p.t0[s0 + m];
    if (s >= tout) {
      c = m;
      v_hi = s;
    } else {
      a = m + 1;
      v_lo = s;
    }
  }
  count = a - first;
}

// A wave examines kPairs (ray, box) pairs: kPairs / K consecutive rays.
// Pairs whose box interval cannot meet the ray's samples (empty, or outside
// [first start, last end]) get a zero count at once; the others are compacted
// into LDS and searched 64 at a time, so one chain of dependent loads serves
// many rays.  Counts and first samples are written ray-major at r * K + b.
__global__ __launch_bounds__(kPackBlock) void pack_count_kernel(PackDev p, PackWs w) {
  __shared__ float c_tin[kPackWaves][kPairs], c_tout[kPackWaves][kPairs];
  __shared__ int32_t c_pair[kPackWaves][kPairs], c_nseg[kPackWaves][kPairs];
  __shared__ Box boxes[kWave];  // the K leaf boxes, built once per block
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  if (threadIdx.x < p.K) boxes[threadIdx.x] = leaf_box(p, threadIdx.x);
  __syncthreads();
  const int rays = kPairs / p.K;
  const int64_t r0 = (static_cast<int64_t>(blockIdx.x) * kPackWaves + wave) * rays;
  for (int i = lane; i < rays; i += kWave) c_nseg[wave][i] = 0;
  const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
  int ncand = 0;
  for (int i0 = 0; i0 < kPairs; i0 += kWave) {
    const int i = i0 + lane;
    const int64_t r = r0 + i / p.K;
    const int b = i % p.K;
    bool cand = false;
    float2 sp = make_float2(INFINITY, -INFINITY);
    if (r < p.R) {
      const int64_t s0 = p.ray_off[r], s1 = p.ray_off[r + 1];
      sp = ray_span(p, r, boxes[b]);
      if (s1 > s0 && sp.x < sp.y) {
        // a piece needs t_in <= some sample's end and t_out > some start
        cand = sp.x <= p.t1[s1 - 1] && sp.y > p.t0[s0];
      }
      if (!cand) {
        w.cnt[r * p.K + b] = 0;
        w.first[r * p.K + b] = 0;
      }
    }
    const unsigned long long m = __ballot(cand);
    if (cand) {
      const int at = ncand + __popcll(m & below);
      c_tin[wave][at] = sp.x;
      c_tout[wave][at] = sp.y;
      c_pair[wave][at] = i;
    }
    ncand += __popcll(m);
  }
  __atomic_signal_fence(__ATOMIC_SEQ_CST);  // (a wave's LDS operations run in order)
  for (int j0 = 0; j0 < ncand; j0 += kWave) {
    const int j = j0 + lane;
    if (j < ncand) {
      const int i = c_pair[wave][j];
      const int64_t r = r0 + i / p.K;
      const int b = i % p.K;
      const int64_t s0 = p.ray_off[r], n = p.ray_off[r + 1] - s0;
      int64_t first, count;
      run_of(p, c_tin[wave][j], c_tout[wave][j], s0, n, first, count);
      // int32 storage with room for a block's sum; all passes use this value
      count = count < kMaxRun ? count : kMaxRun;
      w.cnt[r * p.K + b] = static_cast<int32_t>(count);
      w.first[r * p.K + b] = static_cast<int32_t>(first);
      if (count > 0) atomicAdd(&c_nseg[wave][i / p.K], 1);
    }
  }
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  for (int i = lane; i < rays; i += kWave)
    if (r0 + i < p.R) w.nseg[r0 + i] = c_nseg[wave][i];
}

// Pieces and segments of box b in block blk, one thread per (blk, b).
__global__ void pack_block_sum_kernel(PackDev p, PackWs w) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= p.K * p.nblk) return;
  const int64_t blk = t / p.K;
  const int b = static_cast<int>(t % p.K);
  int64_t pieces = 0, segs = 0;
  for (int j = 0; j < kRayBlock; ++j) {
    const int64_t r = blk * kRayBlock + j;
    if (r >= p.R) break;
    const int32_t c = w.cnt[r * p.K + b];
    if (p.K <= kRayFillMaxK) {
      w.pre[r * p.K + b] = static_cast<int32_t>(pieces);
      w.presg[r * p.K + b] = static_cast<int32_t>(segs);
    }
    pieces += c > 0 ? c : 0;
    segs += c > 0 ? 1 : 0;
  }
  w.bsum[b * p.nblk + blk] = pieces;
  w.bseg[b * p.nblk + blk] = segs;
}

// Small K: one wave per ray.
__global__ __launch_bounds__(kPackBlock) void pack_fill_ray_kernel(PackDev p, PackWs w,
                                                               float* __restrict__ out_t0,
                                                               float* __restrict__ out_t1,
                                                               int64_t* __restrict__ out_src,
                                                               int64_t* __restrict__ seg_offsets,
                                                               int64_t* __restrict__ seg_ids,
                                                               int32_t* __restrict__ seg_box) {
  __shared__ float s_tin[kPackWaves][kWave], s_tout[kPackWaves][kWave];
  __shared__ int32_t s_first[kPackWaves][kWave], s_cnt[kPackWaves][kWave];
  __shared__ int64_t s_base[kPackWaves][kWave];
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int64_t r = static_cast<int64_t>(blockIdx.x) * kPackWaves + wave;
  const bool live = r < p.R;
  int64_t s0 = 0, n = 0;
  if (live) {
    s0 = p.ray_off[r];
    n = p.ray_off[r + 1] - s0;
  }
  // this lane's box: its run on the ray, and its slot and segment id in
  // region-major order ((box, block) start plus the block's earlier rays)
  int32_t c = 0, f = 0;
  int64_t slot = 0, sid = 0;
  if (live && lane < p.K) {
    const int64_t blk = r / kRayBlock, at = r * p.K + lane;
    c = w.cnt[at];
    f = w.first[at];
    slot = w.bpre[lane * p.nblk + blk] + w.pre[at];
    sid = w.bsegpre[lane * p.nblk + blk] + w.presg[at];
  }
  const bool valid = c > 0;
  float tin = INFINITY, tout = -INFINITY;
  if (valid) {
    const float2 sp = ray_span(p, r, leaf_box(p, lane));
    tin = sp.x;
    tout = sp.y;
  }
  s_tin[wave][lane] = valid ? tin : INFINITY;
  __syncthreads();
  // front-to-back rank among the boxes with pieces (ties, which disjoint
  // boxes cannot produce, broken by lane so that ranks stay distinct)
  int rank = 0;
  if (valid)
    for (int k = 0; k < p.K; ++k) {
      const float t = s_tin[wave][k];
      rank += (t < tin || (t == tin && k < lane)) ? 1 : 0;
    }
  const int nv = __popcll(__ballot(valid));
  __syncthreads();
  if (valid) {
    s_tin[wave][rank] = tin;
    s_tout[wave][rank] = tout;
    s_first[wave][rank] = f;
    s_cnt[wave][rank] = c;
    s_base[wave][rank] = slot;
    seg_offsets[sid] = slot;
    if (seg_box) seg_box[sid] = lane;
    seg_ids[w.ray_off[r] + rank] = sid;
  }
  __syncthreads();
  if (!live) return;
  int k0 = 0;
  // the next chunk's interval is loaded before this chunk's pieces are stored
  float s_next = 0.f, e_next = 0.f;
  if (lane < n) {
    s_next = p.t0[s0 + lane];
    e_next = p.t1[s0 + lane];
  }
  for (int64_t j = lane; j < n; j += kWave) {
    const float s = s_next, e = e_next;
    if (j + kWave < n) {
      s_next = p.t0[s0 + j + kWave];
      e_next = p.t1[s0 + j + kWave];
    }
    while (k0 < nv && !(s_tout[wave][k0] > s)) ++k0;  // samples ascend: k0 only grows
    for (int k = k0; k < nv; ++k) {
      const float ti = s_tin[wave][k], to = s_tout[wave][k];
      const bool pos = s < e;
      if (pos && !(ti < e)) break;
      float a0, a1;
      bool piece;
      if (pos) {
        a0 = s > ti ? s : ti;
        a1 = e < to ? e : to;
        piece = a0 < a1;
      } else {
        a0 = a1 = s;
        piece = ti <= s && s < to;
      }
      if (piece) {
        const int64_t q = j - s_first[wave][k];
        if (q >= 0 && q < s_cnt[wave][k]) {
          const int64_t at = s_base[wave][k] + q;
          out_t0[at] = a0;
          out_t1[at] = a1;
          if (out_src) out_src[at] = s0 + j;
        }
      }
      if (!pos) break;  // a zero-length sample has one piece
    }
  }
}

// Large K: one wave per block of 16 rays, taken in order; lanes carry their
// box's running slot and segment id from ray to ray.  Held to 64 registers
// so that eight waves share each SIMD (74 unconstrained, six waves; the fill
// waits on memory more than it computes: measured at K=64, 11.47 -> 11.16 ms
// with the source index, 9.17 -> 7.93 ms without).
__global__ __launch_bounds__(kPackBlock) __attribute__((amdgpu_waves_per_eu(8))) void pack_fill_block_kernel(PackDev p, PackWs w,
                                                               float* __restrict__ out_t0,
                                                               float* __restrict__ out_t1,
                                                               int64_t* __restrict__ out_src,
                                                               int64_t* __restrict__ seg_offsets,
                                                               int64_t* __restrict__ seg_ids,
                                                               int32_t* __restrict__ seg_box) {
  // Each wave uses its own rows, and a wave's LDS operations execute in
  // order, so between the steps only the compiler is held back (a signal
  // fence emits no instruction and no wait on the pieces' stores).
  __shared__ float s_key[kPackWaves][kWave], s_tout[kPackWaves][kWave];
  __shared__ int32_t s_first[kPackWaves][kWave], s_cnt[kPackWaves][kWave];
  __shared__ int64_t s_base[kPackWaves][kWave];
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int64_t blk = static_cast<int64_t>(blockIdx.x) * kPackWaves + wave;
  if (blk >= p.nblk) return;
  // this lane's box, and its running slot and segment id in region-major order
  Box bx;
  int64_t slot = 0, sid = 0;
  if (lane < p.K) {
    bx = leaf_box(p, lane);
    slot = w.bpre[lane * p.nblk + blk];
    sid = w.bsegpre[lane * p.nblk + blk];
  }
  const int64_t r_end = (blk + 1) * kRayBlock < p.R ? (blk + 1) * kRayBlock : p.R;
  const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
  // the first ray's table entries; each ray requests the next ray's before
  // it works on its own samples
  int32_t c_next = 0, f_next = 0;
  if (lane < p.K && blk * kRayBlock < r_end) {
    c_next = w.cnt[blk * kRayBlock * p.K + lane];
    f_next = w.first[blk * kRayBlock * p.K + lane];
  }
  for (int64_t r = blk * kRayBlock; r < r_end; ++r) {
    const int64_t s0 = p.ray_off[r], n = p.ray_off[r + 1] - s0;
    const int32_t c = c_next, f = f_next;
    if (lane < p.K && r + 1 < r_end) {
      c_next = w.cnt[(r + 1) * p.K + lane];
      f_next = w.first[(r + 1) * p.K + lane];
    }
    float tin = INFINITY, tout = -INFINITY;
    if (lane < p.K && c > 0) {
      const float2 sp = ray_span(p, r, bx);
      tin = sp.x;
      tout = sp.y;
    }
    const bool valid = c > 0;
    // front-to-back rank among the boxes with pieces: the few such boxes are
    // compacted first (ties, which disjoint boxes cannot produce, broken by
    // compacted position so that ranks stay distinct)
    const unsigned long long vm = __ballot(valid);
    const int nv = __popcll(vm);
    const int pos = __popcll(vm & below);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);  // the previous ray's table reads come first
    if (valid) s_key[wave][pos] = tin;
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    int rank = 0;
    if (valid)
      for (int k = 0; k < nv; ++k) {
        const float t = s_key[wave][k];
        rank += (t < tin || (t == tin && k < pos)) ? 1 : 0;
      }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    if (valid) {
      s_key[wave][rank] = tin;
      s_tout[wave][rank] = tout;
      s_first[wave][rank] = f;
      s_cnt[wave][rank] = c;
      s_base[wave][rank] = slot;
      seg_offsets[sid] = slot;
      if (seg_box) seg_box[sid] = lane;
      seg_ids[w.ray_off[r] + rank] = sid;
    }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    if (valid) {
      slot += c;
      sid += 1;
    }
    int k0 = 0;
    // the next chunk's interval is loaded before this chunk's pieces are stored
    float s_next = 0.f, e_next = 0.f;
    if (lane < n) {
      s_next = p.t0[s0 + lane];
      e_next = p.t1[s0 + lane];
    }
    for (int64_t j = lane; j < n; j += kWave) {
      const float s = s_next, e = e_next;
      if (j + kWave < n) {
        s_next = p.t0[s0 + j + kWave];
        e_next = p.t1[s0 + j + kWave];
      }
      while (k0 < nv && !(s_tout[wave][k0] > s)) ++k0;  // samples ascend: k0 only grows
      for (int k = k0; k < nv; ++k) {
        const float ti = s_key[wave][k], to = s_tout[wave][k];
        const bool pos = s < e;
        if (pos && !(ti < e)) break;
        float a0, a1;
        bool piece;
        if (pos) {
          a0 = s > ti ? s : ti;
          a1 = e < to ? e : to;
          piece = a0 < a1;
        } else {
          a0 = a1 = s;
          piece = ti <= s && s < to;
        }
        if (piece) {
          const int64_t q = j - s_first[wave][k];
          if (q >= 0 && q < s_cnt[wave][k]) {
            const int64_t at = s_base[wave][k] + q;
            out_t0[at] = a0;
            out_t1[at] = a1;
            if (out_src) out_src[at] = s0 + j;
          }
        }
        if (!pos) break;  // a zero-length sample has one piece
      }
    }
  }
}

struct PackLayout {
  int64_t R, K, RK, nblk, KB;
  size_t scan_elems;
  size_t off[11];
  size_t bytes;
};

PackLayout pack_layout(int64_t R, int levels) {
  PackLayout L;
  L.R = R;
  L.K = int64_t{1} << levels;
  L.RK = L.K * R;
  L.nblk = (R + kRayBlock - 1) / kRayBlock;
  L.KB = L.K * L.nblk;
  L.scan_elems = scan_tmp_elems(L.KB > R ? L.KB : R);
  const size_t sizes[] = {
      sizeof(int32_t) * L.RK,           // cnt
      sizeof(int32_t) * L.RK,           // first
      sizeof(int32_t) * (L.K <= kRayFillMaxK ? L.RK : 0),  // pre
      sizeof(int32_t) * (L.K <= kRayFillMaxK ? L.RK : 0),  // presg
      sizeof(int64_t) * L.KB,           // bsum
      sizeof(int64_t) * L.KB,           // bseg
      sizeof(int64_t) * (L.KB + 1),     // bpre
      sizeof(int64_t) * (L.KB + 1),     // bsegpre
      sizeof(int64_t) * R,              // nseg
      sizeof(int64_t) * (R + 1),        // ray_off
      sizeof(int64_t) * L.scan_elems,   // scan_tmp
  };
  size_t o = 0;
  for (int i = 0; i < 11; ++i) {
    L.off[i] = o;
    o += (sizes[i] + 255) & ~static_cast<size_t>(255);
  }
  L.bytes = o;
  return L;
}

PackWs pack_views(const PackLayout& L, void* ws) {
  char* b = static_cast<char*>(ws);
  PackWs w;
  w.cnt = reinterpret_cast<int32_t*>(b + L.off[0]);
  w.first = reinterpret_cast<int32_t*>(b + L.off[1]);
  w.pre = reinterpret_cast<int32_t*>(b + L.off[2]);
  w.presg = reinterpret_cast<int32_t*>(b + L.off[3]);
  w.bsum = reinterpret_cast<int64_t*>(b + L.off[4]);
  w.bseg = reinterpret_cast<int64_t*>(b + L.off[5]);
  w.bpre = reinterpret_cast<int64_t*>(b + L.off[6]);
  w.bsegpre = reinterpret_cast<int64_t*>(b + L.off[7]);
  w.nseg = reinterpret_cast<int64_t*>(b + L.off[8]);
  w.ray_off = reinterpret_cast<int64_t*>(b + L.off[9]);
  w.scan_tmp = reinterpret_cast<int64_t*>(b + L.off[10]);
  return w;
}

PackDev pack_dev(const xl_rays* rays, const int32_t* axis, const float* plane, int levels) {
  PackDev p;
  p.o = rays->origins;
  p.d = rays->dirs;
  p.t0 = rays->t_start;
  p.t1 = rays->t_end;
  p.ray_off = rays->ray_offsets;
  p.axis = axis;
  p.plane = plane;
  p.R = rays->n_rays;
  p.nblk = (p.R + kRayBlock - 1) / kRayBlock;
  p.levels = levels;
  p.K = 1 << levels;
  return p;
}

unsigned grid_for(int64_t items, int64_t per_block) {
  return static_cast<unsigned>((items + per_block - 1) / per_block);
}

}  // namespace

size_t pack_workspace_bytes(int64_t n_rays, int levels) { return pack_layout(n_rays, levels).bytes; }

hipError_t pack_plan(const xl_rays* rays, const int32_t* axis, const float* plane, int levels,
                     void* ws, hipStream_t st, int64_t* n_pieces, int64_t* n_seg) {
  const PackLayout L = pack_layout(rays->n_rays, levels);
  const PackWs w = pack_views(L, ws);
  const PackDev p = pack_dev(rays, axis, plane, levels);
  if (L.R > 0) {
    hipLaunchKernelGGL(pack_count_kernel, dim3(grid_for(L.R, kPackWaves * (kPairs / p.K))),
                       dim3(kPackBlock), 0, st, p, w);
    hipLaunchKernelGGL(pack_block_sum_kernel, dim3(grid_for(L.KB, 256)), dim3(256), 0, st, p, w);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = scan_exclusive(w.bsum, w.bpre, L.KB, w.scan_tmp, L.scan_elems, st)) != hipSuccess) return e;
  if ((e = scan_exclusive(w.bseg, w.bsegpre, L.KB, w.scan_tmp, L.scan_elems, st)) != hipSuccess) return e;
  if ((e = scan_exclusive(w.nseg, w.ray_off, L.R, w.scan_tmp, L.scan_elems, st)) != hipSuccess) return e;
  int64_t h[2] = {0, 0};
  if ((e = hipMemcpyAsync(&h[0], w.bpre + L.KB, sizeof(int64_t), hipMemcpyDeviceToHost, st)) != hipSuccess)
    return e;
  if ((e = hipMemcpyAsync(&h[1], w.bsegpre + L.KB, sizeof(int64_t), hipMemcpyDeviceToHost, st)) != hipSuccess)
    return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  *n_pieces = h[0];
  *n_seg = h[1];
  return hipSuccess;
}

// First segment of every box (the (box, block 0) segment prefix), and n_seg.
__global__ void pack_region_offsets_kernel(const int64_t* __restrict__ bsegpre, int64_t nblk, int K,
                                           int64_t* __restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b <= K) out[b] = bsegpre[b * nblk];
}

hipError_t pack_fill(const xl_rays* rays, const int32_t* axis, const float* plane, int levels,
                     void* ws, int64_t n_seg, float* t_start, float* t_end, int64_t* src,
                     int64_t* seg_offsets, int64_t* ray_offsets, int64_t* seg_ids, int32_t* seg_box,
                     int64_t* region_offsets, hipStream_t st) {
  const PackLayout L = pack_layout(rays->n_rays, levels);
  const PackWs w = pack_views(L, ws);
  const PackDev p = pack_dev(rays, axis, plane, levels);
  if (L.R > 0)
  {
    if (p.K <= kRayFillMaxK)
      hipLaunchKernelGGL(pack_fill_ray_kernel, dim3(grid_for(L.R, kPackWaves)), dim3(kPackBlock), 0, st, p,
                         w, t_start, t_end, src, seg_offsets, seg_ids, seg_box);
    else
      hipLaunchKernelGGL(pack_fill_block_kernel, dim3(grid_for(L.nblk, kPackWaves)), dim3(kPackBlock), 0,
                         st, p, w, t_start, t_end, src, seg_offsets, seg_ids, seg_box);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = hipMemcpyAsync(seg_offsets + n_seg, w.bpre + L.KB, sizeof(int64_t),
                          hipMemcpyDeviceToDevice, st)) != hipSuccess)
    return e;
  if ((e = hipMemcpyAsync(ray_offsets, w.ray_off, sizeof(int64_t) * (L.R + 1),
                          hipMemcpyDeviceToDevice, st)) != hipSuccess)
    return e;
  if (region_offsets) {
    // (with no rays every block prefix is the single total 0 at bsegpre[0])
    const int64_t nblk = L.nblk > 0 ? L.nblk : 0;
    hipLaunchKernelGGL(pack_region_offsets_kernel, dim3(grid_for(L.K + 1, 256)), dim3(256), 0, st,
                       w.bsegpre, nblk, static_cast<int>(L.K), region_offsets);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace xl
