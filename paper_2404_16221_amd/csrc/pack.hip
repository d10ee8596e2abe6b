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
// Three passes:
//   pack_count  one lane per (ray, box), 64 / K rays per wave: the box's
//               interval and, by two binary searches over the ray's sorted
//               samples, the run of samples that meet it -> piece count at
//               [b][r] (box-major, so an exclusive scan gives region-major
//               slots), a 0/1 segment flag, the run's first sample and the
//               interval;
//   scans       pieces and segment flags over [K][R], segments per ray;
//   pack_fill   one wave per ray: lanes load their box's run, rank the boxes
//               front to back through LDS and write the segment lists, then
//               the wave strides over the ray's samples and writes every piece
//               to its slot (consecutive samples of one box go to consecutive
//               slots).
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

struct PackDev {
  const float* o;        // [R][3]
  const float* d;        // [R][3]
  const float* t0;       // samples, ray-major
  const float* t1;
  const int64_t* ray_off;  // [R + 1] samples of each ray
  const int32_t* axis;   // [K - 1]
  const float* plane;    // [K - 1]
  int64_t R;
  int32_t levels, K;
};

struct PackWs {
  int64_t* cnt;      // [K * R] pieces of ray r in box b, at b * R + r
  int64_t* has;      // [K * R] 1 when that count is positive
  int32_t* first;    // [K * R] first sample of the run (index inside the ray)
  float2* span;      // [K * R] the box's interval (t_in, t_out) on the ray
  int64_t* off;      // [K * R + 1] first slot of those pieces
  int64_t* sid;      // [K * R + 1] id of that segment
  int64_t* nseg;     // [R] segments of each ray
  int64_t* ray_off;  // [R + 1] first entry of each ray in seg_ids
  int64_t* scan_tmp;
};

struct BoxSpan {
  float tin, tout;
  int64_t first, count;  // samples [first, first + count) of the ray meet the box
};

__device__ BoxSpan box_span(const PackDev& p, int64_t r, int b, int64_t s0, int64_t n) {
  float lo[3] = {-INFINITY, -INFINITY, -INFINITY}, hi[3] = {INFINITY, INFINITY, INFINITY};
  int node = b + p.K - 1;
  for (int l = 0; l < p.levels; ++l) {
    const int parent = (node - 1) >> 1;
    const int a = p.axis[parent];
    const float pl = p.plane[parent];
    const bool high = node == 2 * parent + 2;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (a != c) continue;
      if (high) lo[c] = pl > lo[c] ? pl : lo[c];
      else hi[c] = pl < hi[c] ? pl : hi[c];
    }
    node = parent;
  }
  double tin = -INFINITY, tout = INFINITY;
  bool empty = false;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double oc = static_cast<double>(p.o[3 * r + c]);
    const double dc = static_cast<double>(p.d[3 * r + c]);
    const double l = static_cast<double>(lo[c]), h = static_cast<double>(hi[c]);
    if (dc == 0.0) {
      empty |= !(l <= oc && oc < h);
    } else {
      const double ta = (l - oc) / dc, tb = (h - oc) / dc;
      const double near = ta < tb ? ta : tb, far = ta < tb ? tb : ta;
      tin = near > tin ? near : tin;
      tout = far < tout ? far : tout;
    }
  }
  BoxSpan sp;
  sp.tin = empty ? INFINITY : static_cast<float>(tin);
  sp.tout = empty ? -INFINITY : static_cast<float>(tout);
  sp.first = 0;
  sp.count = 0;
  if (!(sp.tin < sp.tout) || n <= 0) return sp;
  // first sample reaching into the box: it ends after t_in, or has zero
  // length at t_in
  int64_t a = 0, c = n;
  while (a < c) {
    const int64_t m = (a + c) >> 1;
    const float e = p.t1[s0 + m];
    const bool in = e > sp.tin || (e == sp.tin && p.t0[s0 + m] == sp.tin);
    if (in) c = m;
    else a = m + 1;
  }
  sp.first = a;
  // first sample starting at or after t_out
  c = n;
  while (a < c) {
    const int64_t m = (a + c) >> 1;
    if (p.t0[s0 + m] >= sp.tout) c = m;
    else a = m + 1;
  }
  sp.count = a - sp.first;
  return sp;
}

// 64 / K rays per wave, K consecutive lanes per ray (K divides 64).
__global__ __launch_bounds__(kPackBlock) void pack_count_kernel(PackDev p, PackWs w) {
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int per_wave = kWave / p.K;
  const int sub = lane / p.K, b = lane % p.K;
  const int64_t r = (static_cast<int64_t>(blockIdx.x) * kPackWaves + wave) * per_wave + sub;
  const bool live = r < p.R;
  int64_t cnt = 0;
  if (live) {
    const int64_t s0 = p.ray_off[r], n = p.ray_off[r + 1] - s0;
    const BoxSpan sp = box_span(p, r, b, s0, n);
    cnt = sp.count;
    const int64_t at = static_cast<int64_t>(b) * p.R + r;
    w.cnt[at] = cnt;
    w.has[at] = cnt > 0 ? 1 : 0;
    w.first[at] = static_cast<int32_t>(sp.first);
    w.span[at] = make_float2(sp.tin, sp.tout);
  }
  const unsigned long long m = __ballot(cnt > 0);
  const unsigned long long group = p.K == kWave ? ~0ull : (((1ull << p.K) - 1) << (sub * p.K));
  if (live && b == 0) w.nseg[r] = __popcll(m & group);
}

__global__ __launch_bounds__(kPackBlock) void pack_fill_kernel(PackDev p, PackWs w,
                                                               float* __restrict__ out_t0,
                                                               float* __restrict__ out_t1,
                                                               int64_t* __restrict__ out_src,
                                                               int64_t* __restrict__ seg_offsets,
                                                               int64_t* __restrict__ seg_ids,
                                                               int32_t* __restrict__ seg_box) {
  __shared__ float s_tin[kPackWaves][kWave], s_tout[kPackWaves][kWave];
  __shared__ int64_t s_first[kPackWaves][kWave], s_cnt[kPackWaves][kWave], s_base[kPackWaves][kWave];
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int64_t r = static_cast<int64_t>(blockIdx.x) * kPackWaves + wave;
  const bool live = r < p.R;
  int64_t s0 = 0, n = 0;
  if (live) {
    s0 = p.ray_off[r];
    n = p.ray_off[r + 1] - s0;
  }
  // this lane's box: the run and interval that the count pass found
  BoxSpan sp;
  sp.tin = INFINITY;
  sp.tout = -INFINITY;
  sp.first = sp.count = 0;
  const int64_t at = static_cast<int64_t>(lane) * p.R + r;
  if (live && lane < p.K) {
    sp.count = w.cnt[at];
    if (sp.count > 0) {
      const float2 ts = w.span[at];
      sp.tin = ts.x;
      sp.tout = ts.y;
      sp.first = w.first[at];
    }
  }
  const bool valid = sp.count > 0;
  s_tin[wave][lane] = valid ? sp.tin : INFINITY;
  __syncthreads();
  // front-to-back rank among the boxes with pieces (their t_in differ: the
  // intervals of disjoint boxes on one ray do not overlap)
  int rank = 0;
  if (valid)
    for (int k = 0; k < p.K; ++k) rank += s_tin[wave][k] < sp.tin ? 1 : 0;
  const int nv = __popcll(__ballot(valid));
  __syncthreads();
  s_cnt[wave][lane] = 0;  // entries no box fills take no pieces
  __syncthreads();
  if (valid) {
    const int64_t base = w.off[at], id = w.sid[at];
    s_tin[wave][rank] = sp.tin;
    s_tout[wave][rank] = sp.tout;
    s_first[wave][rank] = sp.first;
    s_cnt[wave][rank] = sp.count;
    s_base[wave][rank] = base;
    seg_offsets[id] = base;
    if (seg_box) seg_box[id] = lane;
    seg_ids[w.ray_off[r] + rank] = id;
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
      const float tin = s_tin[wave][k], tout = s_tout[wave][k];
      const bool pos = s < e;
      if (pos && !(tin < e)) break;
      float a0, a1;
      bool piece;
      if (pos) {
        a0 = s > tin ? s : tin;
        a1 = e < tout ? e : tout;
        piece = a0 < a1;
      } else {
        a0 = a1 = s;
        piece = tin <= s && s < tout;
      }
      if (piece) {
        const int64_t q = j - s_first[wave][k];
        if (q >= 0 && q < s_cnt[wave][k]) {
          const int64_t slot = s_base[wave][k] + q;
          out_t0[slot] = a0;
          out_t1[slot] = a1;
          if (out_src) out_src[slot] = s0 + j;
        }
      }
      if (!pos) break;  // a zero-length sample has one piece
    }
  }
}

struct PackLayout {
  int64_t R, K, KR;
  size_t scan_elems;
  size_t off[9];
  size_t bytes;
};

PackLayout pack_layout(int64_t R, int levels) {
  PackLayout L;
  L.R = R;
  L.K = int64_t{1} << levels;
  L.KR = L.K * R;
  L.scan_elems = scan_tmp_elems(L.KR > R ? L.KR : R);
  const size_t sizes[] = {
      sizeof(int64_t) * L.KR,           // cnt
      sizeof(int64_t) * L.KR,           // has
      sizeof(int32_t) * L.KR,           // first
      sizeof(float2) * L.KR,            // span
      sizeof(int64_t) * (L.KR + 1),     // off
      sizeof(int64_t) * (L.KR + 1),     // sid
      sizeof(int64_t) * R,              // nseg
      sizeof(int64_t) * (R + 1),        // ray_off
      sizeof(int64_t) * L.scan_elems,   // scan_tmp
  };
  size_t o = 0;
  for (int i = 0; i < 9; ++i) {
    L.off[i] = o;
    o += (sizes[i] + 255) & ~static_cast<size_t>(255);
  }
  L.bytes = o;
  return L;
}

PackWs pack_views(const PackLayout& L, void* ws) {
  char* b = static_cast<char*>(ws);
  PackWs w;
  w.cnt = reinterpret_cast<int64_t*>(b + L.off[0]);
  w.has = reinterpret_cast<int64_t*>(b + L.off[1]);
  w.first = reinterpret_cast<int32_t*>(b + L.off[2]);
  w.span = reinterpret_cast<float2*>(b + L.off[3]);
  w.off = reinterpret_cast<int64_t*>(b + L.off[4]);
  w.sid = reinterpret_cast<int64_t*>(b + L.off[5]);
  w.nseg = reinterpret_cast<int64_t*>(b + L.off[6]);
  w.ray_off = reinterpret_cast<int64_t*>(b + L.off[7]);
  w.scan_tmp = reinterpret_cast<int64_t*>(b + L.off[8]);
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
  p.levels = levels;
  p.K = 1 << levels;
  return p;
}

unsigned ray_blocks(int64_t R, int per_wave = 1) {
  const int64_t per_block = static_cast<int64_t>(kPackWaves) * per_wave;
  return static_cast<unsigned>((R + per_block - 1) / per_block);
}

}  // namespace

size_t pack_workspace_bytes(int64_t n_rays, int levels) { return pack_layout(n_rays, levels).bytes; }

hipError_t pack_plan(const xl_rays* rays, const int32_t* axis, const float* plane, int levels,
                     void* ws, hipStream_t st, int64_t* n_pieces, int64_t* n_seg) {
  const PackLayout L = pack_layout(rays->n_rays, levels);
  const PackWs w = pack_views(L, ws);
  const PackDev p = pack_dev(rays, axis, plane, levels);
  if (L.R > 0)
    hipLaunchKernelGGL(pack_count_kernel, dim3(ray_blocks(L.R, kWave / p.K)), dim3(kPackBlock), 0, st,
                       p, w);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = scan_exclusive(w.cnt, w.off, L.KR, w.scan_tmp, L.scan_elems, st)) != hipSuccess) return e;
  if ((e = scan_exclusive(w.has, w.sid, L.KR, w.scan_tmp, L.scan_elems, st)) != hipSuccess) return e;
  if ((e = scan_exclusive(w.nseg, w.ray_off, L.R, w.scan_tmp, L.scan_elems, st)) != hipSuccess) return e;
  int64_t h[2] = {0, 0};
  if ((e = hipMemcpyAsync(&h[0], w.off + L.KR, sizeof(int64_t), hipMemcpyDeviceToHost, st)) != hipSuccess)
    return e;
  if ((e = hipMemcpyAsync(&h[1], w.sid + L.KR, sizeof(int64_t), hipMemcpyDeviceToHost, st)) != hipSuccess)
    return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  *n_pieces = h[0];
  *n_seg = h[1];
  return hipSuccess;
}

hipError_t pack_fill(const xl_rays* rays, const int32_t* axis, const float* plane, int levels,
                     void* ws, int64_t n_seg, float* t_start, float* t_end, int64_t* src,
                     int64_t* seg_offsets, int64_t* ray_offsets, int64_t* seg_ids, int32_t* seg_box,
                     hipStream_t st) {
  const PackLayout L = pack_layout(rays->n_rays, levels);
  const PackWs w = pack_views(L, ws);
  const PackDev p = pack_dev(rays, axis, plane, levels);
  if (L.R > 0)
    hipLaunchKernelGGL(pack_fill_kernel, dim3(ray_blocks(L.R)), dim3(kPackBlock), 0, st, p, w,
                       t_start, t_end, src, seg_offsets, seg_ids, seg_box);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = hipMemcpyAsync(seg_offsets + n_seg, w.off + L.KR, sizeof(int64_t),
                          hipMemcpyDeviceToDevice, st)) != hipSuccess)
    return e;
  return hipMemcpyAsync(ray_offsets, w.ray_off, sizeof(int64_t) * (L.R + 1), hipMemcpyDeviceToDevice,
                        st);
}

}  // namespace xl
