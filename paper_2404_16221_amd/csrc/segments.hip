// Per-segment composite, forward and backward (Sec. 4.3: each region reduces
// its own samples to per-ray partial tuples before anything is exchanged).
//
// Work decomposition: the packed sample array is cut into fixed tiles of
// kTile = 512 samples, one wavefront per tile and kRun = 8 consecutive samples
// per lane, independent of where segments begin and end.  That keeps every
// load a full, aligned 16-byte vector access and balances ragged segments
// (1..1000+ samples) perfectly.  (16 samples per lane would halve the scan work
// per sample, but the extra registers cost more waves than the scans save.)
// Inside a tile:
//   1. the segment boundaries that fall in the tile are staged in LDS (one
//      entry per sample: local id of the segment ending there, or -1);
//   2. each lane folds its 8 samples serially into ranges (positive form of
//      the merge operator, see xl_device.hpp);
//   3. a segmented wave scan carries the open range across lanes;
//   4. segments that cross a tile boundary are completed by a small fixup
//      kernel from per-tile head/tail ranges; the backward takes a tile's
//      carries (prefix into and suffix out of it) from the neighbouring
//      tile's tail/head range when the segment crosses one boundary, and from
//      the fixup's carry records inside longer chains.
// The backward recomputes transmittance with the same forward scan, takes the
// suffix with a reverse scan, and applies the exact per-sample Jacobian of the
// merge operator, so nothing per sample is stored between the passes.
#include <mutex>

#include "internal.h"
#include "xl_device.hpp"

namespace xl {

int64_t num_tiles(int64_t n) { return (n + kTile - 1) / kTile; }
size_t segments_workspace_bytes(int64_t n) { return TileRecs::bytes(num_tiles(n)); }

// First segment of each tile's window: the segment containing the tile's
// first sample if it starts before the tile, else the first segment (empty
// ones included) starting at the tile's first sample.  One thread per
// segment writes the tiles whose first sample it owns: those starting inside
// it, and the tile starting at its own first sample if no earlier segment
// starts there too.  Every tile gets exactly one writer.
__global__ void plan_kernel(const int64_t* __restrict__ off, int64_t n_seg, int64_t n_tiles,
                            TileRecs recs) {
  const int64_t sg = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (sg >= n_seg) return;
  const int64_t a = off[sg], e = off[sg + 1];
  const bool first_at_a = sg == 0 || off[sg - 1] < a;
  if (first_at_a && a % kTile == 0 && a / kTile < n_tiles) recs.first_seg[a / kTile] = sg;
  for (int64_t t = a / kTile + 1; t * kTile < e && t < n_tiles; ++t) recs.first_seg[t] = sg;
}

__global__ void fill_zero_kernel(float* __restrict__ p, int64_t count) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0.f;
}

__device__ __forceinline__ void write_tuple(float* __restrict__ out, int64_t s, const Range& r,
                                            float tlo = 0.f) {
  store_tup7(out, s, r.tau + tlo, r.cr, r.cg, r.cb, r.A, fmaf(r.A, r.m0, r.F) /* D = sum w m */, r.L);
}
__device__ __forceinline__ void write_tuple(float* __restrict__ out, int64_t s, const Part& p) {
  write_tuple(out, s, p.r, p.tlo);
}

// Stage the segment ends of tile t in LDS and return how many segments the
// tile's window holds (from s_lo on).  endloc[p] = local id (segment -
// s_lo) of the segment whose last sample is base + p, or -1.  Empty segments
// owned by this tile get the identity tuple when WRITE_EMPTY.
constexpr int kStagedSegs = 64;  // segment gradients staged in LDS per tile (backward)
constexpr int kMissing = -2;     // end-table entry of a sample past the array

// Lane samples of tile t that exist (kRun except in the ragged last tile).
__device__ __forceinline__ int lane_count(int64_t n, int64_t t, int lane) {
  const int64_t rem = n - (t * kTile + static_cast<int64_t>(lane) * kRun);
  return rem <= 0 ? 0 : (rem >= kRun ? kRun : static_cast<int>(rem));
}

// The tile's end table starts as -1 (no end) for every sample, and as
// kMissing for the samples past the array in the ragged last tile.
__device__ __forceinline__ void init_ends(int* endloc, int64_t n, int64_t t, int lane) {
  const bool ragged = (t + 1) * kTile > n;  // uniform
#pragma unroll
  for (int j = 0; j < kRun; ++j) endloc[lane + kWave * j] = -1;
  if (ragged) {
#pragma unroll
    for (int j = 0; j < kRun; ++j)
      if (t * kTile + lane + kWave * j >= n) endloc[lane + kWave * j] = kMissing;
  }
}

// The lane's samples of tile t into registers: vector loads, or element
// loads for the ragged last tile.
template <int DT>
__device__ __forceinline__ void load_lane(RawRun<DT>& raw, const SamplesDev& s, int64_t t, int lane) {
  const int64_t i = t * kTile + static_cast<int64_t>(lane) * kRun;
  if ((t + 1) * kTile <= s.n) raw.load(s.sigma, s.rgb, s.t0, s.t1, i);
  else raw.load_part(s.sigma, s.rgb, s.t0, s.t1, i, lane_count(s.n, t, lane));
}

template <bool WRITE_EMPTY>
__device__ __forceinline__ int64_t stage_ends(const int64_t* __restrict__ off, int64_t n_seg,
                                           int64_t n, int64_t t, int64_t n_tiles, int64_t s_lo,
                                           int lane, int* __restrict__ endloc,
                                           float* __restrict__ seg_out,
                                           const float* __restrict__ gseg = nullptr,
                                           float* __restrict__ gl = nullptr) {
  const int64_t base = t * kTile;
  const int64_t tile_end = base + kTile < n ? base + kTile : n;
  const bool last_tile = (t == n_tiles - 1);
  for (int64_t j0 = 0;; j0 += kWave) {
    const int64_t sg = s_lo + j0 + lane;
    bool in = false;
    if (sg < n_seg) {
      const int64_t a = off[sg], e1 = off[sg + 1];
      in = last_tile || a < base + kTile;
      if (in) {
        if (a >= e1) {
          if (WRITE_EMPTY && a >= base) {
            write_tuple(seg_out, sg, range_identity());
          }
        } else {
          const int64_t e = e1 - 1;
          if (e >= base && e < tile_end) {
            const int loc = static_cast<int>(sg - s_lo);
            endloc[e - base] = loc;
            if (gl != nullptr && loc < kStagedSegs) {
              const Tup7 g = load_tup7(gseg, sg);
#pragma unroll
              for (int k = 0; k < 6; ++k) gl[k * kStagedSegs + loc] = g.v[k];
              gl[6 * kStagedSegs + loc] = 2.f * g.v[6];  // the sweep uses 2 g_L
            }
          }
        }
      }
    }
    // Segments are sorted by start: once a lane's segment starts past the tile
    // (or past the last segment), every later one does too.  Returns the number
    // of segments in the tile's window.
    const unsigned long long m = __ballot(in);
    if (m != ~0ull) return j0 + __popcll(m);
  }
}

// Per-lane view of one tile: the lane's kRun samples and the segment ends
// among them.  In the ragged last tile the samples past the array are zeros
// whose end-table entry is kMissing: each acts as a one-sample segment of its
// own that is never written.
// RAGGED: the tile may be the ragged last one, whose missing samples have
// kMissing entries (with RAGGED = false only ids and -1 occur, and the test
// for an end is the cheaper sign test).
template <int DT, bool RAGGED = true>
struct LaneRun {
  Smp x[kRun];
  int ends[kRun];   // local id of the segment ending at sample j, -1, or kMissing
  bool endf[kRun];  // sample j ends a segment (or does not exist)
  bool h0;          // sample 0 starts a segment

  // raw: the lane's samples, already loaded.
  __device__ __forceinline__ void load(const int* endloc, int lane, bool start_head,
                                       const RawRun<DT>* raw) {
#pragma unroll
    for (int j = 0; j < kRun; ++j) ends[j] = endloc[lane * kRun + j];
    h0 = lane == 0 ? start_head : (RAGGED ? endloc[lane * kRun - 1] != -1 : endloc[lane * kRun - 1] >= 0);
    float sg[kRun], c[3 * kRun], a[kRun], b[kRun];
    raw->decode(sg, c, a, b);
#pragma unroll
    for (int j = 0; j < kRun; ++j) {
      x[j] = make_sample(sg[j], c[3 * j], c[3 * j + 1], c[3 * j + 2], a[j], b[j]);
      endf[j] = RAGGED ? ends[j] != -1 : ends[j] >= 0;
    }
  }
  __device__ __forceinline__ bool head(int j) const { return j == 0 ? h0 : endf[j - 1]; }
};

template <int DT>
__device__ __forceinline__ void fwd_tile(const SamplesDev& s, int64_t n_seg, int64_t t,
                                         int64_t s_lo, int64_t n_win, bool start_head, int lane,
                                         int* endloc, float* park,
                                         float* __restrict__ seg_out, const TileRecs& recs,
                                         const RawRun<DT>* raw) {
  LaneRun<DT> R;
  R.load(endloc, lane, start_head, raw);

  // The segment ends are in registers now; their LDS space stages the tuples of
  // segments that end in this tile as kTupStride-word records (slot = local
  // segment id; the last word marks a slot written), which go to seg_out at
  // the end as 16-byte stores of consecutive records.
  static_assert(kTupStride * kStagedSegs <= kTile, "staging must fit the end table");
  // (kept as int so the compiler orders it with the end table's reads)
  int* obuf = endloc;  // [kStagedSegs][kTupStride] float bits
  const bool staged = n_win <= kStagedSegs;  // uniform: no divergence on the path
  if (lane < kStagedSegs) obuf[lane * kTupStride + 7] = 0;
  auto emit = [&](int loc, const Range& r) {
    if (staged) {
      int4* o = reinterpret_cast<int4*>(obuf + loc * kTupStride);
      o[0] = make_int4(__float_as_int(r.tau), __float_as_int(r.cr), __float_as_int(r.cg),
                       __float_as_int(r.cb));
      o[1] = make_int4(__float_as_int(r.A), __float_as_int(fmaf(r.A, r.m0, r.F)), __float_as_int(r.L), 1);
    } else {
      write_tuple(seg_out, s_lo + loc, r);
    }
  };

  // Serial fold of the lane's samples; a head restarts the open range.  The
  // lane's first range, when it continues a segment from an earlier lane, is
  // parked in LDS until the scan has produced what precedes it.
  Range cur = range_identity();
  cur.m0 = R.x[0].m;
  float Tc = 1.f;
  append(cur, Tc, R.x[0]);
  bool cur_head = R.h0, has_pend = false, any_end = false, any_head = R.h0;
  int pend_seg = -1;
#pragma unroll
  for (int j = 0; j < kRun; ++j) {
    if (j > 0) {
      const bool hd = R.head(j);
      restart_if(hd, cur, Tc, R.x[j].m);
      append(cur, Tc, R.x[j]);
      cur_head = cur_head || hd;
      any_head = any_head || hd;
    }
    if (R.endf[j]) {
      any_end = true;
      if (R.ends[j] >= 0) {
        if (cur_head) {
          emit(R.ends[j], cur);
        } else {
          park_range(park, lane, cur);
          pend_seg = R.ends[j];
          has_pend = true;
        }
      }
    }
  }
  const bool have = !R.endf[kRun - 1];

  // Carry the open range across lanes.
  Range inc = have ? cur : range_identity();
  bool fin = have ? cur_head : true;
  scan_up(inc, fin, lane);
  const Range ex = from_lower(inc);
  const int exf = from_lower(static_cast<int>(fin));
  if (has_pend) {
    const Range pend = unpark_range(park, lane);
    if (lane > 0 && exf) {
      emit(pend_seg, combine(ex, pend));
    } else {
      // The tile's first segment end closes a segment that began in an
      // earlier tile: keep the part inside this tile for the fixup.
      recs.put(recs.head, t, lane > 0 ? combine(ex, pend) : pend);
    }
  }
  // Staged tuples out (LDS operations of one wave complete in order): lane q
  // stores half q % 2 of slot q / 2, the pad word as zero.
  wave_lds_fence();
  if (staged) {
    for (int q = lane; q < 2 * static_cast<int>(n_win); q += kWave) {
      const int slot = q >> 1;
      const int4 w = reinterpret_cast<const int4*>(obuf + slot * kTupStride)[q & 1];
      if (obuf[slot * kTupStride + 7]) {
        float4* o = reinterpret_cast<float4*>(seg_out + kTupStride * (s_lo + slot)) + (q & 1);
        *o = make_float4(__int_as_float(w.x), __int_as_float(w.y), __int_as_float(w.z),
                         (q & 1) ? 0.f : __int_as_float(w.w));
      }
    }
  }
  const unsigned long long end_mask = __ballot(any_end);
  const unsigned long long head_mask = __ballot(any_head);
  if (lane == kWave - 1) {
    const int flags = (start_head ? kStartHead : 0) | (end_mask ? kHasEnd : 0) |
                      (head_mask ? kHasHead : 0) | (have ? kTailOpen : 0);
    recs.flags[t] = flags;
    if (have) recs.put(recs.tail, t, inc);
    if (!start_head && !end_mask) recs.put(recs.head, t, inc);
  }
}

// Tiles [t_first, t_end), one wave each; the ragged last tile (if any) loads
// its samples element by element.  The 16-bit forms are held to 64 registers
// (eight waves per SIMD; the ragged tile's code would otherwise push BF16 to
// 65), FP32 to six waves.
template <int DT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(DT == kF32 ? 6 : 8))) void seg_fwd_kernel(SamplesDev s,
                                                         const int64_t* __restrict__ off,
                                                         int64_t n_seg, int64_t n_tiles,
                                                         int64_t t_first, int64_t t_end,
                                                         float* __restrict__ seg_out,
                                                         TileRecs recs) {
  __shared__ __align__(16) int endloc_all[kWavesPerBlock][kTile];
  __shared__ float park_all[kWavesPerBlock][kRangeFields * kWave];
  // wave index made provably uniform, so per-tile loads go through the scalar unit
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x / kWave));
  const int lane = threadIdx.x % kWave;
  const int64_t t = t_first + static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wave;
  const bool active = t < t_end;
  // Issue the sample loads first: their latency overlaps the setup below.
  RawRun<DT> raw;
  if (active) load_lane(raw, s, t, lane);
  int* endloc = endloc_all[wave];
  init_ends(endloc, s.n, t, lane);
  __syncthreads();
  int64_t s_lo = 0, n_win = 0;
  bool start_head = false;
  if (active) {
    s_lo = recs.first_seg[t];
    n_win = stage_ends<true>(off, n_seg, s.n, t, n_tiles, s_lo, lane, endloc, seg_out);
    start_head = (off[s_lo] == t * kTile);
  }
  __syncthreads();
  if (!active) return;
  fwd_tile<DT>(s, n_seg, t, s_lo, n_win, start_head, lane, endloc, park_all[wave],
                     seg_out, recs, &raw);
}

// Completes segments that cross tile boundaries and leaves, in every tile
// such a segment passes through, the carries the backward needs:
//   pre: the part of the tile's first segment that lies before the tile (the
//        open tail of the tile where the segment starts, then the tiles
//        without a head in between);
//   suf: the part of the tile's last segment that lies after it (the tiles
//        without an end up to the tile where it ends, then that tile's head);
//   the tile in which a crossing segment ends writes its tuple, pre (+) head.
// One thread per tile; the thread of the tile where a segment starts folds
// forward along that segment's tiles, the thread of the tile where it ends
// folds backward, so a segment spanning M tiles costs O(M) record reads.
__global__ void seg_fixup_kernel(int64_t n_tiles, int64_t n_seg, float* __restrict__ seg_out,
                                 TileRecs recs) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n_tiles) return;
  const int fl = recs.flags[t];
  // Carries into the tiles after t.  A tile where a segment starts (kHasHead)
  // opens the chain of its last segment: the tiles that follow it, up to the
  // next such tile, receive the running fold of that segment's parts (this
  // tile's tail, then whole tiles) as their prefix, and the tile where the
  // segment ends also completes its tuple.  Each tile is visited by one chain,
  // so the work is linear in the tile count.  (The empty range is not an
  // identity of combine in the positive form, whose depths are relative to the
  // ranges' end midpoints, so each fold starts from its first part.)
  if ((fl & kHasHead) && (fl & kTailOpen)) {
    Part acc = recs.get(recs.tail, t);
    for (int64_t u = t + 1; u < n_tiles; ++u) {
      const int fu = recs.flags[u];
      if (!(fu & kStartHead)) {
        // (the tile right after the start reads the start's tail itself)
        if (u > t + 1) recs.put(recs.pre, u, acc);
        if (fu & kHasEnd) {
          const int64_t sgi = recs.first_seg[u];
          if (sgi >= 0 && sgi < n_seg) write_tuple(seg_out, sgi, combine(acc, recs.get(recs.head, u)));
        }
      }
      if (fu & kHasHead) break;
      acc = combine(acc, recs.get(recs.head, u));
    }
  }
  // Carries out of the tiles before t.  A tile where a segment ends (kHasEnd),
  // and a virtual one past the last tile, closes the chain of the tiles before
  // it whose last segment is still open: walking down, each such tile receives
  // the fold of the following tiles' parts up to the end as its suffix.
  const bool anchor = (fl & kHasEnd) != 0;
  for (int pass = 0; pass < 2; ++pass) {
    int64_t e;
    if (pass == 0) {
      if (!anchor) continue;
      e = t;
    } else {
      if (t != n_tiles - 1) continue;
      e = n_tiles;  // the virtual end
    }
    Part acc;
    bool have = false;
    if (e < n_tiles) {
      acc = recs.get(recs.head, e);
      have = true;
    }
    for (int64_t u = e - 1; u >= 0; --u) {
      const int fu = recs.flags[u];
      // (the tile right before the end reads the end's head itself)
      if (have && (fu & kTailOpen) && u < e - 1) recs.put(recs.suf, u, acc);
      if (fu & kHasEnd) break;
      const Part part = recs.get(recs.head, u);
      acc = have ? combine(part, acc) : part;
      have = true;
    }
  }
}

// One step of the backward's reverse sweep for sample q (see bwd_tile).  g
// holds the ending segment's tuple gradient with g[6] doubled.  BRANCH: the
// restart at a segment end is a branch around rare work rather than selects.
template <bool BRANCH>
__device__ __forceinline__ void reverse_step(const Smp& q, float PTj, float PZj, bool endf,
                                             int endloc_j, int64_t s_lo, int64_t n_seg,
                                             const float* __restrict__ gl,
                                             const float* __restrict__ gseg, float (&g)[7],
                                             float& SG, float& SA, float& SF, float& SL, float& mf,
                                             float& TN, float& dsg, float& dc0, float& dc1,
                                             float& dc2) {
  const float Ti1 = PTj * q.e;
  if (!BRANCH) {
    SG = endf ? 0.f : SG;
    SA = endf ? 0.f : SA; SF = endf ? 0.f : SF; SL = endf ? 0.f : SL;
    mf = endf ? q.m : mf;
    TN = endf ? Ti1 : TN;
  }
  if (!BRANCH || endf) {  // sample j ends its segment: the suffix restarts
    if (BRANCH) {
      SG = 0.f; SA = 0.f; SF = 0.f; SL = 0.f;
      mf = q.m;
      TN = Ti1;
    }
    if (endloc_j >= 0) {
      if (endloc_j < kStagedSegs) {
#pragma unroll
        for (int k = 0; k < 7; ++k) g[k] = gl[k * kStagedSegs + endloc_j];
      } else {
        const Tup7 t = load_tup7(gseg, s_lo + endloc_j);
#pragma unroll
        for (int k = 0; k < 6; ++k) g[k] = t.v[k];
        g[6] = 2.f * t.v[6];
      }
    }
  }
  const float w = PTj * q.alpha;
  const float Zs = fmaf(SA, mf - q.m, SF);  // sum_{k>j} w_k (m_k - m_j)
  const float wd3 = w * q.delta * (1.f / 3.f);
  const float gc = fmaf(g[3], q.c2, fmaf(g[2], q.c1, g[1] * q.c0));  // g_C . c_j
  // half the distortion term: T_N Zp_j + (T_{j+1} - w_j - A_{<j}) Zs + T_{j+1} w_j delta_j / 3 - SL,
  // where A_{<j} = 1 - T_j inside the segment makes T_{j+1} - w_j - A_{<j} = 2 T_{j+1} - 1
  const float hL = fmaf(TN, PZj, fmaf(fmaf(2.f, Ti1, -1.f), Zs, fmaf(Ti1, wd3, -SL)));
  const float dtau = fmaf(g[6], hL, fmaf(g[5], fmaf(q.m, TN, -Zs),
                                         fmaf(g[4], TN, g[0] + fmaf(Ti1, gc, -SG))));
  dsg = q.delta * dtau;
  dc0 = w * g[1];
  dc1 = w * g[2];
  dc2 = w * g[3];
  // sample j joins the suffix
  SG = fmaf(w, gc, SG);
  SL = fmaf(2.f * w, Zs, fmaf(w, wd3, SL));
  SF = Zs;
  SA += w;
  mf = q.m;
}

template <int DT, bool RAGGED>
__device__ __forceinline__ void bwd_tile(const SamplesDev& s, int64_t n_seg, int64_t t,
                                         int flags, int flags_prev, int flags_next, int64_t ts,
                                         int64_t s_lo, int lane, const int* endloc,
                                         const float* __restrict__ gl, float* park,
                                         const TileRecs& recs,
                                         const float* __restrict__ gseg, void* __restrict__ gsig_p,
                                         void* __restrict__ grgb_p, const RawRun<DT>* raw) {
  const bool start_head = (flags & kStartHead) != 0;
  const bool tail_open = (flags & kTailOpen) != 0;
  // Only the 16-bit forms request the tile carries before the lane work and
  // branch around rare restarts (measured: each helps them by a few percent
  // and slows the FP32 form, which runs three waves per SIMD: its 8 KB
  // gradient image fills the LDS).
  constexpr bool kEager = DT != kF32;
  // Tile-uniform carries: the prefix into the tile, the suffix out of it and
  // the gradient of the segment that leaves it (g_L doubled, as in the sweep).
  Part pre_t, suf_t;
  float gt[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  // A segment that crosses only the boundary before the tile has, as prefix,
  // the previous tile's tail record (the fixup writes prefixes only deeper
  // into longer chains); likewise the suffix of one that ends in the next
  // tile is that tile's head record.
  auto load_carries = [&]() {
    // (the common case is requested first, without waiting for the flags)
    if (!start_head) {
      pre_t = recs.get(recs.tail, t - 1);
      if (!(flags_prev & kHasHead)) pre_t = recs.get(recs.pre, t);
    }
    if (tail_open) {
      suf_t = recs.get(recs.head, t + 1);
      if (!(flags_next & kHasEnd)) suf_t = recs.get(recs.suf, t);
      if (ts >= 0 && ts < n_seg) {
        const Tup7 t = load_tup7(gseg, ts);
#pragma unroll
        for (int k = 0; k < 7; ++k) gt[k] = t.v[k];
        gt[6] *= 2.f;
      }
    }
  };
  if (kEager) load_carries();
  LaneRun<DT, RAGGED> R;
  R.load(endloc, lane, start_head, raw);

  // Pass 1: serial fold.  Records, for every sample, the transmittance and
  // sum_{k<j} w_k (m_j - m_k) in front of it, relative to the start of the
  // open range (the lane start for samples before the lane's first head), and
  // keeps the lane's first range (up to its first segment end) for the reverse
  // scan.  Only the fields the prefix needs (tau, A, B, T) restart at heads: no
  // head precedes the lane's first end except sample 0, so colour, F and L
  // extend the same fold unrestarted and are exact wherever they are used.
  float Tl[kRun], Zl[kRun];
  Range cur = range_identity();
  cur.m0 = R.x[0].m;
  cur.m1 = R.x[0].m;
  float Tc = 1.f;
  bool cur_head = R.h0, seen_end = false;
  int first_end = -1;
  int fhp = R.h0 ? 0 : kRun;  // position of the lane's first head
#pragma unroll
  for (int j = 0; j < kRun; ++j) {
    const Smp& q = R.x[j];
    if (kEager) {
      if (j > 0 && R.head(j)) {  // (a branch: heads are rare)
        cur.tau = 0.f;
        cur.A = 0.f;
        cur.B = 0.f;
        Tc = 1.f;
        cur_head = true;
        fhp = fhp == kRun ? j : fhp;
      }
    } else if (j > 0) {
      const bool hd = R.head(j);
      cur.tau = hd ? 0.f : cur.tau;
      cur.A = hd ? 0.f : cur.A;
      cur.B = hd ? 0.f : cur.B;
      Tc = hd ? 1.f : Tc;
      cur_head = cur_head || hd;
      fhp = (hd && fhp == kRun) ? j : fhp;
    }
    const float Z = fmaf(cur.A, q.m - cur.m1, cur.B);  // sum_{k<j} w_k (m_j - m_k)
    Tl[j] = Tc;
    Zl[j] = Z;
    const float w = Tc * q.alpha;
    cur.L = fmaf(w, fmaf(2.f, Z, w * q.delta * (1.f / 3.f)), cur.L);
    cur.F = fmaf(w, q.m - cur.m0, cur.F);
    cur.cr = fmaf(w, q.c0, cur.cr);
    cur.cg = fmaf(w, q.c1, cur.cg);
    cur.cb = fmaf(w, q.c2, cur.cb);
    cur.B = Z;
    cur.A += w;
    cur.tau += q.tau;
    cur.m1 = q.m;
    Tc *= q.e;
    if (R.endf[j] && !seen_end) {
      park_range(park, lane, cur);
      first_end = R.ends[j];
      seen_end = true;
    }
  }
  const bool have = !R.endf[kRun - 1];
  Pre inc = have ? pre_of(cur) : pre_identity();
  bool fin = have ? cur_head : true;
  Range rinc = seen_end ? unpark_range(park, lane) : cur;
  bool rfl = seen_end;
  int rseg = seen_end ? first_end : -1;
  scan_up(inc, fin, lane);
  scan_down(rinc, rfl, rseg, lane);
  const Pre ex = from_lower(inc);
  const int exf = from_lower(static_cast<int>(fin));
  const Range sx = from_upper(rinc);
  const int sxf = from_upper(static_cast<int>(rfl));
  const int sxseg = from_upper(rseg);

  if (!kEager) load_carries();

  // Prefix of the segment in front of the lane (identity if sample 0 is a head).
  Pre pc = pre_identity();
  if (!R.h0) {
    if (lane > 0 && exf) pc = ex;
    else if (!start_head) {
      const Pre pt = pre_of(range_of(pre_t));
      pc = lane > 0 ? combine(pt, ex) : pt;
    }
  }
  // Suffix behind the lane's last sample, in its own frame (unused if that
  // sample ends its segment), and the gradient of the segment it belongs to.
  Range sc = range_identity();
  float g[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (have) {
    if (lane < kWave - 1 && sxf) {
      sc = sx;
      if (kEager && sxseg < kStagedSegs) {
#pragma unroll
        for (int k = 0; k < 7; ++k) g[k] = gl[k * kStagedSegs + sxseg];
      } else {
        const Tup7 t = load_tup7(gseg, s_lo + sxseg);
#pragma unroll
        for (int k = 0; k < 7; ++k) g[k] = t.v[k];
        g[6] *= 2.f;
      }
    } else if (tail_open) {
      const Range st = range_of(suf_t);
      sc = lane < kWave - 1 ? combine(sx, st) : st;
#pragma unroll
      for (int k = 0; k < 7; ++k) g[k] = gt[k];
    }
  }

  // Samples before the lane's first head continue the carried prefix.
  const float Tp = exp_neg(pc.tau);
  float PT[kRun], PZ[kRun];
#pragma unroll
  for (int j = 0; j < kRun; ++j) {
    const bool inF = j < fhp;
    const float Tm = inF ? Tp : 1.f;
    const float Bm = inF ? fmaf(pc.A, R.x[j].m - pc.m1, pc.B) : 0.f;
    PT[j] = Tm * Tl[j];
    PZ[j] = fmaf(Tm, Zl[j], Bm);
  }

  // Pass 3: reverse sweep.  Suffix sums are weighted with each sample's
  // transmittance from the start of its segment:
  //   SC = sum_{k>j} w_k c_k, SA = sum_{k>j} w_k, SF = sum_{k>j} w_k (m_k - mf),
  //   SL = distortion of the samples after j,
  // and dl/dtau_j = g_tau + g_C.(T_{j+1} c_j - SC) + g_A T_N + g_D (m_j T_N - Zs)
  //   + g_L [2 T_N Zp_j - 2 A_{<j} Zs + 2/3 T_{j+1} w_j delta_j - 2 SL + 2 (T_{j+1} - w_j) Zs]
  // with Zs = sum_{k>j} w_k (m_k - m_j) and T_N the segment's transmittance:
  // the derivative of the segment tuple with every difference of positions
  // taken before it is multiplied.
  float SG = 0.f, SA = 0.f, SF = 0.f, SL = 0.f, mf = 0.f, TN = 1.f;
  if (have) {
    const float Tq = PT[kRun - 1] * R.x[kRun - 1].e;
    SG = Tq * fmaf(g[3], sc.cb, fmaf(g[2], sc.cg, g[1] * sc.cr));
    SA = Tq * sc.A; SF = Tq * sc.F; SL = Tq * Tq * sc.L; mf = sc.m0;
    TN = Tq * exp_neg(sc.tau);
  }
  {
    // The lane's samples stay in registers from pass 1 (no re-read).  Each gradient goes to the LDS image of the tile's gradient
    // block (dsigma, then drgb, as laid out in memory) as soon as it is
    // complete; the image is then written with full, contiguous 16-byte
    // stores (stores straight from the lanes, each covering a few bytes of
    // many cache lines, cost the backward 15-20 %).
    float dsg[kRun], dc[3 * kRun];
#pragma unroll
    for (int j = kRun - 1; j >= 0; --j) {
      const Smp& q = R.x[j];
      const int endj = endloc[lane * kRun + j];  // re-read: frees registers across the scans
      reverse_step<kEager>(q, PT[j], PZ[j], RAGGED ? endj != -1 : endj >= 0, endj, s_lo, n_seg, gl, gseg, g, SG, SA, SF,
                   SL, mf, TN, dsg[j], dc[3 * j], dc[3 * j + 1], dc[3 * j + 2]);
      if (DT == kF32) {
        float* img = park;  // [kTile] dsigma, then [kTile][3] drgb
        const int i = lane * kRun + j;
        img[i] = dsg[j];
        img[kTile + 3 * i] = dc[3 * j];
        img[kTile + 3 * i + 1] = dc[3 * j + 1];
        img[kTile + 3 * i + 2] = dc[3 * j + 2];
      } else {
        if ((j & 1) == 0) {  // pairs of 16-bit values
          uint32_t* img = reinterpret_cast<uint32_t*>(park);
          img[(lane * kRun + j) / 2] = pack2<sig_dt(DT)>(dsg[j], dsg[j + 1]);
#pragma unroll
          for (int v = 0; v < 3; ++v)
            img[kTile / 2 + (3 * (lane * kRun + j)) / 2 + v] =
                pack2<rgb_dt(DT)>(dc[3 * j + 2 * v], dc[3 * j + 2 * v + 1]);
        }
      }
    }
    wave_lds_fence();
    if (RAGGED) {
      // Ragged last tile: element stores of the samples that exist.
      const int m = static_cast<int>(s.n - t * kTile);
      using E = std::conditional_t<DT == kF32, float, uint16_t>;
      const E* im = reinterpret_cast<const E*>(park);
      E* gs = static_cast<E*>(gsig_p) + t * kTile;
      E* gc = static_cast<E*>(grgb_p) + 3 * t * kTile;
      for (int k = lane; k < m; k += kWave) gs[k] = im[k];
      for (int k = lane; k < 3 * m; k += kWave) gc[k] = im[kTile + k];
      return;
    }
    // The 16-bit forms write their gradient blocks with non-temporal stores
    // (measured: 616 -> 605 us at K=16, 5.39 -> 5.33 ms at K=64); for the
    // FP32 form, twice the bytes, they cost 2 % (993 -> 1013 us).
    if (DT == kF32) {
      const uint4* img = reinterpret_cast<const uint4*>(park);
      uint4* gs = reinterpret_cast<uint4*>(static_cast<float*>(gsig_p) + t * kTile);
      uint4* gc = reinterpret_cast<uint4*>(static_cast<float*>(grgb_p) + 3 * t * kTile);
#pragma unroll
      for (int q = 0; q < 2; ++q) gs[q * kWave + lane] = img[q * kWave + lane];
#pragma unroll
      for (int q = 0; q < 6; ++q) gc[q * kWave + lane] = img[2 * kWave + q * kWave + lane];
    } else {
      const uint4* img = reinterpret_cast<const uint4*>(park);
      uint4* gs = reinterpret_cast<uint4*>(static_cast<uint16_t*>(gsig_p) + t * kTile);
      uint4* gc = reinterpret_cast<uint4*>(static_cast<uint16_t*>(grgb_p) + 3 * t * kTile);
      constexpr int kSigVec = kTile * 2 / 16;  // 16-byte vectors of dsigma per tile
      static_assert(kSigVec == kWave, "one vector of dsigma per lane");
      store_stream(&gs[lane], img[lane]);
#pragma unroll
      for (int q = 0; q < 3; ++q) store_stream(&gc[q * kWave + lane], img[kSigVec + q * kWave + lane]);
    }
  }
}

template <int DT, bool RAGGED>
__device__ __forceinline__ void seg_bwd_body(
    const SamplesDev& s, const int64_t* __restrict__ off, int64_t n_seg, int64_t n_tiles,
    int64_t t_first, int64_t t_end, const TileRecs& recs,
    const float* __restrict__ gseg, void* __restrict__ gsig_p, void* __restrict__ grgb_p) {
  __shared__ __align__(16) int endloc_all[kWavesPerBlock][kTile];
  __shared__ float gl_all[kWavesPerBlock][7 * kStagedSegs];
  // Parked ranges during the scans; afterwards the image of the tile's
  // gradients (8 or 16 bytes per sample).
  constexpr int kParkWords = DT == kF32 ? 4 * kTile : 2 * kTile;
  __shared__ __align__(16) float park_all[kWavesPerBlock][kParkWords];
  // wave index made provably uniform, so per-tile loads go through the scalar unit
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x / kWave));
  const int lane = threadIdx.x % kWave;
  const int64_t t = t_first + static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wave;
  const bool active = t < t_end;
  RawRun<DT> raw;
  if (active) {
    if (RAGGED) load_lane(raw, s, t, lane);
    else raw.load(s.sigma, s.rgb, s.t0, s.t1, t * kTile + static_cast<int64_t>(lane) * kRun);
  }
  // (requested here so that their latency overlaps the staging below)
  const int flags = active ? recs.flags[t] : 0;
  const int flags_prev = (active && t > 0) ? recs.flags[t - 1] : 0;
  const int flags_next = (active && t + 1 < n_tiles) ? recs.flags[t + 1] : 0;
  // The segment leaving the tile through its last sample, if that segment is
  // open (kTailOpen): the one holding the next tile's first sample.
  const int64_t ts = (active && t + 1 < n_tiles) ? recs.first_seg[t + 1] : -1;
  int* endloc = endloc_all[wave];
  float* gl = gl_all[wave];
  if (RAGGED) {
    init_ends(endloc, s.n, t, lane);
  } else {
#pragma unroll
    for (int j = 0; j < kRun; ++j) endloc[lane + kWave * j] = -1;
  }
  __syncthreads();
  int64_t s_lo = 0;
  if (active) {
    s_lo = recs.first_seg[t];
    stage_ends<false>(off, n_seg, s.n, t, n_tiles, s_lo, lane, endloc, nullptr, gseg, gl);
  }
  __syncthreads();
  if (!active) return;
  bwd_tile<DT, RAGGED>(s, n_seg, t, flags, flags_prev, flags_next, ts, s_lo, lane, endloc, gl, park_all[wave], recs, gseg, gsig_p, grgb_p,
                     &raw);
}

// Full tiles, held to 128 registers so that four waves share each SIMD; the
// ragged last tile (element loads and stores) is a launch of its own, so the
// common instance carries none of its code.
template <int DT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void seg_bwd_kernel(
    SamplesDev s, const int64_t* __restrict__ off, int64_t n_seg, int64_t n_tiles,
    int64_t t_first, int64_t t_end, TileRecs recs,
    const float* __restrict__ gseg, void* __restrict__ gsig_p, void* __restrict__ grgb_p) {
  seg_bwd_body<DT, false>(s, off, n_seg, n_tiles, t_first, t_end, recs, gseg, gsig_p, grgb_p);
}
template <int DT>
__global__ __launch_bounds__(kBlock) void seg_bwd_tail_kernel(
    SamplesDev s, const int64_t* __restrict__ off, int64_t n_seg, int64_t n_tiles,
    int64_t t_first, int64_t t_end, TileRecs recs,
    const float* __restrict__ gseg, void* __restrict__ gsig_p, void* __restrict__ grgb_p) {
  seg_bwd_body<DT, true>(s, off, n_seg, n_tiles, t_first, t_end, recs, gseg, gsig_p, grgb_p);
}

static inline unsigned grid_for(int64_t count, int block) {
  return static_cast<unsigned>((count + block - 1) / block);
}

// All tiles in one launch; the ragged last tile (if any) loads its samples
// element by element.
template <int DT>
static void launch_fwd_dt(const SamplesDev& s, const int64_t* off, int64_t n_seg, int64_t nt,
                          float* seg_out, const TileRecs& recs, hipStream_t st) {
  hipLaunchKernelGGL((seg_fwd_kernel<DT>), dim3(grid_for(nt, kWavesPerBlock)), dim3(kBlock), 0,
                     st, s, off, n_seg, nt, static_cast<int64_t>(0), nt, seg_out, recs);
}

template <int DT>
static void launch_bwd_dt(const SamplesDev& s, const int64_t* off, int64_t n_seg, int64_t nt,
                          const TileRecs& recs, const float* gseg, void* gs, void* gc,
                          hipStream_t st) {
  const int64_t n_full = s.n / kTile;
  if (n_full > 0)
    hipLaunchKernelGGL((seg_bwd_kernel<DT>), dim3(grid_for(n_full, kWavesPerBlock)), dim3(kBlock), 0,
                       st, s, off, n_seg, nt, static_cast<int64_t>(0), n_full, recs, gseg, gs, gc);
  if (n_full < nt)
    hipLaunchKernelGGL((seg_bwd_tail_kernel<DT>), dim3(1), dim3(kBlock), 0, st, s, off, n_seg, nt,
                       n_full, nt, recs, gseg, gs, gc);
}

hipError_t launch_segments_fwd(const SamplesDev& s, const int64_t* off, int64_t n_seg,
                               float* seg_out, void* workspace, hipStream_t stream) {
  if (n_seg == 0) return hipSuccess;
  if (s.n == 0) {
    hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for(kTupStride * n_seg, 256)), dim3(256), 0, stream,
                       seg_out, kTupStride * n_seg);
    return hipGetLastError();
  }
  const int64_t nt = num_tiles(s.n);
  const TileRecs recs = TileRecs::view(workspace, nt);
  hipLaunchKernelGGL(plan_kernel, dim3(grid_for(n_seg, 256)), dim3(256), 0, stream, off, n_seg, nt,
                     recs);
  switch (s.dtype) {
    case kF32: launch_fwd_dt<kF32>(s, off, n_seg, nt, seg_out, recs, stream); break;
    case kBF16: launch_fwd_dt<kBF16>(s, off, n_seg, nt, seg_out, recs, stream); break;
    case kBF16F16: launch_fwd_dt<kBF16F16>(s, off, n_seg, nt, seg_out, recs, stream); break;
    default: launch_fwd_dt<kF16>(s, off, n_seg, nt, seg_out, recs, stream); break;
  }
  hipLaunchKernelGGL(seg_fixup_kernel, dim3(grid_for(nt, 256)), dim3(256), 0, stream, nt, n_seg,
                     seg_out, recs);
  return hipGetLastError();
}

hipError_t launch_segments_bwd(const SamplesDev& s, const int64_t* off, int64_t n_seg,
                               const void* workspace, const float* grad_seg, void* grad_sigma,
                               void* grad_rgb, hipStream_t stream) {
  if (s.n == 0 || n_seg == 0) return hipSuccess;
  const int64_t nt = num_tiles(s.n);
  const TileRecs recs = TileRecs::view(const_cast<void*>(workspace), nt);
  switch (s.dtype) {
    case kF32: launch_bwd_dt<kF32>(s, off, n_seg, nt, recs, grad_seg, grad_sigma, grad_rgb, stream); break;
    case kBF16: launch_bwd_dt<kBF16>(s, off, n_seg, nt, recs, grad_seg, grad_sigma, grad_rgb, stream); break;
    case kBF16F16: launch_bwd_dt<kBF16F16>(s, off, n_seg, nt, recs, grad_seg, grad_sigma, grad_rgb, stream); break;
    default: launch_bwd_dt<kF16>(s, off, n_seg, nt, recs, grad_seg, grad_sigma, grad_rgb, stream); break;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- no-allocation forward
// xl_render_segments_fwd_static keeps the tile records in this file-scope
// device array instead of a caller workspace.  Every GPU the library runs on
// holds its own copy until the process ends.  In host code `scratch` names a
// host-side stand-in, not device memory: host code uses only the address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[XL_STATIC_SCRATCH_BYTES];

hipError_t static_scratch(void** ptr) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (addr[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

}  // namespace xl
