// Synthetic sample generator on the device: the stand-in for per-region NeRF
// evaluation in the serving loop, and the fast path for large benchmark
// inputs.  It is the device twin of the host generator in synth.py: the same
// counter-based draws (SplitMix64 output function, Steele, Lea & Flood 2014),
// the same float32 log/exp/cos built from IEEE operations in a fixed order
// (no fused multiply-add), the same sequential float64 position sums and box
// tags, so every sample, the segment structure and the region-major layout
// are bit-identical to the host's.
//
// Pipeline for a batch of rays (all asynchronous on one stream):
//   gen_struct   one lane per ray: widths, positions and box tags -> the ray's
//                segments (runs of one box) and its position scale/start
//   block_hist   per block of 256 rays, segments per box
//   scan         exclusive scans (segments per ray -> ray_offsets; per-box
//                block counts -> stable region-major slots)
//   gen_rank     packed index of every segment (stable counting sort by box)
//   scan         packed segment lengths -> seg_offsets
//   gen_fill     one lane per 64-sample chunk of a ray: regenerate its samples
//                into their packed slots
#include <cstdio>

#include "../../include/xl.h"
#include "internal.h"
#include "xl_device.hpp"

// Every floating-point operation in this file rounds on its own, as on the
// host, which never fuses a multiply into an add.  The __*_rn wrappers of the
// HIP headers are plain operators that the compiler still contracts into
// fused multiply-adds, so the generator uses these, defined where contraction
// is off.  Division and square root are the correctly rounded ones.
#pragma clang fp contract(off)

namespace xl {

__device__ __forceinline__ float f_mul(float a, float b) { return a * b; }
__device__ __forceinline__ float f_add(float a, float b) { return a + b; }
__device__ __forceinline__ float f_sub(float a, float b) { return a - b; }
__device__ __forceinline__ float f_div(float a, float b) { return a / b; }
// (__fsqrt_rn is the approximate hardware square root in these headers; the
// builtin is correctly rounded.)
__device__ __forceinline__ float f_sqrt(float a) { return __builtin_sqrtf(a); }
__device__ __forceinline__ double d_mul(double a, double b) { return a * b; }
__device__ __forceinline__ double d_add(double a, double b) { return a + b; }
__device__ __forceinline__ double d_sub(double a, double b) { return a - b; }
__device__ __forceinline__ double d_div(double a, double b) { return a / b; }
__device__ __forceinline__ double d_sqrt(double a) { return __builtin_sqrt(a); }

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
constexpr int kRayBlock = 256;
constexpr int kDirTries = 64;
constexpr int kRaySlots = 256;
constexpr int kSampleStride = 2;

__host__ __device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}
__device__ __forceinline__ uint64_t draw(uint64_t key, uint64_t slot) {
  return mix64(key + (slot + 1ull) * kGamma);
}
__device__ __forceinline__ double u53(uint64_t v) {
  return static_cast<double>(v >> 11) * 0x1p-53;
}
// Bits [shift, shift + bits) of v as k / 2^bits.
__device__ __forceinline__ double field(uint64_t v, int shift, int bits) {
  return static_cast<double>((v >> shift) & ((1ull << bits) - 1ull)) * ldexp(1.0, -bits);
}
__device__ __forceinline__ float u24_open0(uint64_t v) {
  return f_mul(static_cast<float>((v >> 40) + 1ull), 0x1p-24f);
}

// float32 natural log from IEEE operations only: u = 2^e x, x in
// [sqrt(1/2), sqrt(2)), log x = 2 atanh(s) with s = (x - 1)/(x + 1), summed to
// s^9.  Operation order and constants match the host twin exactly.
__device__ __forceinline__ float log_f32(float u) {
  const int bits = __float_as_int(u);
  int e = ((bits >> 23) & 0xff) - 127;
  float x = __int_as_float((bits & 0x7fffff) | 0x3f800000);
  if (x > __int_as_float(0x3FB504F3)) {
    x = f_mul(x, 0.5f);
    e += 1;
  }
  const float s = f_div(f_sub(x, 1.f), f_add(x, 1.f));
  const float s2 = f_mul(s, s);
  float p = f_add(__int_as_float(0x3E124925), f_mul(s2, __int_as_float(0x3DE38E39)));
  p = f_add(__int_as_float(0x3E4CCCCD), f_mul(s2, p));
  p = f_add(__int_as_float(0x3EAAAAAB), f_mul(s2, p));
  p = f_mul(s2, p);
  const float lx = f_mul(2.f, f_add(s, f_mul(s, p)));
  return f_add(f_mul(static_cast<float>(e), __int_as_float(0x3F317218)), lx);
}

// exp of float32 values in (-87, 88) from IEEE operations only (twin of the host
// generator's exp_f32): k = rint(y / ln 2), r = (y - k ln2_hi) - k ln2_lo
// (Cody & Waite), exp r by its Taylor series to r^7 (Horner), times 2^k.
__device__ __forceinline__ float exp_f32(float y) {
  const float k = rintf(f_mul(y, __int_as_float(0x3FB8AA3B)));
  const float r = f_sub(f_sub(y, f_mul(k, __int_as_float(0x3F317200))),
                            f_mul(k, __int_as_float(0x35BFBE8E)));
  float p = f_add(1.f, f_mul(r, static_cast<float>(1.0 / 7.0)));
  p = f_add(1.f, f_mul(f_mul(r, static_cast<float>(1.0 / 6.0)), p));
  p = f_add(1.f, f_mul(f_mul(r, static_cast<float>(1.0 / 5.0)), p));
  p = f_add(1.f, f_mul(f_mul(r, static_cast<float>(1.0 / 4.0)), p));
  p = f_add(1.f, f_mul(f_mul(r, static_cast<float>(1.0 / 3.0)), p));
  p = f_add(1.f, f_mul(f_mul(r, static_cast<float>(1.0 / 2.0)), p));
  p = f_add(1.f, f_mul(f_mul(r, 1.f), p));
  return ldexpf(p, static_cast<int>(k));
}

// cos(2 pi u) for u in [0, 1) from IEEE operations only (twin of cos2pi_f32):
// exact quadrant split of 4u, angle in [0, pi/4], Taylor series to a^9 / a^8.
__device__ __forceinline__ float cos2pi_f32(float u) {
  const float t = f_mul(u, 4.f);
  const float n = floorf(t);
  const float f = f_sub(t, n);
  const bool flip = f > 0.5f;
  const float a = f_mul(flip ? f_sub(1.f, f) : f, __int_as_float(0x3FC90FDB));
  const float a2 = f_mul(a, a);
  // cos a = 1 - (a2/2)(1 - (a2/12)(1 - (a2/30)(1 - a2/56)))
  float c = f_sub(1.f, f_mul(a2, static_cast<float>(1.0 / 56.0)));
  c = f_sub(1.f, f_mul(f_mul(a2, static_cast<float>(1.0 / 30.0)), c));
  c = f_sub(1.f, f_mul(f_mul(a2, static_cast<float>(1.0 / 12.0)), c));
  c = f_sub(1.f, f_mul(f_mul(a2, 0.5f), c));
  // sin a = a (1 - (a2/6)(1 - (a2/20)(1 - (a2/42)(1 - a2/72))))
  float sn = f_sub(1.f, f_mul(a2, static_cast<float>(1.0 / 72.0)));
  sn = f_sub(1.f, f_mul(f_mul(a2, static_cast<float>(1.0 / 42.0)), sn));
  sn = f_sub(1.f, f_mul(f_mul(a2, static_cast<float>(1.0 / 20.0)), sn));
  sn = f_sub(1.f, f_mul(f_mul(a2, static_cast<float>(1.0 / 6.0)), sn));
  sn = f_mul(a, sn);
  const float ca = flip ? sn : c;
  const float sa = flip ? c : sn;
  const int q = static_cast<int>(n) & 3;
  return q == 0 ? ca : (q == 1 ? -sa : (q == 2 ? -ca : sa));
}

// Samples of a ray are generated in chunks of kChunk by independent threads;
// the structure pass records the running position at every chunk start, so
// each chunk continues the same sequential float64 sum.
constexpr int kChunk = 64;

struct GenDev {
  int64_t n_rays, ray0;
  int32_t n_min, n_max, gx, gy, gz, max_segs;
  int32_t chunks;  // chunks per ray: ceil(n_max / kChunk)
  float wm, mu, sg;
  double zero_frac, t_far;
  uint64_t seedkey;  // mix64(seed)
};

struct RayState {
  uint64_t key;
  int32_t count;
  double o[3], d[3];
  double u_start;
};

__device__ __forceinline__ RayState ray_state(const GenDev& g, int64_t r) {
  RayState s;
  s.key = mix64(g.seedkey + static_cast<uint64_t>(g.ray0 + r) * kGamma);
#pragma unroll
  for (int c = 0; c < 3; ++c) s.o[c] = d_sub(d_mul(2.0, u53(draw(s.key, c))), 1.0);
  const uint64_t span = static_cast<uint64_t>(g.n_max - g.n_min + 1);
  s.count = g.n_min + static_cast<int32_t>(((draw(s.key, 3) >> 32) * span) >> 32);
  s.u_start = u53(draw(s.key, 4));
  s.d[0] = 0.0; s.d[1] = 0.0; s.d[2] = 1.0;
  for (int j = 0; j < kDirTries; ++j) {
    double v[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
      v[c] = d_sub(d_mul(2.0, u53(draw(s.key, 16 + 3 * j + c))), 1.0);
    const double r2 = d_add(d_add(d_mul(v[0], v[0]), d_mul(v[1], v[1])),
                                d_mul(v[2], v[2]));
    if (r2 > 1e-12 && r2 <= 1.0) {
      const double q = d_sqrt(r2);
#pragma unroll
      for (int c = 0; c < 3; ++c) s.d[c] = d_div(v[c], q);
      break;
    }
  }
  return s;
}

__device__ __forceinline__ double width_of(const GenDev& g, uint64_t key, int i) {
  const uint64_t v = draw(key, kRaySlots + static_cast<uint64_t>(kSampleStride) * i);
  return static_cast<double>(-f_mul(g.wm, log_f32(u24_open0(v))));
}

__device__ __forceinline__ int box_of(const GenDev& g, const RayState& s, float t0, float t1) {
  const double mid = d_mul(0.5, d_add(static_cast<double>(t0), static_cast<double>(t1)));
  const int gsz[3] = {g.gx, g.gy, g.gz};
  int cell[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double p = d_add(s.o[c], d_mul(mid, s.d[c]));
    const double f = floor(d_mul(d_mul(d_add(p, 1.0), 0.5), static_cast<double>(gsz[c])));
    int64_t k = static_cast<int64_t>(f);
    k = k < 0 ? 0 : (k > gsz[c] - 1 ? gsz[c] - 1 : k);
    cell[c] = static_cast<int>(k);
  }
  return cell[0] + g.gx * (cell[1] + g.gy * cell[2]);
}

// Workspace views (all per-ray arrays have n_rays entries; segment lists have
// max_segs entries per ray).
struct GenWs {
  int32_t* nseg;      // [R]
  int32_t* seg_box;   // [R * M]
  int32_t* seg_len;   // [R * M]
  int64_t* seg_pid;   // [R * M] packed index
  double* scale;      // [R]
  double* s0;         // [R]
  int64_t* nseg64;    // [R]      scan input
  int64_t* ray_off;   // [R + 1]  scan output (ray_offsets)
  int64_t* blk_cnt;   // [K * nblk]
  int64_t* blk_base;  // [K * nblk + 1]
  int64_t* plen;      // [R * M]  packed segment lengths
  int64_t* seg_off;   // [R * M + 1]
  int64_t* seg_ids;   // [R * M]
  int64_t* scan_tmp;  // scan scratch
  int32_t* err;       // [1] 1 if some ray had more segments than max_segs
  double* chunk_run;  // [R * chunks] position at the start of each chunk
  int64_t* nchunk;    // [R]      chunks of each ray (scan input)
  int64_t* chunk_base;// [R + 1]  first compact chunk of each ray (scan output)
  int32_t* chunk_ray; // [R * chunks] ray of each compact chunk
};

// Structure of one ray: its position scale and start, the position at every
// chunk start, and its segments (runs of samples in one box).
__device__ __forceinline__ void struct_ray(const GenDev& g, const GenWs& w, int64_t r) {
  const RayState s = ray_state(g, r);
  double tot = 0.0;
  for (int i = 0; i < s.count; ++i) tot = d_add(tot, width_of(g, s.key, i));
  const double scale = tot > g.t_far ? d_div(g.t_far, tot) : 1.0;
  const double rest = d_sub(g.t_far, d_mul(tot, scale));
  const double s0 = d_mul(s.u_start, rest > 0.0 ? rest : 0.0);
  w.scale[r] = scale;
  w.s0[r] = s0;
  const int M = g.max_segs;
  // The open segment's length stays in a register and is stored when the
  // segment closes: a read-modify-write of memory per sample would put a
  // memory round trip on this serial loop.  Past max_segs the last segment
  // takes the remaining samples (and err is raised).
  int k = -1, cur = -1, len = 0;
  double run = s0;
  for (int i = 0; i < s.count; ++i) {
    if (i % kChunk == 0) w.chunk_run[r * g.chunks + i / kChunk] = run;
    const double t0 = run;
    run = d_add(run, d_mul(width_of(g, s.key, i), scale));
    const int b = box_of(g, s, static_cast<float>(t0), static_cast<float>(run));
    if (b != cur) {
      if (k + 1 < M) {
        if (k >= 0) w.seg_len[r * M + k] = len;
        ++k;
        w.seg_box[r * M + k] = b;
        len = 0;
      } else {
        w.err[0] = 1;
      }
      cur = b;
    }
    ++len;
  }
  if (k >= 0) w.seg_len[r * M + k] = len;
  w.nseg[r] = k + 1;
  w.nseg64[r] = k + 1;
  w.nchunk[r] = (s.count + kChunk - 1) / kChunk;
}

// One lane per ray.  The lanes of a wave loop as long as their longest ray,
// so each block first ranks its kStructRays rays by sample count; a lane then
// takes the rays of rank tid and tid + kStructBlock, and each wave's loops
// run over rays of similar length.  (Blocks stay at two waves: wider ones
// are starved of slots next to another stream's kernels of two-wave blocks.)
constexpr int kStructBlock = 128;
constexpr int kStructRays = 2 * kStructBlock;

__global__ __launch_bounds__(kStructBlock) void gen_struct_kernel(GenDev g, GenWs w) {
  __shared__ int cnt[kStructRays];
  __shared__ int perm[kStructRays];
  const int tid = threadIdx.x;
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kStructRays;
  const uint64_t span = static_cast<uint64_t>(g.n_max - g.n_min + 1);
  int mine[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int64_t r = r0 + tid + h * kStructBlock;
    mine[h] = 0x7fffffff;  // past the last ray: ranked last
    if (r < g.n_rays) {
      const uint64_t key = mix64(g.seedkey + static_cast<uint64_t>(g.ray0 + r) * kGamma);
      mine[h] = g.n_min + static_cast<int32_t>(((draw(key, 3) >> 32) * span) >> 32);
    }
    cnt[tid + h * kStructBlock] = mine[h];
  }
  __syncthreads();
  int rank[2] = {0, 0};
  for (int j = 0; j < kStructRays; ++j) {
    const int c = cnt[j];
#pragma unroll
    for (int h = 0; h < 2; ++h)
      rank[h] += (c < mine[h] || (c == mine[h] && j < tid + h * kStructBlock)) ? 1 : 0;
  }
  perm[rank[0]] = tid;
  perm[rank[1]] = tid + kStructBlock;
  __syncthreads();
#pragma unroll 1
  for (int h = 0; h < 2; ++h) {
    const int64_t r = r0 + perm[tid + h * kStructBlock];
    if (r < g.n_rays) struct_ray(g, w, r);
  }
}

// Ray of every compact chunk (the chunks of all rays, ray after ray).
__global__ void chunk_map_kernel(GenDev g, GenWs w) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= g.n_rays) return;
  const int64_t b = w.chunk_base[r], e = w.chunk_base[r + 1];
  for (int64_t i = b; i < e; ++i) w.chunk_ray[i] = static_cast<int32_t>(r);
}

// Segments per box in each block of kRayBlock rays (box-major layout).
__global__ void block_hist_kernel(GenDev g, GenWs w, int64_t nblk, int K) {
  __shared__ int hist[256];
  const int64_t blk = blockIdx.x;
  for (int b = threadIdx.x; b < K; b += blockDim.x) hist[b] = 0;
  __syncthreads();
  const int64_t r = blk * kRayBlock + threadIdx.x;
  if (r < g.n_rays) {
    const int M = g.max_segs;
    for (int k = 0; k < w.nseg[r]; ++k) atomicAdd(&hist[w.seg_box[r * M + k]], 1);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < K; b += blockDim.x) w.blk_cnt[b * nblk + blk] = hist[b];
}

// Stable region-major slot of every segment: all segments of box b in earlier
// blocks and earlier boxes (blk_base), plus those of earlier rays in the block.
__global__ void gen_rank_kernel(GenDev g, GenWs w, int64_t nblk, int K) {
  __shared__ int wave_cnt[kRayBlock / kWave][256];
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int64_t blk = blockIdx.x;
  const int64_t r = blk * kRayBlock + threadIdx.x;
  const bool valid = r < g.n_rays;
  const int M = g.max_segs;
  const int ns = valid ? w.nseg[r] : 0;
  int boxes[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) boxes[k] = (k < ns && k < M) ? w.seg_box[r * M + k] : -1;
  int rank_in_wave[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) rank_in_wave[k] = 0;
  const unsigned long long lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  for (int b = 0; b < K; ++b) {
    bool has = false;
#pragma unroll
    for (int k = 0; k < 16; ++k) has |= boxes[k] == b;
    const unsigned long long m = __ballot(has);
    if (lane == 0) wave_cnt[wave][b] = __popcll(m);
    const int rk = __popcll(m & lt);
#pragma unroll
    for (int k = 0; k < 16; ++k)
      if (boxes[k] == b) rank_in_wave[k] = rk;
  }
  __syncthreads();
  if (!valid) return;
  for (int k = 0; k < ns && k < 16; ++k) {
    const int b = boxes[k];
    int before = 0;
    for (int v = 0; v < wave; ++v) before += wave_cnt[v][b];
    const int64_t p = w.blk_base[b * nblk + blk] + before + rank_in_wave[k];
    w.seg_pid[r * M + k] = p;
    w.plen[p] = w.seg_len[r * M + k];
    w.seg_ids[w.ray_off[r] + k] = p;
  }
}

template <int DT>
__device__ __forceinline__ void put_sample(void* sigma, void* rgb, int64_t i, float sg, float c0,
                                           float c1, float c2) {
  if (DT == kF32) {
    static_cast<float*>(sigma)[i] = sg;
    float* C = static_cast<float*>(rgb) + 3 * i;
    C[0] = c0; C[1] = c1; C[2] = c2;
  } else {
    static_cast<uint16_t*>(sigma)[i] = from_f32<sig_dt(DT)>(sg);
    uint16_t* C = static_cast<uint16_t*>(rgb) + 3 * i;
    C[0] = from_f32<rgb_dt(DT)>(c0); C[1] = from_f32<rgb_dt(DT)>(c1); C[2] = from_f32<rgb_dt(DT)>(c2);
  }
}

// Samples are written in aligned groups of kGroup packed slots, so a group that
// lies inside one segment is a handful of 16-byte stores instead of six
// scattered scalar stores per sample (each lane writes its own ray's samples,
// so lanes never share a store).
constexpr int kGroup = 8;

template <int DT>
__device__ __forceinline__ void store_group(void* sigma, void* rgb, float* t_start, float* t_end,
                                            int64_t g0, const float (&sg)[kGroup],
                                            const float (&c)[3 * kGroup], const float (&a)[kGroup],
                                            const float (&b)[kGroup]) {
  if (DT == kF32) {
    float4* S = reinterpret_cast<float4*>(static_cast<float*>(sigma) + g0);
    float4* C = reinterpret_cast<float4*>(static_cast<float*>(rgb) + 3 * g0);
#pragma unroll
    for (int q = 0; q < kGroup / 4; ++q)
      S[q] = make_float4(sg[4 * q], sg[4 * q + 1], sg[4 * q + 2], sg[4 * q + 3]);
#pragma unroll
    for (int q = 0; q < 3 * kGroup / 4; ++q)
      C[q] = make_float4(c[4 * q], c[4 * q + 1], c[4 * q + 2], c[4 * q + 3]);
  } else {
    uint4* S = reinterpret_cast<uint4*>(static_cast<uint16_t*>(sigma) + g0);
    uint4* C = reinterpret_cast<uint4*>(static_cast<uint16_t*>(rgb) + 3 * g0);
    *S = make_uint4(pack2<sig_dt(DT)>(sg[0], sg[1]), pack2<sig_dt(DT)>(sg[2], sg[3]),
                    pack2<sig_dt(DT)>(sg[4], sg[5]), pack2<sig_dt(DT)>(sg[6], sg[7]));
#pragma unroll
    for (int q = 0; q < 3; ++q)
      C[q] = make_uint4(pack2<rgb_dt(DT)>(c[8 * q], c[8 * q + 1]),
                        pack2<rgb_dt(DT)>(c[8 * q + 2], c[8 * q + 3]),
                        pack2<rgb_dt(DT)>(c[8 * q + 4], c[8 * q + 5]),
                        pack2<rgb_dt(DT)>(c[8 * q + 6], c[8 * q + 7]));
  }
  float4* A = reinterpret_cast<float4*>(t_start + g0);
  float4* B = reinterpret_cast<float4*>(t_end + g0);
#pragma unroll
  for (int q = 0; q < kGroup / 4; ++q) {
    A[q] = make_float4(a[4 * q], a[4 * q + 1], a[4 * q + 2], a[4 * q + 3]);
    B[q] = make_float4(b[4 * q], b[4 * q + 1], b[4 * q + 2], b[4 * q + 3]);
  }
}

// One thread per compact chunk: chunk c of ray r is samples [c kChunk,
// (c + 1) kChunk) along the ray, and the chunks of all rays are numbered ray
// after ray, so every thread below the total has a full chunk of work (but a
// ray's last) and the threads above it leave at once.
template <int DT>
__global__ void gen_fill_kernel(GenDev g, GenWs w, void* __restrict__ sigma, void* __restrict__ rgb,
                                float* __restrict__ t_start, float* __restrict__ t_end) {
  const int64_t ci = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (ci >= w.chunk_base[g.n_rays]) return;
  const int64_t r = w.chunk_ray[ci];
  const int c = static_cast<int>(ci - w.chunk_base[r]);
  const uint64_t key = mix64(g.seedkey + static_cast<uint64_t>(g.ray0 + r) * kGamma);
  const uint64_t span = static_cast<uint64_t>(g.n_max - g.n_min + 1);
  const int count = g.n_min + static_cast<int32_t>(((draw(key, 3) >> 32) * span) >> 32);
  const int i_begin = c * kChunk;
  if (i_begin >= count) return;
  const int i_end = i_begin + kChunk < count ? i_begin + kChunk : count;
  const double scale = w.scale[r];
  double run = w.chunk_run[r * g.chunks + c];
  const int M = g.max_segs;
  const int ns = w.nseg[r];
  // the segment holding sample i_begin, and the sample index its run starts at
  int k = 0, first = 0;
  while (k + 1 < ns && first + w.seg_len[r * M + k] <= i_begin) {
    first += w.seg_len[r * M + k];
    ++k;
  }
  // One loop over the aligned groups of packed slots of every segment the
  // chunk touches (the segment changes inside the loop): lanes whose chunks
  // cross segment boundaries at different samples then take as many passes
  // as their own groups, not the sum over segments of the longest lane's.
  int i = i_begin;
  int len = w.seg_len[r * M + k];
  int64_t d0 = w.seg_off[w.seg_pid[r * M + k]] + (i - first);  // first slot to write
  int64_t d1 = d0 + ((i_end < first + len ? i_end : first + len) - i);
  int64_t g0 = d0 & ~static_cast<int64_t>(kGroup - 1);
  while (i < i_end) {
    float sg[kGroup], cl[3 * kGroup], a[kGroup], b[kGroup];
#pragma unroll
    for (int q = 0; q < kGroup; ++q) {
      sg[q] = 0.f; cl[3 * q] = cl[3 * q + 1] = cl[3 * q + 2] = 0.f; a[q] = b[q] = 0.f;
      const int64_t p = g0 + q;
      if (p < d0 || p >= d1) continue;
      const double t0 = run;
      run = d_add(run, d_mul(width_of(g, key, i), scale));
      const uint64_t base = kRaySlots + static_cast<uint64_t>(kSampleStride) * i;
      const uint64_t v1 = draw(key, base), v2 = draw(key, base + 1);
      // 20- and 16-bit fields are exact in float32, so they are formed there
      // (the same values as the float64 field() rounded to float32)
      const float u1 = f_mul(static_cast<float>(static_cast<uint32_t>((v1 >> 20) & 0xFFFFFu) + 1u), 0x1p-20f);
      const float u2 = f_mul(static_cast<float>(static_cast<uint32_t>(v1 & 0xFFFFFu)), 0x1p-20f);
      const float z = f_mul(f_sqrt(f_mul(-2.f, log_f32(u1))), cos2pi_f32(u2));
      const float v = exp_f32(f_add(g.mu, f_mul(g.sg, z)));
      sg[q] = field(v2, 48, 16) < g.zero_frac ? 0.f : v;
      cl[3 * q] = f_mul(static_cast<float>(static_cast<uint32_t>((v2 >> 32) & 0xFFFFu)), 0x1p-16f);
      cl[3 * q + 1] = f_mul(static_cast<float>(static_cast<uint32_t>((v2 >> 16) & 0xFFFFu)), 0x1p-16f);
      cl[3 * q + 2] = f_mul(static_cast<float>(static_cast<uint32_t>(v2 & 0xFFFFu)), 0x1p-16f);
      a[q] = static_cast<float>(t0);
      b[q] = static_cast<float>(run);
      ++i;
    }
    if (g0 >= d0 && g0 + kGroup <= d1) {
      store_group<DT>(sigma, rgb, t_start, t_end, g0, sg, cl, a, b);
    } else {
#pragma unroll
      for (int q = 0; q < kGroup; ++q) {
        const int64_t p = g0 + q;
        if (p < d0 || p >= d1) continue;
        put_sample<DT>(sigma, rgb, p, sg[q], cl[3 * q], cl[3 * q + 1], cl[3 * q + 2]);
        t_start[p] = a[q];
        t_end[p] = b[q];
      }
    }
    g0 += kGroup;
    if (g0 >= d1 && i < i_end) {  // this segment's part of the chunk is written: the next one
      first += len;
      ++k;
      len = w.seg_len[r * M + k];
      d0 = w.seg_off[w.seg_pid[r * M + k]];
      d1 = d0 + ((i_end < first + len ? i_end : first + len) - i);
      g0 = d0 & ~static_cast<int64_t>(kGroup - 1);
    }
  }
}

// ---------------------------------------------------------------- scan
// Exclusive scan of int64 with out[n] = total.  Blocks of 1024 elements, block
// totals scanned recursively (scratch: ceil(n/1024) + ceil(n/1024^2) + ...).
constexpr int kScanBlock = 1024;

// With a single block (sums == nullptr) the block also writes the total to out[n].
__global__ __launch_bounds__(kScanBlock) void scan_block_kernel(const int64_t* __restrict__ in,
                                                                int64_t* __restrict__ out, int64_t n,
                                                                int64_t* __restrict__ sums) {
  __shared__ int64_t wsum[kScanBlock / kWave];
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kScanBlock + threadIdx.x;
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int64_t x = i < n ? in[i] : 0;
  int64_t v = x;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int64_t y = __shfl_up(v, d);
    if (lane >= d) v += y;
  }
  if (lane == kWave - 1) wsum[wave] = v;
  __syncthreads();
  if (wave == 0) {
    int64_t s = lane < kScanBlock / kWave ? wsum[lane] : 0;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      const int64_t y = __shfl_up(s, d);
      if (lane >= d) s += y;
    }
    if (lane < kScanBlock / kWave) wsum[lane] = s;
  }
  __syncthreads();
  const int64_t before = wave > 0 ? wsum[wave - 1] : 0;
  if (i < n) out[i] = before + v - x;
  if (threadIdx.x == kScanBlock - 1) {
    if (sums) sums[blockIdx.x] = wsum[kScanBlock / kWave - 1];
    else out[n] = wsum[kScanBlock / kWave - 1];
  }
}

// Adds the scanned block totals; offs has nb + 1 entries, offs[nb] = total.
__global__ void scan_add_kernel(int64_t* __restrict__ out, int64_t n, const int64_t* __restrict__ offs) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kScanBlock + threadIdx.x;
  if (i < n) out[i] += offs[blockIdx.x];
  if (i == 0) out[n] = offs[gridDim.x];
}

__global__ void scan_total_kernel(int64_t* __restrict__ out, int64_t n, const int64_t* __restrict__ in) {
  out[n] = n > 0 ? out[n - 1] + in[n - 1] : 0;
}

// Elements of tmp that scan_exclusive(in, out, n, tmp) writes: a level with
// nb > 1 blocks keeps nb block sums and their nb + 1 scanned offsets, then
// scans the sums with the space after them; one block writes one sum.
size_t scan_tmp_elems(int64_t n) {
  if (n <= 0) return 0;
  const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  if (nb == 1) return 1;
  return static_cast<size_t>(2 * nb + 1) + scan_tmp_elems(nb);
}

// out has n + 1 entries; tmp has scan_tmp_elems(n) entries.
hipError_t scan_exclusive(const int64_t* in, int64_t* out, int64_t n, int64_t* tmp, size_t tmp_elems,
                          hipStream_t st) {
  if (scan_tmp_elems(n) > tmp_elems) return hipErrorInvalidValue;
  if (n <= 0) {
    hipLaunchKernelGGL(scan_total_kernel, dim3(1), dim3(1), 0, st, out, static_cast<int64_t>(0), in);
    return hipGetLastError();
  }
  const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  int64_t* sums = tmp;
  int64_t* offs = tmp + nb;
  hipLaunchKernelGGL(scan_block_kernel, dim3(static_cast<unsigned>(nb)), dim3(kScanBlock), 0, st, in,
                     out, n, nb > 1 ? sums : nullptr);
  if (nb > 1) {
    hipError_t e = scan_exclusive(sums, offs, nb, offs + nb + 1, tmp_elems - (2 * nb + 1), st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scan_add_kernel, dim3(static_cast<unsigned>(nb)), dim3(kScanBlock), 0, st,
                       out, n, offs);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- host side
struct GenLayout {
  int64_t R, M, K, nblk, RM, C;
  size_t scan_elems;  // scan scratch, enough for the longest of the three scans
  size_t off[19];
  size_t bytes;
};

static GenLayout layout(const xl_gen_params* p) {
  GenLayout L;
  L.R = p->n_rays;
  L.M = p->grid[0] + p->grid[1] + p->grid[2] - 2;
  if (L.M < 1) L.M = 1;
  L.K = static_cast<int64_t>(p->grid[0]) * p->grid[1] * p->grid[2];
  L.C = (static_cast<int64_t>(p->n_max) + kChunk - 1) / kChunk;
  if (L.C < 1) L.C = 1;
  L.nblk = (L.R + kRayBlock - 1) / kRayBlock;
  L.RM = L.R * L.M;
  const int64_t KB = L.K * L.nblk;
  const int64_t longest = L.RM > KB ? (L.RM > L.R ? L.RM : L.R) : (KB > L.R ? KB : L.R);
  L.scan_elems = scan_tmp_elems(longest);
  const size_t sizes[] = {
      sizeof(int32_t) * L.R,           // nseg
      sizeof(int32_t) * L.RM,          // seg_box
      sizeof(int32_t) * L.RM,          // seg_len
      sizeof(int64_t) * L.RM,          // seg_pid
      sizeof(double) * L.R,            // scale
      sizeof(double) * L.R,            // s0
      sizeof(int64_t) * L.R,           // nseg64
      sizeof(int64_t) * (L.R + 1),     // ray_off
      sizeof(int64_t) * KB,            // blk_cnt
      sizeof(int64_t) * (KB + 1),      // blk_base
      sizeof(int64_t) * L.RM,          // plen
      sizeof(int64_t) * (L.RM + 1),    // seg_off
      sizeof(int64_t) * L.RM,          // seg_ids
      sizeof(int64_t) * L.scan_elems,  // scan_tmp
      sizeof(int32_t) * 4,             // err
      sizeof(double) * L.R * L.C,      // chunk_run
      sizeof(int64_t) * L.R,           // nchunk
      sizeof(int64_t) * (L.R + 1),     // chunk_base
      sizeof(int32_t) * L.R * L.C,     // chunk_ray
  };
  size_t o = 0;
  for (int i = 0; i < 19; ++i) {
    L.off[i] = o;
    o += (sizes[i] + 255) & ~static_cast<size_t>(255);
  }
  L.bytes = o;
  return L;
}

static GenWs views(const GenLayout& L, void* ws) {
  char* b = static_cast<char*>(ws);
  GenWs w;
  w.nseg = reinterpret_cast<int32_t*>(b + L.off[0]);
  w.seg_box = reinterpret_cast<int32_t*>(b + L.off[1]);
  w.seg_len = reinterpret_cast<int32_t*>(b + L.off[2]);
  w.seg_pid = reinterpret_cast<int64_t*>(b + L.off[3]);
  w.scale = reinterpret_cast<double*>(b + L.off[4]);
  w.s0 = reinterpret_cast<double*>(b + L.off[5]);
  w.nseg64 = reinterpret_cast<int64_t*>(b + L.off[6]);
  w.ray_off = reinterpret_cast<int64_t*>(b + L.off[7]);
  w.blk_cnt = reinterpret_cast<int64_t*>(b + L.off[8]);
  w.blk_base = reinterpret_cast<int64_t*>(b + L.off[9]);
  w.plen = reinterpret_cast<int64_t*>(b + L.off[10]);
  w.seg_off = reinterpret_cast<int64_t*>(b + L.off[11]);
  w.seg_ids = reinterpret_cast<int64_t*>(b + L.off[12]);
  w.scan_tmp = reinterpret_cast<int64_t*>(b + L.off[13]);
  w.err = reinterpret_cast<int32_t*>(b + L.off[14]);
  w.chunk_run = reinterpret_cast<double*>(b + L.off[15]);
  w.nchunk = reinterpret_cast<int64_t*>(b + L.off[16]);
  w.chunk_base = reinterpret_cast<int64_t*>(b + L.off[17]);
  w.chunk_ray = reinterpret_cast<int32_t*>(b + L.off[18]);
  return w;
}

static GenDev dev_params(const xl_gen_params* p, const GenLayout& L) {
  GenDev g;
  g.n_rays = p->n_rays;
  g.ray0 = p->ray0;
  g.n_min = p->n_min;
  g.n_max = p->n_max;
  g.gx = p->grid[0];
  g.gy = p->grid[1];
  g.gz = p->grid[2];
  g.max_segs = static_cast<int32_t>(L.M);
  g.chunks = static_cast<int32_t>(L.C);
  g.wm = static_cast<float>(p->width_mean);
  g.mu = static_cast<float>(p->sigma_mu);
  g.sg = static_cast<float>(p->sigma_s);
  g.zero_frac = p->zero_frac;
  g.t_far = p->t_far;
  g.seedkey = mix64(p->seed);
  return g;
}

size_t gen_workspace_bytes(const xl_gen_params* p) { return layout(p).bytes; }

int64_t gen_max_segments(const xl_gen_params* p) { return layout(p).RM; }

static inline unsigned blocks(int64_t n, int b) { return static_cast<unsigned>((n + b - 1) / b); }

hipError_t gen_plan(const xl_gen_params* p, void* ws, hipStream_t st, int64_t* n_samples,
                    int64_t* n_seg, int* overflow, int64_t* pinned) {
  // The three values read back go through `pinned` (page-locked host memory,
  // >= 3 int64) when given, so the copies are plain stream work.
  int64_t local[3];
  int64_t* h = pinned ? pinned : local;
  const GenLayout L = layout(p);
  const GenWs w = views(L, ws);
  const GenDev g = dev_params(p, L);
  hipError_t e = hipMemsetAsync(w.err, 0, sizeof(int32_t), st);
  if (e != hipSuccess) return e;
  const bool any = L.R > 0;  // (an empty grid is not a valid launch)
  if (any) {
    hipLaunchKernelGGL(gen_struct_kernel, dim3(blocks(L.R, kStructRays)), dim3(kStructBlock), 0, st, g, w);
    hipLaunchKernelGGL(block_hist_kernel, dim3(static_cast<unsigned>(L.nblk)), dim3(kRayBlock), 0, st,
                       g, w, L.nblk, static_cast<int>(L.K));
  }
  if ((e = scan_exclusive(w.nseg64, w.ray_off, L.R, w.scan_tmp, L.scan_elems, st)) != hipSuccess) return e;
  if ((e = scan_exclusive(w.nchunk, w.chunk_base, L.R, w.scan_tmp, L.scan_elems, st)) != hipSuccess) return e;
  if (any) hipLaunchKernelGGL(chunk_map_kernel, dim3(blocks(L.R, 128)), dim3(128), 0, st, g, w);
  if ((e = scan_exclusive(w.blk_cnt, w.blk_base, L.K * L.nblk, w.scan_tmp, L.scan_elems, st)) != hipSuccess) return e;
  if (any)
    hipLaunchKernelGGL(gen_rank_kernel, dim3(static_cast<unsigned>(L.nblk)), dim3(kRayBlock), 0, st, g,
                       w, L.nblk, static_cast<int>(L.K));
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(&h[0], w.ray_off + L.R, sizeof(int64_t), hipMemcpyDeviceToHost, st)) != hipSuccess)
    return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  const int64_t ns = h[0];
  if (ns < 0 || ns > L.RM) return hipErrorInvalidValue;  // at most max_segs per ray
  if ((e = scan_exclusive(w.plen, w.seg_off, ns, w.scan_tmp, L.scan_elems, st)) != hipSuccess) return e;
  h[2] = 0;
  if ((e = hipMemcpyAsync(&h[1], w.seg_off + ns, sizeof(int64_t), hipMemcpyDeviceToHost, st)) != hipSuccess)
    return e;
  if ((e = hipMemcpyAsync(&h[2], w.err, sizeof(int32_t), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  *n_samples = h[1];
  *n_seg = ns;
  *overflow = static_cast<int32_t>(h[2]) != 0;
  return hipSuccess;
}

__global__ void fill_zero_i64_kernel(int64_t* __restrict__ p, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// First segment of every region (box-major block bases of block 0), and n_seg.
__global__ void region_offsets_kernel(const int64_t* __restrict__ blk_base, int64_t nblk, int K,
                                      int64_t* __restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b <= K) out[b] = blk_base[b * nblk];
}

hipError_t gen_fill(const xl_gen_params* p, int dtype, void* ws, int64_t n_seg, void* sigma, void* rgb,
                    float* t_start, float* t_end, int64_t* seg_offsets, int64_t* ray_offsets,
                    int64_t* seg_ids, int64_t* region_offsets, hipStream_t st) {
  const GenLayout L = layout(p);
  const GenWs w = views(L, ws);
  const GenDev g = dev_params(p, L);
  const dim3 grid(blocks(L.R * L.C, 128));  // at least the compact chunk count
  if (L.R > 0) switch (dtype) {
    case kF32:
      hipLaunchKernelGGL(gen_fill_kernel<kF32>, grid, dim3(128), 0, st, g, w, sigma, rgb, t_start, t_end);
      break;
    case kBF16:
      hipLaunchKernelGGL(gen_fill_kernel<kBF16>, grid, dim3(128), 0, st, g, w, sigma, rgb, t_start, t_end);
      break;
    case kBF16F16:
      hipLaunchKernelGGL(gen_fill_kernel<kBF16F16>, grid, dim3(128), 0, st, g, w, sigma, rgb, t_start,
                         t_end);
      break;
    default:
      hipLaunchKernelGGL(gen_fill_kernel<kF16>, grid, dim3(128), 0, st, g, w, sigma, rgb, t_start, t_end);
      break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (seg_offsets && (e = hipMemcpyAsync(seg_offsets, w.seg_off, sizeof(int64_t) * (n_seg + 1),
                                         hipMemcpyDeviceToDevice, st)) != hipSuccess)
    return e;
  if (ray_offsets && (e = hipMemcpyAsync(ray_offsets, w.ray_off, sizeof(int64_t) * (L.R + 1),
                                         hipMemcpyDeviceToDevice, st)) != hipSuccess)
    return e;
  if (seg_ids && (e = hipMemcpyAsync(seg_ids, w.seg_ids, sizeof(int64_t) * n_seg,
                                     hipMemcpyDeviceToDevice, st)) != hipSuccess)
    return e;
  if (region_offsets) {
    if (L.nblk > 0) {
      hipLaunchKernelGGL(region_offsets_kernel, dim3(blocks(L.K + 1, 256)), dim3(256), 0, st,
                         w.blk_base, L.nblk, static_cast<int>(L.K), region_offsets);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    } else {
      // no rays: every region is empty (a small fill kernel, no memset node)
      hipLaunchKernelGGL(fill_zero_i64_kernel, dim3(blocks(L.K + 1, 256)), dim3(256), 0, st,
                         region_offsets, L.K + 1);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

}  // namespace xl
