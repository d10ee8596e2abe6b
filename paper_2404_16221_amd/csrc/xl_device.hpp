// Device-side building blocks of the partitioned renderer (gfx950, wave64).
//
// A "range" is the partial tuple of a contiguous run of one segment's
// samples.  Ranges combine front to back with the associative operator of
// Eq. 3-8 (Sec. 4.3): colour, opacity and depth of the later range are
// weighted by the earlier range's transmittance, and the distortion loss gains
// the cross term of Eq. 7/8.  The cross term is evaluated in a form where every
// added quantity is non-negative: with F = sum w (m - m0) (depth measured from
// the range's first midpoint m0) and B = sum w (m1 - m) (measured back from its
// last midpoint m1),
//   sum_{i in y, j in x} w_i w_j (m_i - m_j) = A_x F_y + A_x A_y (m0_y - m1_x) + A_y B_x,
// which equals D_y A_x - A_y D_x of Eq. 8 without its cancellation.
#pragma once

#include <type_traits>

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/xl.h"

namespace xl {

constexpr int kWave = 64;                 // CDNA wavefront
constexpr int kRun = 8;                   // consecutive samples per lane
constexpr int kTile = kWave * kRun;       // samples per wave tile
constexpr int kWavesPerBlock = 4;
constexpr int kBlock = kWave * kWavesPerBlock;

// Segment tuples, and their gradients, are records of kTupStride floats, one
// per segment: tau, r, g, b, A, D, L and a pad that is written as zero.  A
// record is 32 bytes (the arrays are 32-byte aligned), so a tuple is two
// 16-byte accesses and the records of consecutive segments are one stream.
constexpr int kTupStride = XL_TUPLE_STRIDE;

struct Tup7 {
  float v[7];
};
__device__ __forceinline__ Tup7 load_tup7(const float* __restrict__ p, int64_t s) {
  const float4* q = reinterpret_cast<const float4*>(p + kTupStride * s);
  const float4 a = q[0], b = q[1];
  return Tup7{{a.x, a.y, a.z, a.w, b.x, b.y, b.z}};
}
__device__ __forceinline__ void store_tup7(float* __restrict__ p, int64_t s, float tau, float cr,
                                           float cg, float cb, float A, float D, float L) {
  float4* q = reinterpret_cast<float4*>(p + kTupStride * s);
  q[0] = make_float4(tau, cr, cg, cb);
  q[1] = make_float4(A, D, L, 0.f);
}

enum Dtype : int { kF32 = 0, kBF16 = 1, kF16 = 2, kBF16F16 = 3 };
// Storage type of the densities and of the colours (and of their gradients):
// kBF16F16 keeps densities in bfloat16 and colours in float16.
constexpr int sig_dt(int dt) { return dt == kBF16F16 ? kBF16 : dt; }
constexpr int rgb_dt(int dt) { return dt == kBF16F16 ? kF16 : dt; }

struct Range {
  float tau;        // sum of optical depths sigma * delta; transmittance is exp(-tau)
  float cr, cg, cb; // colour
  float A;          // opacity (sum of weights)
  float F;          // sum w (m - m0)
  float B;          // sum w (m1 - m)
  float L;          // distortion loss inside the range
  float m0, m1;     // first and last sample midpoints
};

constexpr int kStartHead = 1;  // first sample starts a segment
constexpr int kHasEnd = 2;     // some segment ends inside the tile
constexpr int kHasHead = 4;    // some segment starts inside the tile
constexpr int kTailOpen = 8;   // the last sample's segment continues past the tile

__device__ __forceinline__ Range range_identity() {
  Range r;
  r.tau = 0.f; r.cr = r.cg = r.cb = 0.f; r.A = 0.f;
  r.F = 0.f; r.B = 0.f; r.L = 0.f; r.m0 = 0.f; r.m1 = 0.f;
  return r;
}

__device__ __forceinline__ float exp_neg(float tau) {
  return __builtin_amdgcn_exp2f(-1.4426950408889634f * tau);
}

// Error-free transformation of a sum (Knuth's TwoSum): a + b = s + e exactly,
// for any ordering of magnitudes.  Optical depths are summed in two levels.
// Inside a tile the sum is plain: serial over a lane's kRun samples, then a
// tree of log2(kWave) levels in the wave scan, so a tile's partial depth has
// at most kRun - 1 + 6 roundings on any path.  Across tiles (the fixup) and
// across segments (the merge), where the number of joins grows with the
// length of a segment or ray, partial depths are joined as pairs (tau, tlo)
// that keep the rounding error of every join in tlo.  A segment's
// log-transmittance therefore has a relative error bounded independently of
// how many samples and tiles it spans.
__device__ __forceinline__ float two_sum(float a, float b, float& e) {
  const float s = a + b;
  const float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
  return s;
}
__device__ __forceinline__ void add_tau(float& tau, float& tlo, float hi, float lo) {
  float e;
  tau = two_sum(tau, hi, e);
  tlo += e + lo;
}

// Every field but the optical depth, x then y, where T1 is x's transmittance.
__device__ __forceinline__ void combine_rest(Range& r, const Range& x, const Range& y, float T1) {
  r.cr = fmaf(T1, y.cr, x.cr);
  r.cg = fmaf(T1, y.cg, x.cg);
  r.cb = fmaf(T1, y.cb, x.cb);
  r.A = fmaf(T1, y.A, x.A);
  r.F = fmaf(T1, fmaf(y.A, y.m0 - x.m0, y.F), x.F);
  r.B = fmaf(T1, y.B, fmaf(x.A, y.m1 - x.m1, x.B));
  const float cross = fmaf(x.A, fmaf(y.A, y.m0 - x.m1, y.F), y.A * x.B);
  r.L = fmaf(T1 * T1, y.L, fmaf(2.f * T1, cross, x.L));
  r.m0 = x.m0;
  r.m1 = y.m1;
}

// x then y (x in front), inside a tile.  Transmittance across lanes is taken
// as exp(-sum tau), one rounding, never as a running product of per-sample
// factors (whose roundings would add up).
__device__ __forceinline__ Range combine(const Range& x, const Range& y) {
  Range r;
  r.tau = x.tau + y.tau;
  combine_rest(r, x, y, exp_neg(x.tau));
  return r;
}

// A range kept across tiles: its optical depth is the compensated pair
// r.tau + tlo.
struct Part {
  Range r;
  float tlo;
};
__device__ __forceinline__ Part part_of(const Range& r) { return Part{r, 0.f}; }
// The in-tile form (the pair rounded to one float).
__device__ __forceinline__ Range range_of(const Part& p) {
  Range r = p.r;
  r.tau = p.r.tau + p.tlo;
  return r;
}
__device__ __forceinline__ Part combine(const Part& x, const Part& y) {
  Part p;
  p.r.tau = x.r.tau;
  p.tlo = x.tlo;
  add_tau(p.r.tau, p.tlo, y.r.tau, y.tlo);
  combine_rest(p.r, x.r, y.r, exp_neg(x.r.tau + x.tlo));
  return p;
}

// One sample, reduced to what the composite needs.
struct Smp {
  float tau, e, alpha, m, delta, c0, c1, c2;  // e = exp(-tau)
};

// 1 - exp(-tau) without cancellation: for tau < 1/4, tau times a degree-4
// polynomial fitted to (1 - exp(-tau)) / tau on [0, 1/4] (relative error of
// the fit 2.5e-9; evaluated in float32 with fused multiply-adds the result is
// within 9.6e-8 relative of the exact value), else 1 - exp(-tau), where the
// subtraction is exact and only e's rounding remains.
__device__ __forceinline__ float one_minus_exp_neg(float tau, float e) {
  float q = fmaf(0.0075102211f, tau, -0.041488953f);
  q = fmaf(q, tau, 0.16665082f);
  q = fmaf(q, tau, -0.49999949f);
  q = fmaf(q, tau, 1.f);
  return tau < 0.25f ? tau * q : 1.f - e;
}

__device__ __forceinline__ Smp make_sample(float sigma, float c0, float c1, float c2, float t0,
                                           float t1) {
  Smp s;
  s.delta = t1 - t0;
  s.m = 0.5f * (t0 + t1);
  s.tau = sigma * s.delta;
  s.e = exp_neg(s.tau);
  s.alpha = one_minus_exp_neg(s.tau, s.e);
  s.c0 = c0; s.c1 = c1; s.c2 = c2;
  return s;
}

// Restart r as the empty range at midpoint m when `head` (a segment starts at
// the next sample appended); Tr is the range's transmittance.
__device__ __forceinline__ void restart_if(bool head, Range& r, float& Tr, float m) {
  r.tau = head ? 0.f : r.tau;
  r.cr = head ? 0.f : r.cr; r.cg = head ? 0.f : r.cg; r.cb = head ? 0.f : r.cb;
  r.A = head ? 0.f : r.A;
  r.F = head ? 0.f : r.F;
  r.B = head ? 0.f : r.B;
  r.L = head ? 0.f : r.L;
  r.m0 = head ? m : r.m0;
  Tr = head ? 1.f : Tr;
}

// Append one sample behind range r whose transmittance is Tr (updated).
// Inside one lane Tr is a product of at most kRun per-sample factors, so its
// rounding error stays bounded; across lanes and tiles transmittance is always
// exp(-tau) (see combine).
__device__ __forceinline__ void append(Range& r, float& Tr, const Smp& s) {
  const float w = Tr * s.alpha;
  const float Z = fmaf(r.A, s.m - r.m1, r.B);  // sum_{j<i} w_j (m_i - m_j)
  r.L = fmaf(w, fmaf(2.f, Z, w * s.delta * (1.f / 3.f)), r.L);
  r.F = fmaf(w, s.m - r.m0, r.F);
  r.B = Z;
  r.cr = fmaf(w, s.c0, r.cr);
  r.cg = fmaf(w, s.c1, r.cg);
  r.cb = fmaf(w, s.c2, r.cb);
  r.A += w;
  r.tau += s.tau;  // at most kRun terms (see two_sum)
  r.m1 = s.m;
  Tr *= s.e;
}

// Orders the calling wave's LDS accesses for the compiler; the hardware
// already performs one wave's LDS operations in order.
// A 16-byte store marked non-temporal (streaming: written once, not re-read
// by this kernel).
__device__ __forceinline__ void store_stream(uint4* p, uint4 v) {
  typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
  __builtin_nontemporal_store(u32x4{v.x, v.y, v.z, v.w}, reinterpret_cast<u32x4*>(p));
}

__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// ---------------------------------------------------------------- storage
__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
  return __uint_as_float(static_cast<uint32_t>(h) << 16);
}
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
// Round to nearest even (gfx950 converts two values per instruction).
__device__ __forceinline__ uint16_t f32_to_bf16(float x) {
  return __builtin_bit_cast(uint16_t, static_cast<__bf16>(x));
}
__device__ __forceinline__ float f16_to_f32(uint16_t h) {
  return static_cast<float>(__builtin_bit_cast(_Float16, h));
}
__device__ __forceinline__ uint16_t f32_to_f16(float x) {
  return __builtin_bit_cast(uint16_t, static_cast<_Float16>(x));
}

template <int DT>
__device__ __forceinline__ float to_f32(uint16_t h) {
  return DT == kBF16 ? bf16_to_f32(h) : f16_to_f32(h);
}
template <int DT>
__device__ __forceinline__ uint16_t from_f32(float x) {
  return DT == kBF16 ? f32_to_bf16(x) : f32_to_f16(x);
}
// Two values rounded to nearest even and packed (first in the low half).
template <int DT>
__device__ __forceinline__ uint32_t pack2(float a, float b) {
  const f32x2 v = {a, b};
  if (DT == kBF16) return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, f16x2));
}

// The raw storage of kRun consecutive samples (i % kRun == 0, all present),
// loaded as 16-byte vectors and decoded later: a tile issues these loads
// before its setup so their latency overlaps it.
template <int DT>
struct RawRun {
  static constexpr int kSigmaVec = DT == kF32 ? kRun / 4 : kRun / 8;
  static constexpr int kRgbVec = 3 * kSigmaVec;
  uint4 sg[kSigmaVec];
  uint4 rgb[kRgbVec];
  float4 t0[kRun / 4], t1[kRun / 4];

  __device__ __forceinline__ void load(const void* __restrict__ sigma_p, const void* __restrict__ rgb_p,
                                       const float* __restrict__ t0_p, const float* __restrict__ t1_p,
                                       int64_t i) {
    const int es = DT == kF32 ? 4 : 2;
    const uint4* S = reinterpret_cast<const uint4*>(static_cast<const char*>(sigma_p) + es * i);
    const uint4* C = reinterpret_cast<const uint4*>(static_cast<const char*>(rgb_p) + 3 * es * i);
#pragma unroll
    for (int q = 0; q < kSigmaVec; ++q) sg[q] = S[q];
#pragma unroll
    for (int q = 0; q < kRgbVec; ++q) rgb[q] = C[q];
#pragma unroll
    for (int q = 0; q < kRun / 4; ++q) {
      t0[q] = reinterpret_cast<const float4*>(t0_p + i)[q];
      t1[q] = reinterpret_cast<const float4*>(t1_p + i)[q];
    }
  }

  // The first cnt (0 <= cnt <= kRun) of the lane's samples by element loads,
  // zeros for the rest: for the ragged last tile, whose vector loads would
  // read past the arrays.  A zero sample is finite (as the scans' masked joins
  // need) and adds nothing.
  __device__ __forceinline__ void load_part(const void* __restrict__ sigma_p,
                                            const void* __restrict__ rgb_p,
                                            const float* __restrict__ t0_p,
                                            const float* __restrict__ t1_p, int64_t i, int cnt) {
    uint32_t sw[4 * kSigmaVec], cw[4 * kRgbVec];
    if constexpr (DT == kF32) {
      const uint32_t* S = static_cast<const uint32_t*>(sigma_p) + i;
      const uint32_t* C = static_cast<const uint32_t*>(rgb_p) + 3 * i;
#pragma unroll
      for (int k = 0; k < kRun; ++k) sw[k] = k < cnt ? S[k] : 0u;
#pragma unroll
      for (int k = 0; k < 3 * kRun; ++k) cw[k] = k < 3 * cnt ? C[k] : 0u;
    } else {
      const uint16_t* S = static_cast<const uint16_t*>(sigma_p) + i;
      const uint16_t* C = static_cast<const uint16_t*>(rgb_p) + 3 * i;
#pragma unroll
      for (int k = 0; k < kRun / 2; ++k)
        sw[k] = (2 * k < cnt ? S[2 * k] : 0u) | (2 * k + 1 < cnt ? uint32_t(S[2 * k + 1]) << 16 : 0u);
#pragma unroll
      for (int k = 0; k < 3 * kRun / 2; ++k)
        cw[k] = (2 * k < 3 * cnt ? C[2 * k] : 0u) |
                (2 * k + 1 < 3 * cnt ? uint32_t(C[2 * k + 1]) << 16 : 0u);
    }
#pragma unroll
    for (int q = 0; q < kSigmaVec; ++q) sg[q] = make_uint4(sw[4 * q], sw[4 * q + 1], sw[4 * q + 2], sw[4 * q + 3]);
#pragma unroll
    for (int q = 0; q < kRgbVec; ++q) rgb[q] = make_uint4(cw[4 * q], cw[4 * q + 1], cw[4 * q + 2], cw[4 * q + 3]);
    float a[kRun], b[kRun];
#pragma unroll
    for (int k = 0; k < kRun; ++k) {
      a[k] = k < cnt ? t0_p[i + k] : 0.f;
      b[k] = k < cnt ? t1_p[i + k] : 0.f;
    }
#pragma unroll
    for (int q = 0; q < kRun / 4; ++q) {
      t0[q] = make_float4(a[4 * q], a[4 * q + 1], a[4 * q + 2], a[4 * q + 3]);
      t1[q] = make_float4(b[4 * q], b[4 * q + 1], b[4 * q + 2], b[4 * q + 3]);
    }
  }

  __device__ __forceinline__ void decode(float (&sgf)[kRun], float (&c)[3 * kRun], float (&a)[kRun],
                                         float (&b)[kRun]) const {
    auto unpack = [](const uint4* v, int nvec, float* out, auto kind) {
      constexpr int K = decltype(kind)::value;
#pragma unroll
      for (int q = 0; q < nvec; ++q) {
        const uint32_t w[4] = {v[q].x, v[q].y, v[q].z, v[q].w};
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          if (K == kF32) {
            out[4 * q + h] = __uint_as_float(w[h]);
          } else {
            out[8 * q + 2 * h] = to_f32<K>(static_cast<uint16_t>(w[h] & 0xffffu));
            out[8 * q + 2 * h + 1] = to_f32<K>(static_cast<uint16_t>(w[h] >> 16));
          }
        }
      }
    };
    unpack(sg, kSigmaVec, sgf, std::integral_constant<int, sig_dt(DT)>{});
    unpack(rgb, kRgbVec, c, std::integral_constant<int, rgb_dt(DT)>{});
#pragma unroll
    for (int q = 0; q < kRun / 4; ++q) {
      a[4 * q] = t0[q].x; a[4 * q + 1] = t0[q].y; a[4 * q + 2] = t0[q].z; a[4 * q + 3] = t0[q].w;
      b[4 * q] = t1[q].x; b[4 * q + 1] = t1[q].y; b[4 * q + 2] = t1[q].z; b[4 * q + 3] = t1[q].w;
    }
  }
};

// ---------------------------------------------------------------- wave scans
// The part of a range that the backward's prefix needs: optical depth,
// opacity and the back-relative depth at the last midpoint.
struct Pre {
  float tau, A, B, m1;
};
__device__ __forceinline__ Pre pre_of(const Range& r) { return Pre{r.tau, r.A, r.B, r.m1}; }
__device__ __forceinline__ Pre pre_identity() { return Pre{0.f, 0.f, 0.f, 0.f}; }
__device__ __forceinline__ Pre combine(const Pre& x, const Pre& y) {
  const float T1 = exp_neg(x.tau);
  Pre r;
  r.tau = x.tau + y.tau;
  r.A = fmaf(T1, y.A, x.A);
  r.B = fmaf(T1, y.B, fmaf(x.A, y.m1 - x.m1, x.B));
  r.m1 = y.m1;
  return r;
}

// Field-wise maps: a lane move of a whole range, a branch-free select.
template <typename Op>
__device__ __forceinline__ Range map_fields(const Range& x, Op op) {
  Range y;
  y.tau = op(x.tau);
  y.cr = op(x.cr); y.cg = op(x.cg); y.cb = op(x.cb);
  y.A = op(x.A); y.F = op(x.F); y.B = op(x.B); y.L = op(x.L);
  y.m0 = op(x.m0); y.m1 = op(x.m1);
  return y;
}
template <typename Op>
__device__ __forceinline__ Pre map_fields(const Pre& x, Op op) {
  return Pre{op(x.tau), op(x.A), op(x.B), op(x.m1)};
}
__device__ __forceinline__ Range select(bool c, const Range& a, const Range& b) {
  Range r;
  r.tau = c ? a.tau : b.tau;
  r.cr = c ? a.cr : b.cr; r.cg = c ? a.cg : b.cg; r.cb = c ? a.cb : b.cb;
  r.A = c ? a.A : b.A; r.F = c ? a.F : b.F; r.B = c ? a.B : b.B; r.L = c ? a.L : b.L;
  r.m0 = c ? a.m0 : b.m0; r.m1 = c ? a.m1 : b.m1;
  return r;
}
__device__ __forceinline__ Pre select(bool c, const Pre& a, const Pre& b) {
  return Pre{c ? a.tau : b.tau, c ? a.A : b.A, c ? a.B : b.B, c ? a.m1 : b.m1};
}

// Lane moves.  DPP (GFX9 controls) moves a register between lanes inside the
// VALU instruction itself: row shifts stay within a row of 16 lanes, the row
// broadcasts copy lane 15 of each row into the next row and lane 31 into rows
// 2-3, and the wave shifts move every lane by one.  Moves with no DPP form
// (lane 16(r+1) into row r, lane 32 into rows 0-1) use ds_bpermute.
constexpr int kRowShl1 = 0x101, kRowShl2 = 0x102, kRowShl4 = 0x104, kRowShl8 = 0x108;
constexpr int kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114, kRowShr8 = 0x118;
constexpr int kWaveShl1 = 0x130, kWaveShr1 = 0x138;
constexpr int kRowBcast15 = 0x142, kRowBcast31 = 0x143;

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int dpp_i(int v) {
  // Lanes of disabled rows are left undefined and lanes whose source is
  // outside the row or wave read 0; the scans never use either.
  return __builtin_amdgcn_mov_dpp(v, CTRL, ROW_MASK, 0xF, true);
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_f(float v) {
  return __builtin_bit_cast(float, dpp_i<CTRL, ROW_MASK>(__builtin_bit_cast(int, v)));
}
template <int CTRL, int ROW_MASK, typename T>
__device__ __forceinline__ T dpp_fields(const T& x) {
  return map_fields(x, [](float v) { return dpp_f<CTRL, ROW_MASK>(v); });
}
template <typename T>
__device__ __forceinline__ T lane_fields(const T& x, int src) {
  return map_fields(x, [src](float v) { return __shfl(v, src); });
}

// Value of lane - 1 (lane 0: unspecified) and of lane + 1 (lane 63: unspecified).
template <typename T>
__device__ __forceinline__ T from_lower(const T& x) { return dpp_fields<kWaveShr1, 0xF>(x); }
__device__ __forceinline__ int from_lower(int v) { return dpp_i<kWaveShr1, 0xF>(v); }
template <typename T>
__device__ __forceinline__ T from_upper(const T& x) { return dpp_fields<kWaveShl1, 0xF>(x); }
__device__ __forceinline__ int from_upper(int v) { return dpp_i<kWaveShl1, 0xF>(v); }

// Masked combines.  A scan step either joins the received range y to the
// lane's own x or leaves x as it is.  Instead of computing the join and then
// selecting field by field, the choice is folded into the arithmetic: y's
// additive fields are scaled by k in {0, 1} (and, behind x, y's weight T1 is
// zeroed), which reproduces x exactly when k = 0 because every received value
// is finite (row shifts with bound_ctrl read 0 outside the row).  One select
// remains per join, for the midpoint the join would move.
//
// y in front of x (prefix scans), or x unchanged.
__device__ __forceinline__ Pre join_front(const Pre& y, const Pre& x, bool use) {
  const float k = use ? 1.f : 0.f;
  const Pre z{k * y.tau, k * y.A, k * y.B, y.m1};  // y, or a left identity of x
  return combine(z, x);
}
__device__ __forceinline__ Range join_front(const Range& y, const Range& x, bool use) {
  const float k = use ? 1.f : 0.f;
  Range z;  // y, or a left identity of x
  z.tau = k * y.tau;
  z.cr = k * y.cr; z.cg = k * y.cg; z.cb = k * y.cb;
  z.A = k * y.A; z.F = k * y.F; z.B = k * y.B; z.L = k * y.L;
  z.m0 = use ? y.m0 : x.m0;
  z.m1 = y.m1;
  return combine(z, x);
}
// y behind x (suffix scan), or x unchanged.
__device__ __forceinline__ Range join_back(const Range& x, const Range& y, bool use) {
  const float k = use ? 1.f : 0.f;
  const float T1 = use ? exp_neg(x.tau) : 0.f;
  const float m1 = use ? y.m1 : x.m1;
  Range r;
  r.tau = fmaf(k, y.tau, x.tau);
  r.cr = fmaf(T1, y.cr, x.cr);
  r.cg = fmaf(T1, y.cg, x.cg);
  r.cb = fmaf(T1, y.cb, x.cb);
  r.A = fmaf(T1, y.A, x.A);
  r.F = fmaf(T1, fmaf(y.A, y.m0 - x.m0, y.F), x.F);
  r.B = fmaf(T1, y.B, fmaf(x.A, m1 - x.m1, x.B));
  const float cross = fmaf(x.A, fmaf(y.A, y.m0 - x.m1, y.F), y.A * x.B);
  r.L = fmaf(T1 * T1, y.L, fmaf(2.f * T1, cross, x.L));
  r.m0 = x.m0;
  r.m1 = m1;
  return r;
}

// One step of the prefix scan: y is what precedes x's window; `ok` says the
// lane received one.  Row shifts use the masked join; the row broadcasts
// leave the lanes of disabled rows undefined, so they select instead.
template <int CTRL, int ROW_MASK, typename T>
__device__ __forceinline__ void up_step(T& x, bool& f, bool ok) {
  const T y = dpp_fields<CTRL, ROW_MASK>(x);
  const int fy = dpp_i<CTRL, ROW_MASK>(static_cast<int>(f));
  const bool use = ok && !f;
  if constexpr (ROW_MASK == 0xF) {
    x = join_front(y, x, use);
  } else {
    x = select(use, combine(y, x), x);
  }
  f = f || (ok && fy != 0);
}

// Inclusive segmented scan in lane order.  A lane whose flag is set starts a
// new segment: nothing from lower lanes is combined into it.  Each step is
// branch-free (combine, then select) so the wave never splits.  Rows of 16
// lanes scan by shifts of 1, 2, 4, 8; then row r takes the total of row r - 1
// (rows 1 and 3) and rows 2-3 the total of lanes 0..31.
template <typename T>
__device__ __forceinline__ void scan_up(T& x, bool& f, int lane) {
  const int r = lane & 15;
  up_step<kRowShr1, 0xF>(x, f, r >= 1);
  up_step<kRowShr2, 0xF>(x, f, r >= 2);
  up_step<kRowShr4, 0xF>(x, f, r >= 4);
  up_step<kRowShr8, 0xF>(x, f, r >= 8);
  up_step<kRowBcast15, 0xA>(x, f, (lane & 16) != 0);
  up_step<kRowBcast31, 0xC>(x, f, lane >= 32);
}

__device__ __forceinline__ void down_apply(Range& x, bool& f, int& seg, const Range& y, int fy,
                                           int sy, bool ok) {
  const bool use = ok && !f;
  x = join_back(x, y, use);
  seg = use ? sy : seg;
  f = f || (ok && fy != 0);
}
template <int CTRL>
__device__ __forceinline__ void down_step(Range& x, bool& f, int& seg, bool ok) {
  const Range y = dpp_fields<CTRL, 0xF>(x);
  const int fy = dpp_i<CTRL, 0xF>(static_cast<int>(f));
  const int sy = dpp_i<CTRL, 0xF>(seg);
  down_apply(x, f, seg, y, fy, sy, ok);
}
__device__ __forceinline__ void down_step_from(Range& x, bool& f, int& seg, int src, bool ok) {
  const Range y = lane_fields(x, src);
  const int fy = __shfl(static_cast<int>(f), src);
  const int sy = __shfl(seg, src);
  down_apply(x, f, seg, y, fy, sy, ok);
}

// Inclusive segmented scan against lane order (suffix).  A lane whose flag is
// set ends its segment: nothing from higher lanes is combined into it.  `seg`
// travels with the range (the segment whose end closes it).  Rows scan by
// shifts of 1, 2, 4, 8 toward lane 0; rows 0 and 2 then take the first lane of
// the next row, and rows 0-1 take lane 32.
__device__ __forceinline__ void scan_down(Range& x, bool& f, int& seg, int lane) {
  const int r = lane & 15;
  down_step<kRowShl1>(x, f, seg, r + 1 < 16);
  down_step<kRowShl2>(x, f, seg, r + 2 < 16);
  down_step<kRowShl4>(x, f, seg, r + 4 < 16);
  down_step<kRowShl8>(x, f, seg, r + 8 < 16);
  down_step_from(x, f, seg, (lane | 15) + 1, (lane & 16) == 0);
  down_step_from(x, f, seg, 32, lane < 32);
}

// A range parked in LDS, structure of arrays over the 64 lanes of a wave.
constexpr int kRangeFields = 10;
__device__ __forceinline__ void park_range(float* __restrict__ lds, int lane, const Range& r) {
  lds[0 * kWave + lane] = r.tau; lds[1 * kWave + lane] = r.cr; lds[2 * kWave + lane] = r.cg;
  lds[3 * kWave + lane] = r.cb; lds[4 * kWave + lane] = r.A; lds[5 * kWave + lane] = r.F;
  lds[6 * kWave + lane] = r.B; lds[7 * kWave + lane] = r.L; lds[8 * kWave + lane] = r.m0;
  lds[9 * kWave + lane] = r.m1;
}
__device__ __forceinline__ Range unpark_range(const float* __restrict__ lds, int lane) {
  Range r;
  r.tau = lds[0 * kWave + lane]; r.cr = lds[1 * kWave + lane]; r.cg = lds[2 * kWave + lane];
  r.cb = lds[3 * kWave + lane]; r.A = lds[4 * kWave + lane]; r.F = lds[5 * kWave + lane];
  r.B = lds[6 * kWave + lane]; r.L = lds[7 * kWave + lane]; r.m0 = lds[8 * kWave + lane];
  r.m1 = lds[9 * kWave + lane];
  return r;
}

// Per-tile records kept in the workspace between forward and backward.  The
// scalar fields are arrays over tiles (a thread per tile reads them
// coalesced); each partial range is one 48-byte record (three 16-byte
// vectors), so that the one lane that writes it issues three stores instead of
// one per field, and the backward reads it with two scalar loads.  The tile
// count is padded to a multiple of kRecGroup so that every array starts
// 256-byte aligned.
constexpr int64_t kRecGroup = 64;
constexpr int kPartVecs = 3;  // (tau, r, g, b), (A, F, B, L), (m0, m1, tlo, 0)
constexpr size_t kRecBytesPerTile = 8 + 4 + 4 * 16 * kPartVecs;

__host__ __device__ inline int64_t rec_stride(int64_t n_tiles) {
  const int64_t nt = n_tiles > 0 ? n_tiles : 1;
  return (nt + kRecGroup - 1) / kRecGroup * kRecGroup;
}

struct TileRecs {
  int64_t* first_seg;  // segment containing the tile's first sample (or the
                       // first segment starting at it, empty ones included)
  int32_t* flags;      // kStartHead | kHasEnd | kHasHead | kTailOpen
  float4* head;  // [stride][kPartVecs] first sample .. first segment end (whole tile if none)
  float4* tail;  // last segment head .. last sample
  float4* pre;   // carry-in: the first sample's segment before this tile
  float4* suf;   // carry-in: the last sample's segment after this tile
  int64_t stride;

  __host__ __device__ static TileRecs view(void* ws, int64_t n_tiles) {
    TileRecs r;
    r.stride = rec_stride(n_tiles);
    char* p = static_cast<char*>(ws);
    r.first_seg = reinterpret_cast<int64_t*>(p); p += 8 * r.stride;
    r.flags = reinterpret_cast<int32_t*>(p); p += 4 * r.stride;
    const int64_t rb = 16 * kPartVecs * r.stride;
    r.head = reinterpret_cast<float4*>(p); p += rb;
    r.tail = reinterpret_cast<float4*>(p); p += rb;
    r.pre = reinterpret_cast<float4*>(p); p += rb;
    r.suf = reinterpret_cast<float4*>(p);
    return r;
  }
  __host__ __device__ static size_t bytes(int64_t n_tiles) { return kRecBytesPerTile * rec_stride(n_tiles); }

  __device__ Part get(const float4* a, int64_t t) const {
    const float4 u = a[kPartVecs * t], v = a[kPartVecs * t + 1], w = a[kPartVecs * t + 2];
    Part p;
    Range& r = p.r;
    r.tau = u.x; r.cr = u.y; r.cg = u.z; r.cb = u.w;
    r.A = v.x; r.F = v.y; r.B = v.z; r.L = v.w;
    r.m0 = w.x; r.m1 = w.y; p.tlo = w.z;
    return p;
  }
  __device__ void put(float4* a, int64_t t, const Part& p) const {
    const Range& r = p.r;
    a[kPartVecs * t] = make_float4(r.tau, r.cr, r.cg, r.cb);
    a[kPartVecs * t + 1] = make_float4(r.A, r.F, r.B, r.L);
    a[kPartVecs * t + 2] = make_float4(r.m0, r.m1, p.tlo, 0.f);
  }
  __device__ void put(float4* a, int64_t t, const Range& r) const { put(a, t, part_of(r)); }
};

}  // namespace xl
